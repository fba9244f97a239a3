"""Manufactured solution for the Dirichlet Poisson solve (Sec. 4.1 checks its
solver on a sine solution and states optimal convergence).

u = sin(pi x) sin(pi y) sin(pi z) on the unit cube vanishes on the boundary
and solves -Laplace u = 3 pi^2 u.  With f = 3 pi^2 u sampled at the cell
rule points, the oracle's stiffness matrix (Dirichlet rows as identity) and
load vector give a discrete solution whose L2 error decays like h^(p+1) for
nodal Lagrange elements of degree p.  The error is evaluated with the
degree-6 rule at points X0 + J x_q; the rate between two meshes is
log(e_coarse / e_fine) / log(N_fine / N_coarse).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth


def exact(x):
    return np.prod(np.sin(np.pi * np.asarray(x)), axis=-1)


def rule_points(xyz, tets, qpts):
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return X[:, None, 0, :] + np.einsum("eab,qb->eqa", J, qpts), np.abs(np.linalg.det(J))


def source(xyz, tets, qpts):
    """f = 3 pi^2 u at the cell rule points, [n_cell, n_q] (user layout)."""
    P, _ = rule_points(xyz, tets, qpts)
    return 3.0 * np.pi ** 2 * exact(P)


def l2_error(xyz, tets, p, x, dofmap):
    """||u_h - u||_L2 with u_h = sum_j x[dofmap[e, j]] phi_j on each cell."""
    q6, w6 = synth.tet_rule(6)
    P, adet = rule_points(xyz, tets, q6)
    phi, _ = oracle.eval_basis(p, q6)
    uh = np.einsum("qk,ek->eq", phi, x[dofmap])
    return float(np.sqrt(np.sum(w6[None, :] * adet[:, None] * (uh - exact(P)) ** 2)))


def oracle_solution(p, n):
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, dirichlet=True)
    b = oracle.load_vector(xyz, tets, p, qp, qw, f=source(xyz, tets, qp), dirichlet=True, dofs=d)
    x = spla.spsolve(A.tocsc(), b)
    return xyz, tets, d, x


@pytest.mark.parametrize("p,ns", [(1, (8, 16)), (2, (4, 8)), (3, (4, 8))])
def test_optimal_l2_rate(p, ns):
    errs = []
    for n in ns:
        xyz, tets, d, x = oracle_solution(p, n)
        assert np.all(x[d["constrained"]] == 0.0)
        errs.append(l2_error(xyz, tets, p, x, d["dofmap"]))
    rate = np.log(errs[0] / errs[1]) / np.log(ns[1] / ns[0])
    assert p + 1 - 0.25 <= rate <= p + 1 + 0.4, (p, errs, rate)


def test_interpolant_error_below_solution_error_bound():
    """The discrete solution's L2 error is within a small factor of the
    nodal interpolant's (quasi-optimality of the Galerkin solution)."""
    p, n = 2, 4
    xyz, tets, d, x = oracle_solution(p, n)
    e_sol = l2_error(xyz, tets, p, x, d["dofmap"])
    e_int = l2_error(xyz, tets, p, exact(d["xyz"]), d["dofmap"])
    assert e_sol < 3.0 * e_int
    assert e_int < 3.0 * e_sol
