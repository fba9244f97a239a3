"""Pins of the oracle's curved-cell path (a Jacobian per quadrature point,
Sec. 3.2) against closed forms of the synthetic map
Phi(x, y, z) = (x + e y^2, y + e z^2, z + e x^2) on the unit cube:

* det grad Phi = 1 + 8 e^3 x y z, so the deformed volume is 1 + e^3, and the
  integrand |det J_q| is a cubic in the reference coordinates (exact for
  rules of degree >= 3);
* the physical coordinate field a . x = a . Phi(X) is quadratic in the
  reference coordinates of every cell, so it lies in the P2 and P3 spaces
  exactly, with gradient a in physical space: its energy u^T K u is
  |a|^2 (1 + e^3), and K applied to a constant is zero;
* 1^T M 1 = 1 + e^3 for the mass part and the load vector of f = 1;
* with the affine Jacobian at every point the curved path equals the
  straight-sided one.
A transposed Jacobian, the affine determinant in place of the per-point one,
or a wrong point index changes the first three values."""
import numpy as np
import pytest

import oracle
import synth

EPS = 0.25


def curved_case(n, p, qdeg, seed=0):
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, seed)
    qp, qw = synth.tet_rule(qdeg)
    jac = synth.curved_jacobians(xyz, tets, qp, EPS)
    return xyz, tets, qp, qw, jac


@pytest.mark.parametrize("p,qdeg", [(2, 4), (3, 6), (3, 4)])
def test_curved_energy_of_coordinate_field(p, qdeg):
    xyz, tets, qp, qw, jac = curved_case(3, p, qdeg)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, jac=jac)
    a = np.array([0.3, -1.2, 0.7])
    u = synth.curved_map(d["xyz"], EPS) @ a
    assert abs(u @ (A @ u) - (a @ a) * (1 + EPS ** 3)) <= 1e-12 * (a @ a)
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_curved_volume_mass_and_load(p):
    xyz, tets, qp, qw, jac = curved_case(3, p, 4)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, sigma=1.0, jac=jac)
    K, _ = oracle.assemble_cg(xyz, tets, p, qp, qw, jac=jac, dofs=d)
    one = np.ones(A.shape[0])
    assert abs(one @ ((A - K) @ one) - (1 + EPS ** 3)) <= 1e-12
    b = oracle.load_vector(xyz, tets, p, qp, qw, dofs=d, jac=jac)
    assert abs(b.sum() - (1 + EPS ** 3)) <= 1e-12


def test_curved_with_affine_jacobians_is_straight():
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 1)
    qp, qw = synth.tet_rule(6)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.0)
    kap = synth.lognormal(1, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size))
    A0, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=kap, sigma=0.5)
    A1, _ = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=kap, sigma=0.5, dofs=d, jac=jac)
    assert abs(A0 - A1).max() <= 1e-13 * abs(A0).max()


def test_curved_kappa_gradient_is_the_form_derivative():
    """dkappa_{e,q} from cg_kappa_grad equals g^T A(indicator of (e, q)) u for
    sampled (e, q) with curved cells."""
    xyz, tets, qp, qw, jac = curved_case(2, 2, 4, seed=2)
    A, d = oracle.assemble_cg(xyz, tets, 2, qp, qw, jac=jac)
    u = synth.uniform(2, synth.STREAM_U, A.shape[0])
    g = synth.uniform(2, synth.STREAM_F, A.shape[0])
    dk = oracle.cg_kappa_grad(xyz, tets, 2, qp, qw, u, g, dofs=d, jac=jac)
    rng = np.random.default_rng(0)
    for e, q in zip(rng.integers(0, tets.shape[0], 4), rng.integers(0, qw.size, 4)):
        ind = np.zeros((tets.shape[0], qw.size))
        ind[e, q] = 1.0
        Ai, _ = oracle.assemble_cg(xyz, tets, 2, qp, qw, kappa=ind, dofs=d, jac=jac)
        assert abs(g @ (Ai @ u) - dk[e, q]) <= 1e-13 * max(1.0, abs(dk[e, q]))
