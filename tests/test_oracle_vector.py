"""Pins of the oracle's vector-valued (components-batched) operator: the
block-diagonal operator of a vector field without coupling between
components.

* the coordinate field u = (x, y, z), each component in the P1..P3 space,
  has u^T A u = sum_c int |grad x_c|^2 = 3 |Omega| = 3 on the unit cube
  (kappa = 1), and A applied to a constant vector field is zero;
* with a mass term sigma, 1^T (A - K) 1 over all components is 3 sigma;
* the kappa gradient of the vector form equals the derivative of
  g^T A(kappa) u with respect to an indicator coefficient.
A component placed in the wrong block or a missing block changes these."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("p,qdeg", [(1, 2), (2, 4), (3, 6)])
def test_vector_coordinate_field(p, qdeg):
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(qdeg)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw)
    Av = oracle.vector_operator(A, 3)
    u = np.concatenate([d["xyz"][:, c] for c in range(3)])
    assert abs(u @ (Av @ u) - 3.0) <= 1e-12
    assert np.max(np.abs(Av @ np.ones(3 * A.shape[0]))) <= 1e-12


def test_vector_mass():
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 1)
    qp, qw = synth.tet_rule(4)
    A, d = oracle.assemble_cg(xyz, tets, 2, qp, qw, sigma=2.0)
    K, _ = oracle.assemble_cg(xyz, tets, 2, qp, qw, dofs=d)
    one = np.ones(3 * A.shape[0])
    M = oracle.vector_operator(A, 3) - oracle.vector_operator(K, 3)
    assert abs(one @ (M @ one) - 3 * 2.0) <= 1e-12


def test_vector_kappa_gradient():
    xyz, tets = synth.kuhn_cube_mesh(2, 0.15, 2)
    qp, qw = synth.tet_rule(4)
    A, d = oracle.assemble_cg(xyz, tets, 2, qp, qw)
    n = A.shape[0]
    u = synth.uniform(2, synth.STREAM_U, 3 * n)
    g = synth.uniform(2, synth.STREAM_F, 3 * n)
    dk = oracle.vector_kappa_grad(lambda a, b: oracle.cg_kappa_grad(xyz, tets, 2, qp, qw, a, b, dofs=d), u, g, 3, n)
    rng = np.random.default_rng(1)
    for e, q in zip(rng.integers(0, tets.shape[0], 3), rng.integers(0, qw.size, 3)):
        ind = np.zeros((tets.shape[0], qw.size))
        ind[e, q] = 1.0
        Ai, _ = oracle.assemble_cg(xyz, tets, 2, qp, qw, kappa=ind, dofs=d)
        ref = g @ (oracle.vector_operator(Ai, 3) @ u)
        assert abs(ref - dk[e, q]) <= 1e-13 * max(1.0, abs(ref))
