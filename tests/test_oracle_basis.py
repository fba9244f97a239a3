"""Pins for oracle.basis: nodal property, partition of unity, textbook P1."""
import numpy as np
import pytest

from oracle.basis import eval_basis, node_coords, nodes


@pytest.mark.parametrize("p", [1, 2, 3])
def test_sizes(p):
    # (p+3)!/(3! p!) DoFs per simplex (Sec. 2.3, paragraph before eq. (8))
    assert nodes(p).shape[0] == {1: 4, 2: 10, 3: 20}[p]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_nodal(p):
    v, _ = eval_basis(p, node_coords(p))
    assert np.allclose(v, np.eye(v.shape[0]), atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_partition_of_unity(p):
    x = np.random.default_rng(0).dirichlet(np.ones(4), size=50)[:, 1:]
    v, g = eval_basis(p, x)
    assert np.allclose(v.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(g.sum(axis=2), 0.0, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reproduces_polynomials(p):
    """sum_j q(x_j) phi_j = q for every monomial q of degree <= p; gradients too."""
    rng = np.random.default_rng(1)
    x = rng.dirichlet(np.ones(4), size=20)[:, 1:]
    v, g = eval_basis(p, x)
    xn = node_coords(p)
    for a in range(p + 1):
        for b in range(p + 1 - a):
            for c in range(p + 1 - a - b):
                qn = xn[:, 0] ** a * xn[:, 1] ** b * xn[:, 2] ** c
                q = x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
                assert np.allclose(v @ qn, q, atol=1e-13)
                if a:
                    dq = a * x[:, 0] ** (a - 1) * x[:, 1] ** b * x[:, 2] ** c
                    assert np.allclose(g[:, 0, :] @ qn, dq, atol=1e-12)


def test_p1_is_barycentric():
    x = np.array([[0.1, 0.2, 0.3]])
    v, g = eval_basis(1, x)
    # lexicographic multi-indices: (0,0,0,1), (0,0,1,0), (0,1,0,0), (1,0,0,0)
    assert np.allclose(v[0], [0.3, 0.2, 0.1, 0.4])
    assert np.allclose(g[0].T, [[0, 0, 1], [0, 1, 0], [1, 0, 0], [-1, -1, -1]])


def test_finite_difference_gradient():
    rng = np.random.default_rng(2)
    x = rng.dirichlet(np.ones(4), size=5)[:, 1:]
    h = 1e-6
    _, g = eval_basis(3, x)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        vp, _ = eval_basis(3, x + e)
        vm, _ = eval_basis(3, x - e)
        assert np.allclose((vp - vm) / (2 * h), g[:, k, :], atol=1e-7)
