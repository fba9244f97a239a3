"""Pins of the oracle's Chebyshev-Jacobi smoother (Sec. 4.1) against the
closed form of its error polynomial: for a generalised eigenpair
A v = lam D v the smoother maps the error e = x* - x to p(lam) e with
p(t) = T_k((theta - t) / delta) / T_k(theta / delta), T_k the Chebyshev
polynomial of the first kind (numpy's chebval), independent of the
three-term recurrence the oracle runs."""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import chebyshev as npcheb

import oracle
import synth


def _p(t, k, lmin, lmax):
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    ck = np.zeros(k + 1)
    ck[k] = 1.0
    return npcheb.chebval((theta - t) / delta, ck) / npcheb.chebval(theta / delta, ck)


def _system(p, dirichlet):
    xyz, tets = synth.kuhn_cube_mesh(2, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    A, _ = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=0.3, dirichlet=dirichlet)
    A = A.toarray()
    return A, A.diagonal().copy()


@pytest.mark.parametrize("p,dirichlet", [(1, False), (2, True)])
@pytest.mark.parametrize("k", [1, 2, 5])
def test_eigenvector_damping(p, dirichlet, k):
    A, dg = _system(p, dirichlet)
    lam, V = sla.eigh(A, np.diag(dg))
    lmax = 1.1 * lam[-1]
    lmin = lmax / 8.0
    for j in (0, lam.size // 2, lam.size - 1):
        v = V[:, j]
        b = A @ v  # exact solution v; from x0 = 0 the error is v
        x = oracle.chebyshev(A, 1.0 / dg, b, None, k, lmin, lmax)
        expect = (1.0 - _p(lam[j], k, lmin, lmax)) * v
        assert np.abs(x - expect).max() <= 1e-10 * np.abs(v).max()


@pytest.mark.parametrize("k", [3, 5])
def test_error_polynomial_general_start(k):
    A, dg = _system(2, False)
    lam, V = sla.eigh(A, np.diag(dg))  # V^T A V = diag(lam), V^T D V = I
    lmax = 1.05 * lam[-1]
    lmin = lmax / 10.0
    rng = np.random.default_rng(7)
    xs = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    x = oracle.chebyshev(A, 1.0 / dg, A @ xs, x0, k, lmin, lmax)
    # error coefficients in the eigenbasis: c = V^T D (xs - x)
    c0 = V.T @ (dg * (xs - x0))
    c = V.T @ (dg * (xs - x))
    assert np.abs(c - _p(lam, k, lmin, lmax) * c0).max() <= 1e-9 * np.abs(c0).max()


def test_degree_one_is_damped_jacobi():
    A, dg = _system(1, False)
    rng = np.random.default_rng(1)
    b, x0 = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    lmin, lmax = 0.2, 2.0
    x = oracle.chebyshev(A, 1.0 / dg, b, x0, 1, lmin, lmax)
    omega = 2.0 / (lmin + lmax)
    assert np.abs(x - (x0 + omega * (b - A @ x0) / dg)).max() <= 1e-13 * np.abs(x).max()
