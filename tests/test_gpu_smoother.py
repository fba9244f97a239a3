"""GPU parity of the Chebyshev-Jacobi smoother (Sec. 4.1) with the oracle's
recurrence on the assembled matrix, and of the Lanczos estimate of the
largest eigenvalue of D^-1 A with the exact generalised eigenvalue."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from tests.tetmf_cases import cg_map, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(n, p, qdeg, sigma, bc, precision):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(qdeg)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=sigma, dirichlet=(bc == "dirichlet"))
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), sigma=sigma, bc=bc, precision=precision)
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    return A, op, idx, kl


@pytest.mark.parametrize("p,qdeg,sigma,bc", [(2, 4, 0.3, "neumann"), (3, 6, 0.0, "dirichlet")])
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("zero_guess", [True, False])
def test_chebyshev_vs_oracle(p, qdeg, sigma, bc, precision, tol, zero_guess):
    A, op, idx, kl = _case(4, p, qdeg, sigma, bc, precision)
    dg = A.diagonal()
    lam = sla.eigh(A.toarray(), np.diag(dg), eigvals_only=True)
    lmax = 1.1 * lam[-1]
    lmin = lmax / 8.0
    rng = np.random.default_rng(11)
    b = rng.uniform(-1, 1, A.shape[0])
    x0 = None if zero_guess else rng.uniform(-1, 1, A.shape[0])
    if precision != "f64":  # both sides see the rounded inputs
        b = b.astype(np.float32).astype(np.float64)
        x0 = None if x0 is None else x0.astype(np.float32).astype(np.float64)
    x_ref = oracle.chebyshev(A, 1.0 / dg, b, x0, 5, lmin, lmax)
    dev = torch.device("cuda", 0)
    inv = 1.0 / op.diagonal(kl)
    bt = torch.from_numpy(b[idx]).to(dev, op.dtype)
    xt = None if x0 is None else torch.from_numpy(x0[idx]).to(dev, op.dtype)
    x = op.chebyshev(bt, inv, 5, lmin, lmax, x=xt, kappa=kl).double().cpu().numpy()
    assert rel_err(x, x_ref[idx]) <= tol


@pytest.mark.parametrize("p,qdeg,sigma,bc", [(2, 4, 0.3, "neumann"), (3, 6, 0.0, "dirichlet")])
def test_lambda_max_estimate(p, qdeg, sigma, bc):
    A, op, idx, kl = _case(4, p, qdeg, sigma, bc, "f64")
    dg = A.diagonal()
    lam = sla.eigh(A.toarray(), np.diag(dg), eigvals_only=True)
    inv = 1.0 / op.diagonal(kl)
    est = op.estimate_lambda_max(inv, n_iter=30, kappa=kl)
    print(f"P{p} {bc}: lambda_max(D^-1 A) = {lam[-1]:.6f}, Lanczos estimate (30 steps) {est:.6f}")
    # a Ritz value: below the true maximum (up to rounding), and close to it
    assert est <= lam[-1] * (1 + 1e-9)
    assert est >= 0.97 * lam[-1]
