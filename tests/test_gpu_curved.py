"""GPU parity of the continuous-Galerkin operator on curved cells (a
Jacobian per rule point, Sec. 3.2) against the oracle, on the synthetic
smooth map of ``synth.curved_jacobians`` (the oracle's curved path is pinned
to closed forms in test_oracle_curved.py).  Bars as for straight cells:
relative 2-norm error <= 1e-12 (FP64), <= 1e-5 (FP32)."""
import numpy as np
import pytest

import oracle
import synth
from tests.tetmf_cases import cg_map, rel_err, row_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
EPS = 0.25


def setup_curved(n, p, qdeg, mass=0.0, bc="neumann", precision="f64", kappa=True, seed=0):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, seed)
    qp, qw = synth.tet_rule(qdeg)
    jac = synth.curved_jacobians(xyz, tets, qp, EPS)
    kap = synth.lognormal(seed, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5) if kappa else None
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=mass, dirichlet=(bc == "dirichlet"), jac=jac)
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), precision=precision, bc=bc, sigma=mass, q_jacobians=jac)
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    dev = torch.device("cuda", 0)
    kl = None if kap is None else op.cell_data_to_library(torch.from_numpy(kap).to(dev))
    return dict(A=A, d=d, op=op, idx=idx, kl=kl, dev=dev, xyz=xyz, tets=tets, qp=qp, qw=qw, jac=jac)


@pytest.mark.parametrize("p,qdeg,n", [(1, 2, 5), (2, 4, 5), (3, 6, 4), (3, 4, 4)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_curved_apply(p, qdeg, n, precision):
    c = setup_curved(n, p, qdeg, precision=precision)
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"], c["op"].dtype)
    v = c["op"].apply(ut, c["kl"]).double().cpu().numpy()
    assert rel_err(v, (c["A"] @ u)[c["idx"]]) <= TOL[precision]
    assert row_err(v, c["A"], u, c["idx"]) <= TOL[precision]


@pytest.mark.parametrize("p,qdeg,mass", [(1, 2, 0.0), (2, 4, 1000.0), (3, 6, 0.0), (3, 6, 3000.0)])
def test_curved_apply_bf16_operands(p, qdeg, mass):
    """BF16 operands (FP32 geometry, coefficient and accumulation) on curved
    cells: the error against the FP64 oracle is printed; the 3e-2 bound
    guards against layout mistakes, which give O(1) errors.  The Helmholtz
    cases take a mass coefficient large enough for the mass term to be a
    sizeable part of the result."""
    c = setup_curved(4, p, qdeg, mass=mass, precision="bf16in")
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0]).astype(np.float32).astype(np.float64)
    if mass > 0:
        kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (c["tets"].shape[0], c["qw"].size), sigma=0.5)
        K, _ = oracle.assemble_cg(c["xyz"], c["tets"], p, c["qp"], c["qw"], kappa=kap, jac=c["jac"])
        y = c["A"] @ u
        assert np.linalg.norm(y - K @ u) > 0.2 * np.linalg.norm(y)
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"], c["op"].dtype)
    v = c["op"].apply(ut, c["kl"]).double().cpu().numpy()
    err = rel_err(v, (c["A"] @ u)[c["idx"]])
    print(f"BF16-operand curved apply, P{p} degree-{qdeg} rule, sigma={mass}: relative error {err:.3e}")
    assert err <= 3e-2


@pytest.mark.parametrize("p,qdeg", [(2, 4), (3, 6)])
def test_curved_helmholtz_dirichlet(p, qdeg):
    c = setup_curved(4, p, qdeg, mass=1.0, bc="dirichlet")
    u = synth.uniform(1, synth.STREAM_U, c["A"].shape[0])
    v = c["op"].apply(torch.from_numpy(u[c["idx"]]).to(c["dev"]), c["kl"]).cpu().numpy()
    assert rel_err(v, (c["A"] @ u)[c["idx"]]) <= 1e-12
    assert row_err(v, c["A"], u, c["idx"]) <= 1e-12


def test_curved_coordinate_field_energy():
    """u = a . Phi(X) lies in the P3 space; u^T A u = |a|^2 (1 + e^3) with
    kappa = 1 (closed form, independent of the oracle)."""
    c = setup_curved(4, 3, 6, kappa=False)
    a = np.array([0.3, -1.2, 0.7])
    u = synth.curved_map(c["d"]["xyz"], EPS) @ a
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"])
    e = torch.dot(ut, c["op"].apply(ut)).item()
    assert abs(e - (a @ a) * (1 + EPS ** 3)) <= 1e-12 * (a @ a)


@pytest.mark.parametrize("mass", [0.0, 1.0])
def test_curved_diagonal_and_load_vector(mass):
    c = setup_curved(4, 3, 6, mass=mass, bc="dirichlet")
    dg = c["op"].diagonal(c["kl"]).cpu().numpy()
    assert rel_err(dg, c["A"].diagonal()[c["idx"]]) <= 1e-12
    f = synth.lognormal(0, synth.STREAM_F, (c["tets"].shape[0], c["qw"].size), sigma=0.5)
    b = c["op"].load_vector(c["op"].cell_data_to_library(torch.from_numpy(f).to(c["dev"]))).cpu().numpy()
    bo = oracle.load_vector(c["xyz"], c["tets"], 3, c["qp"], c["qw"], f=f, dirichlet=True, dofs=c["d"],
                            jac=c["jac"])
    assert rel_err(b, bo[c["idx"]]) <= 1e-12


@pytest.mark.parametrize("p,qdeg,mass,precision", [
    (2, 4, 0.5, "f64"), (1, 2, 0.0, "f64"), (3, 6, 0.0, "f64"), (3, 6, 0.5, "f64"),
    (2, 4, 0.5, "f32"), (3, 6, 0.0, "f32"), (3, 6, 0.5, "f32"),
])
def test_curved_backward(p, qdeg, mass, precision):
    """du = A^T g and the per-point coefficient gradient on curved cells,
    every degree, Poisson and Helmholtz forms, FP64 and FP32."""
    c = setup_curved(4, p, qdeg, mass=mass, precision=precision)
    n = c["A"].shape[0]
    u = synth.uniform(2, synth.STREAM_U, n)
    g = synth.uniform(2, synth.STREAM_F, n)
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    dt = c["op"].dtype
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"], dt)
    gt = torch.from_numpy(g[c["idx"]]).to(c["dev"], dt)
    du, dk = c["op"].backward(ut, gt, c["kl"])
    du = du.double().cpu().numpy()
    assert rel_err(du, (c["A"].T @ g)[c["idx"]]) <= TOL[precision]
    assert row_err(du, c["A"].T.tocsr(), g, c["idx"]) <= TOL[precision]
    dko = oracle.cg_kappa_grad(c["xyz"], c["tets"], p, c["qp"], c["qw"], u, g, dofs=c["d"], jac=c["jac"])
    assert rel_err(c["op"].cell_data_to_user(dk).double().cpu().numpy(), dko) <= TOL[precision]


@pytest.mark.parametrize("method", [None, "refinement", "reliable"])
def test_curved_solve(method):
    """Jacobi-PCG on the curved Helmholtz operator reaches the oracle's
    direct solution: plain FP64, and with an FP32 curved inner operator
    (same Jacobians and coefficient) by both mixed-precision methods."""
    import scipy.sparse.linalg as spla
    import paper_2509_10226_amd as tm
    c = setup_curved(4, 2, 4, mass=1.0, bc="dirichlet")
    A = c["A"].tocsc()
    free = ~c["d"]["constrained"]
    b = np.where(free, synth.uniform(3, synth.STREAM_F, A.shape[0]), 0.0)
    x_ref = spla.spsolve(A, b)
    bt = torch.from_numpy(b[c["idx"]]).to(c["dev"])
    kw = {}
    if method is not None:
        op32 = tm.Operator(tm.Mesh(c["xyz"], c["tets"]), 2, (c["qp"], c["qw"]), precision="f32", bc="dirichlet",
                           sigma=1.0, q_jacobians=c["jac"])
        kw = dict(inner=op32, kappa_inner=c["kl"].float(), method=method, inner_rtol=1e-2)
    x, stats, ok = c["op"].solve(bt, kappa=c["kl"], rtol=1e-10, **kw)
    assert ok, stats
    assert stats["final_relres"] <= 1e-10
    assert rel_err(x.cpu().numpy(), x_ref[c["idx"]]) <= 1e-8
