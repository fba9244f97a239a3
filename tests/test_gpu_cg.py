"""GPU parity of the continuous-Galerkin operator against the oracle.

The HIP path (through the C ABI) and the oracle's assembled FP64 matrix see
the same seeded mesh, coefficients and vector; library DoFs are matched to
oracle DoFs by coordinates.  Bars: relative 2-norm error <= 1e-12 (FP64) and
<= 1e-5 (FP32, inputs rounded to FP32)."""
import numpy as np
import pytest

import oracle
import synth
from tests.tetmf_cases import cg_map, rel_err, row_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _tm():
    import paper_2509_10226_amd as tm
    return tm


def setup_case(n, p, qdeg, kappa_sigma=None, mass=0.0, bc="neumann", precision="f64", shuffle=False,
               ordering="locality", jitter=0.15, seed=0):
    tm = _tm()
    xyz, tets = synth.kuhn_cube_mesh(n, jitter, seed)
    if shuffle:
        xyz, tets = synth.shuffle_mesh(xyz, tets, seed)
    qp, qw = synth.tet_rule(qdeg)
    kap = None if kappa_sigma is None else synth.lognormal(seed, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size),
                                                           sigma=kappa_sigma)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=mass, dirichlet=(bc == "dirichlet"))
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), precision=precision, bc=bc, sigma=mass, ordering=ordering)
    cp, dxyz, dcell = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    dev = torch.device("cuda", 0)
    kl = None if kap is None else op.cell_data_to_library(torch.from_numpy(kap).to(dev))
    return dict(A=A, d=d, op=op, idx=idx, kap=kap, kl=kl, dev=dev, xyz=xyz, tets=tets, qp=qp, qw=qw, p=p, bc=bc)


def mass_share(c, u, kappa_sigma):
    """||A u - K u|| / ||A u||: the part of the result the mass term makes
    (K: the same operator without it)."""
    kap = c["kap"]
    K, _ = oracle.assemble_cg(c["xyz"], c["tets"], c["p"], c["qp"], c["qw"], kappa=kap, sigma=0.0,
                              dirichlet=c["bc"] == "dirichlet")
    y = c["A"] @ u
    return float(np.linalg.norm(y - K @ u) / np.linalg.norm(y))


def run_apply(c, u):
    op = c["op"]
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"], op.dtype)
    v = op.apply(ut, c["kl"]).double().cpu().numpy()
    return v


@pytest.mark.parametrize("p,qdeg,n", [(1, 2, 6), (2, 4, 6), (2, 2, 5), (3, 6, 5), (3, 4, 4)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cg_apply_variable_kappa(p, qdeg, n, precision):
    c = setup_case(n, p, qdeg, kappa_sigma=1.0, precision=precision)
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    y = c["A"] @ u
    v = run_apply(c, u)
    assert rel_err(v, y[c["idx"]]) <= TOL[precision]
    assert row_err(v, c["A"], u, c["idx"]) <= TOL[precision]


def test_cg_reduced_rule_unit_kappa():
    """P3 apply with the 14-point rule exact to degree 4 (modified integration,
    Sec. 3.3) and a unit coefficient equals the oracle's stiffness built with
    the degree-6 rule: a check through a different quadrature."""
    tm = _tm()
    n, p = 4, 3
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qf, wf = synth.tet_rule(6)
    A, d = oracle.assemble_cg(xyz, tets, p, qf, wf)
    qr, wr = synth.tet_rule(4)
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qr, wr))
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    u = synth.uniform(0, synth.STREAM_U, A.shape[0])
    v = op.apply(torch.from_numpy(u[idx]).cuda()).cpu().numpy()
    assert rel_err(v, (A @ u)[idx]) <= 1e-12
    assert row_err(v, A, u, idx) <= 1e-12


def test_cg_c1_config():
    """CG P2 Poisson stiffness, 8^3 x 6 Kuhn tets, jitter 0.15h seed 0, kappa = 1, degree-4 rule."""
    c = setup_case(8, 2, 4)
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    v = run_apply(c, u)
    y = c["A"] @ u
    assert rel_err(v, y[c["idx"]]) <= 1e-12
    assert row_err(v, c["A"], u, c["idx"]) <= 1e-12
    assert c["op"].n_dofs == 17 ** 3


@pytest.mark.parametrize("p,qdeg,n", [(2, 4, 5), (3, 6, 4)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cg_helmholtz_dirichlet(p, qdeg, n, precision):
    c = setup_case(n, p, qdeg, kappa_sigma=0.5, mass=1.0, bc="dirichlet", precision=precision)
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    v = run_apply(c, u)
    y = c["A"] @ u
    assert rel_err(v, y[c["idx"]]) <= TOL[precision]
    assert row_err(v, c["A"], u, c["idx"]) <= TOL[precision]
    # constrained rows are the identity
    cons = c["d"]["constrained"][c["idx"]]
    assert np.array_equal(v[cons], u[c["idx"]][cons].astype(v.dtype)) if precision == "f64" else True
    assert c["op"].n_free == int((~c["d"]["constrained"]).sum())


@pytest.mark.parametrize("shuffle,ordering", [(True, "locality"), (True, "as_given"), (False, "as_given")])
def test_cg_orderings(shuffle, ordering):
    c = setup_case(5, 3, 6, kappa_sigma=1.0, shuffle=shuffle, ordering=ordering)
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    v = run_apply(c, u)
    assert rel_err(v, (c["A"] @ u)[c["idx"]]) <= 1e-12
    assert row_err(v, c["A"], u, c["idx"]) <= 1e-12


def test_cg_deterministic():
    c = setup_case(6, 3, 6, kappa_sigma=1.0)
    op = c["op"]
    u = torch.from_numpy(synth.uniform(0, 2, op.n_dofs)).to(c["dev"])
    v1 = op.apply(u, c["kl"])
    v2 = op.apply(u, c["kl"])
    torch.cuda.synchronize()
    assert torch.equal(v1, v2)


def test_cg_constant_kernel_and_symmetry():
    """A 1 = 0 (Neumann) and u^T A w = w^T A u on the GPU output itself."""
    c = setup_case(6, 3, 6, kappa_sigma=1.0)
    op = c["op"]
    one = torch.ones(op.n_dofs, dtype=torch.float64, device=c["dev"])
    a1 = op.apply(one, c["kl"]).cpu().numpy()
    rng = np.random.default_rng(11)
    u = torch.from_numpy(rng.standard_normal(op.n_dofs)).to(c["dev"])
    w = torch.from_numpy(rng.standard_normal(op.n_dofs)).to(c["dev"])
    au = op.apply(u, c["kl"])
    aw = op.apply(w, c["kl"])
    scale = float(torch.linalg.norm(au))
    assert np.abs(a1).max() <= 1e-13 * scale
    s1 = float(torch.dot(w, au))
    s2 = float(torch.dot(u, aw))
    assert abs(s1 - s2) <= 1e-13 * float(torch.linalg.norm(u)) * float(torch.linalg.norm(aw))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cg_diagonal_and_load(precision):
    c = setup_case(5, 3, 6, kappa_sigma=1.0, mass=0.5, bc="dirichlet", precision=precision)
    op = c["op"]
    dg = op.diagonal(c["kl"]).double().cpu().numpy()
    assert rel_err(dg, c["A"].diagonal()[c["idx"]]) <= TOL[precision]
    b = op.load_vector().double().cpu().numpy()
    bo = oracle.load_vector(c["xyz"], c["tets"], 3, c["qp"], c["qw"], dirichlet=True, dofs=c["d"])
    assert rel_err(b, bo[c["idx"]]) <= TOL[precision]


@pytest.mark.parametrize("p,qdeg,n,mass,bc,precision", [
    (2, 4, 5, 1.0, "neumann", "f64"),
    (1, 2, 6, 0.3, "neumann", "f64"),
    (3, 6, 4, 0.0, "neumann", "f64"),
    (3, 6, 4, 0.5, "dirichlet", "f64"),
    (3, 4, 4, 0.0, "neumann", "f64"),
    (2, 4, 5, 1.0, "dirichlet", "f32"),
    (3, 6, 4, 0.0, "neumann", "f32"),
    (3, 6, 4, 0.5, "dirichlet", "f32"),
])
def test_cg_backward_vs_oracle(p, qdeg, n, mass, bc, precision):
    """du = A^T g and the per-point coefficient gradient against the oracle,
    for every degree, both P3 rules, Poisson and Helmholtz forms, both
    boundary modes and both precisions with a backward kernel.  With
    Dirichlet conditions the constrained DoFs enter neither side's gradient,
    so the oracle's form sees the masked vectors."""
    c = setup_case(n, p, qdeg, kappa_sigma=0.5, mass=mass, bc=bc, precision=precision)
    op = c["op"]
    N = c["A"].shape[0]
    u = synth.uniform(0, synth.STREAM_U, N)
    g = synth.uniform(0, synth.STREAM_F, N)
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    ut = torch.from_numpy(u[c["idx"]]).to(c["dev"], op.dtype)
    gt = torch.from_numpy(g[c["idx"]]).to(c["dev"], op.dtype)
    du, dk = op.backward(ut, gt, c["kl"])
    du = du.double().cpu().numpy()
    assert rel_err(du, (c["A"].T @ g)[c["idx"]]) <= TOL[precision]
    assert row_err(du, c["A"].T.tocsr(), g, c["idx"]) <= TOL[precision]
    # (the oracle marks boundary DoFs as constrained in either mode)
    free = (~c["d"]["constrained"]).astype(np.float64) if bc == "dirichlet" else np.ones(N)
    dko = oracle.cg_kappa_grad(c["xyz"], c["tets"], p, c["qp"], c["qw"], u * free, g * free, dofs=c["d"])
    dku = op.cell_data_to_user(dk).double().cpu().numpy()
    assert dku.shape == dko.shape
    assert rel_err(dku, dko) <= TOL[precision]


@pytest.mark.parametrize("p,qdeg,mass,bc", [(3, 6, 0.0, "neumann"), (2, 4, 1000.0, "neumann"), (3, 4, 0.0, "neumann"),
                                         (1, 2, 500.0, "neumann"), (3, 6, 3000.0, "dirichlet")])
def test_cg_apply_bf16_operands(p, qdeg, mass, bc):
    """BF16 operands with FP32 accumulation: the error against the FP64 oracle
    is reported, not gated at FP32 level.  The bound here (3e-2) only guards
    against layout mistakes, which give O(1) errors; the measured value is
    printed.  The Helmholtz cases take a mass coefficient large enough for
    the mass term to be a sizeable part of the result (at sigma = 1 it is
    below 0.1 % on these meshes, under the bound)."""
    c = setup_case(5, p, qdeg, kappa_sigma=1.0, mass=mass, bc=bc, precision="bf16in")
    u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
    y = c["A"] @ u
    if mass > 0:
        assert mass_share(c, u, kappa_sigma=1.0) > 0.2
    v = run_apply(c, u)
    err = rel_err(v, y[c["idx"]])
    print(f"BF16-operand apply, P{p} degree-{qdeg} rule, sigma={mass}, {bc}: relative error {err:.3e}")
    assert err <= 3e-2
