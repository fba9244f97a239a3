"""GPU parity of the vector-valued (components-batched, Sec. 3.2) CG
operator against the oracle's block-diagonal operator: three components
without coupling, vectors stored component by component.  Bars as for the
scalar operator: relative 2-norm error <= 1e-12 (FP64), <= 1e-5 (FP32)."""
import numpy as np
import pytest

import oracle
import synth
from tests.tetmf_cases import cg_map, rel_err, row_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def setup_vec(n, p, qdeg, mass=0.0, bc="neumann", precision="f64", curved=False, kappa=True, seed=0):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, seed)
    qp, qw = synth.tet_rule(qdeg)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25) if curved else None
    kap = synth.lognormal(seed, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5) if kappa else None
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=mass, dirichlet=(bc == "dirichlet"), jac=jac)
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), precision=precision, bc=bc, sigma=mass, q_jacobians=jac,
                     n_components=3)
    assert op.n_components == 3 and op.n_vec == 3 * A.shape[0]
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    idx3 = np.concatenate([c * A.shape[0] + idx for c in range(3)])
    dev = torch.device("cuda", 0)
    kl = None if kap is None else op.cell_data_to_library(torch.from_numpy(kap).to(dev))
    return dict(A=A, Av=oracle.vector_operator(A, 3), d=d, op=op, idx3=idx3, kl=kl, dev=dev, xyz=xyz, tets=tets,
                qp=qp, qw=qw, jac=jac)


@pytest.mark.parametrize("p,qdeg,n", [(1, 2, 5), (2, 4, 5), (3, 6, 4), (3, 4, 4)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_vector_apply(p, qdeg, n, precision):
    c = setup_vec(n, p, qdeg, precision=precision)
    u = synth.uniform(0, synth.STREAM_U, c["Av"].shape[0])
    ut = torch.from_numpy(u[c["idx3"]]).to(c["dev"], c["op"].dtype)
    v = c["op"].apply(ut, c["kl"]).double().cpu().numpy()
    assert rel_err(v, (c["Av"] @ u)[c["idx3"]]) <= TOL[precision]
    assert row_err(v, c["Av"], u, c["idx3"]) <= TOL[precision]


@pytest.mark.parametrize("curved", [False, True])
def test_vector_helmholtz_dirichlet(curved):
    c = setup_vec(4, 3, 6, mass=1.0, bc="dirichlet", curved=curved)
    u = synth.uniform(1, synth.STREAM_U, c["Av"].shape[0])
    v = c["op"].apply(torch.from_numpy(u[c["idx3"]]).to(c["dev"]), c["kl"]).cpu().numpy()
    assert rel_err(v, (c["Av"] @ u)[c["idx3"]]) <= 1e-12
    assert row_err(v, c["Av"], u, c["idx3"]) <= 1e-12


def test_vector_coordinate_field_energy():
    """u = (x, y, z): u^T A u = 3 |Omega| = 3 with kappa = 1 (closed form)."""
    c = setup_vec(4, 2, 4, kappa=False)
    u = np.concatenate([c["d"]["xyz"][:, k] for k in range(3)])
    ut = torch.from_numpy(u[c["idx3"]]).to(c["dev"])
    assert abs(torch.dot(ut, c["op"].apply(ut)).item() - 3.0) <= 1e-12


def test_vector_components_are_independent():
    """A component's result does not depend on the other components."""
    c = setup_vec(4, 3, 6)
    n = c["A"].shape[0]
    u = torch.from_numpy(synth.uniform(3, synth.STREAM_U, 3 * n)).to(c["dev"])
    v = c["op"].apply(u, c["kl"])
    u2 = u.clone()
    u2[:n] = 0.0
    u2[2 * n:] = 0.0
    v2 = c["op"].apply(u2, c["kl"])
    assert torch.equal(v2[n:2 * n], v[n:2 * n])
    assert torch.count_nonzero(v2[:n]) == 0 and torch.count_nonzero(v2[2 * n:]) == 0


@pytest.mark.parametrize("p,qdeg,precision,curved", [
    (2, 4, "f64", False), (3, 6, "f64", False), (3, 6, "f32", False), (3, 6, "f64", True), (2, 4, "f32", True),
])
def test_vector_backward_and_diagonal(p, qdeg, precision, curved):
    c = setup_vec(4, p, qdeg, mass=0.5, bc="dirichlet", precision=precision, curved=curved)
    tol = TOL[precision]
    n = c["A"].shape[0]
    u = synth.uniform(2, synth.STREAM_U, 3 * n)
    g = synth.uniform(2, synth.STREAM_F, 3 * n)
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    dt = c["op"].dtype
    ut = torch.from_numpy(u[c["idx3"]]).to(c["dev"], dt)
    gt = torch.from_numpy(g[c["idx3"]]).to(c["dev"], dt)
    du, dk = c["op"].backward(ut, gt, c["kl"])
    assert rel_err(du.double().cpu().numpy(), (c["Av"].T @ g)[c["idx3"]]) <= tol
    # constrained DoFs enter neither side's gradient: the oracle's form uses
    # the Dirichlet-masked vectors
    free = ~c["d"]["constrained"]
    mask = np.concatenate([free] * 3).astype(np.float64)
    dko = oracle.vector_kappa_grad(
        lambda a, b: oracle.cg_kappa_grad(c["xyz"], c["tets"], p, c["qp"], c["qw"], a, b, dofs=c["d"],
                                          jac=c["jac"]),
        u * mask, g * mask, 3, n)
    assert rel_err(c["op"].cell_data_to_user(dk).double().cpu().numpy(), dko) <= tol
    dg = c["op"].diagonal(c["kl"]).double().cpu().numpy()
    assert rel_err(dg, np.concatenate([c["A"].diagonal()] * 3)[c["idx3"]]) <= tol


@pytest.mark.parametrize("method", [None, "reliable"])
def test_vector_solve(method):
    """Jacobi-PCG on the vector Helmholtz operator (the velocity step of
    Sec. 4.2) reaches the oracle's direct solution: plain FP64, and with an
    FP32 three-component inner operator by reliable updates."""
    import scipy.sparse.linalg as spla
    import paper_2509_10226_amd as tm
    c = setup_vec(4, 2, 4, mass=1.0, bc="dirichlet")
    Av = c["Av"].tocsc()
    free = np.concatenate([~c["d"]["constrained"]] * 3)
    b = np.where(free, synth.uniform(3, synth.STREAM_F, Av.shape[0]), 0.0)
    x_ref = spla.spsolve(Av, b)
    bt = torch.from_numpy(b[c["idx3"]]).to(c["dev"])
    kw = {}
    if method is not None:
        op32 = tm.Operator(tm.Mesh(c["xyz"], c["tets"]), 2, (c["qp"], c["qw"]), precision="f32", bc="dirichlet",
                           sigma=1.0, n_components=3)
        kw = dict(inner=op32, kappa_inner=c["kl"].float(), method=method, inner_rtol=1e-2)
    x, stats, ok = c["op"].solve(bt, kappa=c["kl"], rtol=1e-10, **kw)
    assert ok, stats
    assert stats["final_relres"] <= 1e-10
    assert rel_err(x.cpu().numpy(), x_ref[c["idx3"]]) <= 1e-8


def test_vector_load_vector_unsupported():
    import paper_2509_10226_amd as tm
    c = setup_vec(2, 1, 2)
    with pytest.raises(tm.TetmfError):
        c["op"].load_vector()


def test_vector_solve_rejects_mismatched_inner_operator():
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(4)
    mesh = tm.Mesh(xyz, tets)
    opv = tm.Operator(mesh, 2, (qp, qw), bc="dirichlet", n_components=3)
    ops32 = tm.Operator(mesh, 2, (qp, qw), bc="dirichlet", precision="f32")
    b = torch.zeros(opv.n_vec, dtype=torch.float64, device="cuda")
    with pytest.raises(tm.TetmfError) as e:
        opv.solve(b, inner=ops32)
    assert e.value.status == -1


def test_vector_autograd():
    """torch.autograd through apply_autograd on a vector field returns the
    kernel gradients (the kappa gradient summed over the components)."""
    import paper_2509_10226_amd as tm
    c = setup_vec(3, 2, 4)
    n = c["op"].n_vec
    ut = torch.from_numpy(synth.uniform(6, synth.STREAM_U, n)).cuda().requires_grad_()
    gt = torch.from_numpy(synth.uniform(6, synth.STREAM_F, n)).cuda()
    kc = c["kl"].clone().requires_grad_()
    (tm.apply_autograd(c["op"], ut, kc) * gt).sum().backward()
    du, dk = c["op"].backward(ut.detach(), gt, c["kl"])
    assert torch.equal(ut.grad, du) and torch.equal(kc.grad, dk)


@pytest.mark.parametrize("curved", [False, True])
def test_vector_equals_scalar_per_component(curved):
    """Each component of the vector apply and of the Chebyshev smoother (no
    inner products) is bitwise the scalar operator's result on that
    component: the same kernel arithmetic runs per component."""
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(5, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25) if curved else None
    mesh = tm.Mesh(xyz, tets)
    opv = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", sigma=0.5, q_jacobians=jac, n_components=3)
    ops = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", sigma=0.5, q_jacobians=jac)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    kl = ops.cell_data_to_library(torch.from_numpy(kap).cuda())
    n = ops.n_dofs
    u = torch.from_numpy(synth.uniform(7, synth.STREAM_U, 3 * n)).cuda()
    v = opv.apply(u, kl)
    for c in range(3):
        assert torch.equal(v[c * n:(c + 1) * n], ops.apply(u[c * n:(c + 1) * n].contiguous(), kl))
    dv, ds = opv.diagonal(kl), ops.diagonal(kl)
    assert all(torch.equal(dv[c * n:(c + 1) * n], ds) for c in range(3))
    inv = 1.0 / dv
    lam_v = opv.estimate_lambda_max(inv, kappa=kl)
    lam_s = ops.estimate_lambda_max(1.0 / ds, kappa=kl)
    assert abs(lam_v - lam_s) <= 0.05 * lam_s
    xv = opv.chebyshev(u, inv, 4, lam_s / 15, 1.1 * lam_s, kappa=kl)
    for c in range(3):
        xs = ops.chebyshev(u[c * n:(c + 1) * n].contiguous(), 1.0 / ds, 4, lam_s / 15, 1.1 * lam_s, kappa=kl)
        assert torch.equal(xv[c * n:(c + 1) * n], xs)
