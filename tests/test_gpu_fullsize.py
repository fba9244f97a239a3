"""Parity at the full workload sizes, in the launch configuration bench.py
times, on outputs the oracle can compute one by one:

* CG P3, 64^3 x 6 cells, lognormal(0, 1) coefficient: sampled rows of the
  FP64 / FP32 / BF16-operand apply against oracle rows (only the cells around
  each sampled DoF are assembled), and of the FP64 / FP32 apply on curved
  cells (the same mesh through a smooth map, a Jacobian per rule point);
  the 3-component vector field, straight and curved: each component bitwise
  equal to the scalar apply;
* SIPG P3, 32^3 x 6 cells, lognormal(0, 0.5) cell and face coefficients,
  Dirichlet mirror: the rows of sampled cells;
* CG P2 Helmholtz (stiffness + 1.0 mass), 48^3 x 6 cells: backward -- sampled
  rows of du = A g, sampled coefficient gradients against the oracle formula,
  and central finite differences (step 1e-6) on 64 coefficient entries of
  L = 1/2 ||A(kappa) u - f||^2, differenced row by row over the rows the
  entry touches (L is quadratic in each entry, so the difference quotient is
  exact up to rounding);
* CG P3 Dirichlet Poisson, f = 1, 64^3 x 6 cells: FP32-inner iterative
  refinement and plain FP64 PCG reach a true relative residual of 1e-10, the
  residual re-checked on sampled rows with the oracle.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from oracle.basis import node_coords

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def _tm():
    import paper_2509_10226_amd as tm
    return tm


def oracle_local_node(xyz, tets, cells, coords, p):
    """Lexicographic local node of each (user cell, coordinate) pair."""
    geo = oracle.Geometry(xyz, tets[cells])
    xn = node_coords(p)
    X = geo.X0[:, None, :] + np.einsum("eij,kj->eki", geo.J, xn)
    d = np.linalg.norm(X - coords[:, None, :], axis=2)
    j = np.argmin(d, axis=1)
    assert d[np.arange(j.size), j].max() < 1e-12
    return j


def key_coords(keys, xyz, p):
    return np.array([sum(m * xyz[v] for v, m in k) / p for k in keys])


def cg_row_values(xyz, tets, p, qp, qw, lib_rows, dof_xyz, dof_cell, u_lib, tree, kappa=None, sigma=0.0):
    """Oracle (A u)_i for sampled library DoFs i, with u given in library order."""
    cells = dof_cell[lib_rows]
    locs = oracle_local_node(xyz, tets, cells, dof_xyz[lib_rows], p)
    keys, rows = oracle.cg_rows(xyz, tets, p, qp, qw, cells, locs, kappa=kappa, sigma=sigma)
    vals, scales = [], []
    for rk, row in zip(keys, rows):
        ck = list(row.keys())
        cols = tree.query(key_coords(ck, xyz, p))[1]
        coef = np.array([row[c] for c in ck])
        vals.append(float(coef @ u_lib[cols]))
        scales.append(float(np.abs(coef) @ np.abs(u_lib[cols])))
    return np.array(vals), np.array(scales)


@pytest.fixture(scope="module")
def c3():
    tm = _tm()
    n, p = 64, 3
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=1.0)
    mesh = tm.Mesh(xyz, tets)
    return dict(tm=tm, xyz=xyz, tets=tets, qp=qp, qw=qw, kap=kap, mesh=mesh, p=p)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16in", 3e-2)])
def test_c3_sampled_rows(c3, precision, tol):
    tm = c3["tm"]
    op = tm.Operator(c3["mesh"], 3, (c3["qp"], c3["qw"]), precision=precision)
    assert op.n_dofs == 193 ** 3
    _, dof_xyz, dof_cell = op.numbering()
    kl = op.cell_data_to_library(torch.from_numpy(c3["kap"]).to(DEV))
    u = synth.uniform(0, synth.STREAM_U, op.n_dofs)
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)  # the oracle sees the rounded input
    v = op.apply(torch.from_numpy(u).to(DEV, op.dtype), kl).double().cpu().numpy()
    rng = np.random.default_rng(42)
    rows = rng.choice(op.n_dofs, 48, replace=False)
    tree = cKDTree(dof_xyz)
    y, scale = cg_row_values(c3["xyz"], c3["tets"], 3, c3["qp"], c3["qw"], rows, dof_xyz, dof_cell, u, tree,
                             kappa=c3["kap"])
    err = np.abs(v[rows] - y) / scale
    print(f"C3 {precision}: max row error / sum|a u| = {err.max():.3e}")
    assert err.max() <= tol


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_f3_curved_sampled_rows(c3, precision, tol):
    """The same workload on curved cells (per-point Jacobians of the smooth
    map of synth.curved_jacobians, as bench.py --config f3 runs it)."""
    tm = c3["tm"]
    jac = synth.curved_jacobians(c3["xyz"], c3["tets"], c3["qp"], 0.25)
    op = tm.Operator(c3["mesh"], 3, (c3["qp"], c3["qw"]), precision=precision, q_jacobians=jac)
    _, dof_xyz, dof_cell = op.numbering()
    kl = op.cell_data_to_library(torch.from_numpy(c3["kap"]).to(DEV))
    u = synth.uniform(1, synth.STREAM_U, op.n_dofs)
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)
    v = op.apply(torch.from_numpy(u).to(DEV, op.dtype), kl).double().cpu().numpy()
    rows = np.random.default_rng(43).choice(op.n_dofs, 48, replace=False)
    tree = cKDTree(dof_xyz)
    cells = dof_cell[rows]
    locs = oracle_local_node(c3["xyz"], c3["tets"], cells, dof_xyz[rows], 3)
    keys, orows = oracle.cg_rows(c3["xyz"], c3["tets"], 3, c3["qp"], c3["qw"], cells, locs, kappa=c3["kap"],
                                 jac=jac)
    y, scale = [], []
    for row in orows:
        ck = list(row.keys())
        cols = tree.query(key_coords(ck, c3["xyz"], 3))[1]
        coef = np.array([row[k] for k in ck])
        y.append(float(coef @ u[cols]))
        scale.append(float(np.abs(coef) @ np.abs(u[cols])))
    err = np.abs(v[rows] - np.array(y)) / np.array(scale)
    print(f"F3 curved {precision}: max row error / sum|a u| = {err.max():.3e}")
    assert err.max() <= tol


@pytest.mark.parametrize("curved", [False, True])
def test_f2_vector_components_full_size(c3, curved):
    """The vector field (3 components) at full size, as bench.py --config f2
    runs it: every component of the apply is bitwise the scalar operator's
    apply of that component (which the sampled-row tests above check against
    the oracle), for straight and curved cells."""
    tm = c3["tm"]
    jac = synth.curved_jacobians(c3["xyz"], c3["tets"], c3["qp"], 0.25) if curved else None
    opv = tm.Operator(c3["mesh"], 3, (c3["qp"], c3["qw"]), q_jacobians=jac, n_components=3)
    ops = tm.Operator(c3["mesh"], 3, (c3["qp"], c3["qw"]), q_jacobians=jac)
    kl = ops.cell_data_to_library(torch.from_numpy(c3["kap"]).to(DEV))
    n = ops.n_dofs
    u = torch.from_numpy(synth.uniform(2, synth.STREAM_U, 3 * n)).to(DEV)
    v = opv.apply(u, kl)
    for c in range(3):
        assert torch.equal(v[c * n:(c + 1) * n], ops.apply(u[c * n:(c + 1) * n].contiguous(), kl))


def test_c2_dg_sampled_cells():
    tm = _tm()
    n, p = 32, 3
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    fp, fw = synth.tri_rule(6)
    mesh = tm.Mesh(xyz, tets)
    kc = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    kf = synth.lognormal(0, synth.STREAM_KAPPA_FACE, (mesh.n_face, fw.size), sigma=0.5)
    op = tm.Operator(mesh, p, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    assert op.n_dofs == 20 * 6 * n ** 3
    cp, dof_xyz, dof_cell = op.numbering()
    u = synth.uniform(0, synth.STREAM_U, op.n_dofs)  # library order
    klc = op.cell_data_to_library(torch.from_numpy(kc).to(DEV))
    klf = torch.from_numpy(kf.T.copy()).to(DEV)
    v = op.apply(torch.from_numpy(u).to(DEV), klc, klf).cpu().numpy()
    # oracle numbering (user cell, lexicographic node) of every library DoF, chunked
    nd = 20
    o_idx = np.empty(op.n_dofs, dtype=np.int64)
    for s in range(0, op.n_dofs, 400000):
        sl = slice(s, min(op.n_dofs, s + 400000))
        o_idx[sl] = dof_cell[sl].astype(np.int64) * nd + oracle_local_node(xyz, tets, dof_cell[sl], dof_xyz[sl], p)
    u_or = np.empty(op.n_dofs)
    u_or[o_idx] = u
    rng = np.random.default_rng(7)
    sel = rng.choice(tets.shape[0], 16, replace=False)
    R = oracle.dg_rows(xyz, tets, p, qp, qw, fp, fw, sel, kc, kf, bc="dirichlet")
    y = R @ u_or
    scale = abs(R) @ np.abs(u_or)
    lib_of = np.empty(op.n_dofs, dtype=np.int64)
    lib_of[o_idx] = np.arange(op.n_dofs)
    rows_lib = lib_of[(sel[:, None] * nd + np.arange(nd)).ravel()]
    err = np.abs(v[rows_lib] - y) / scale
    print(f"C2 DG: max row error / sum|a u| = {err.max():.3e}")
    assert err.max() <= 1e-12


def test_c4_backward_and_finite_differences():
    tm = _tm()
    n, p = 48, 2
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(4)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    mesh = tm.Mesh(xyz, tets)
    op = tm.Operator(mesh, p, (qp, qw), sigma=1.0)
    assert op.n_dofs == (2 * n + 1) ** 3
    cp, dof_xyz, dof_cell = op.numbering()
    kl = op.cell_data_to_library(torch.from_numpy(kap).to(DEV))
    u = synth.uniform(0, synth.STREAM_U, op.n_dofs)
    f = synth.uniform(0, synth.STREAM_F, op.n_dofs)
    ut = torch.from_numpy(u).to(DEV)
    ft = torch.from_numpy(f).to(DEV)
    # L = 1/2 ||A u - f||^2 through the autograd function
    kv = kl.clone().requires_grad_(True)
    uv = ut.clone().requires_grad_(True)
    v = tm.apply_autograd(op, uv, kv)
    loss = 0.5 * torch.sum((v - ft) ** 2)
    loss.backward()
    g = (v - ft).detach().cpu().numpy()
    du = uv.grad.cpu().numpy()
    dk_user = op.cell_data_to_user(kv.grad).cpu().numpy()
    tree = cKDTree(dof_xyz)
    rng = np.random.default_rng(5)
    rows = rng.choice(op.n_dofs, 32, replace=False)
    y, scale = cg_row_values(xyz, tets, p, qp, qw, rows, dof_xyz, dof_cell, g, tree, kappa=kap, sigma=1.0)
    assert (np.abs(du[rows] - y) / scale).max() <= 1e-12
    # coefficient gradient of sampled cells against the oracle formula on those cells
    cells = rng.choice(tets.shape[0], 24, replace=False)
    sub = tets[cells]
    d_sub = oracle.cg_dofs(xyz, sub, p)
    cols = tree.query(d_sub["xyz"])[1]
    dko = oracle.cg_kappa_grad(xyz, sub, p, qp, qw, u[cols], g[cols], dofs=d_sub)
    assert np.abs(dk_user[cells] - dko).max() <= 1e-12 * np.abs(dko).max()
    # central finite differences on 64 entries, differenced over the touched rows
    picks = synth.fd_picks(0, tets.shape[0] * qw.size, 64)
    h = 1e-6
    worst = 0.0
    lib_of_user = np.empty(tets.shape[0], dtype=np.int64)
    lib_of_user[cp] = np.arange(tets.shape[0])
    ad_max = np.abs(dk_user).max()
    for pk in picks:
        e, q = divmod(int(pk), qw.size)
        cell_dofs = tree.query(oracle.cg_dofs(xyz, tets[e:e + 1], p)["xyz"])[1]
        le = lib_of_user[e]
        vals = []
        for sgn in (1.0, -1.0):
            kk = kl.clone()
            kk[op.cell_data_index(q, int(le))] += sgn * h
            vv = op.apply(ut, kk).cpu().numpy()[cell_dofs]
            vals.append(vv)
        vp, vm = vals
        fd = np.sum(0.5 * (vp - vm) * (vp + vm - 2.0 * f[cell_dofs])) / (2 * h)
        ad = dk_user[e, q]
        rel = abs(fd - ad) / max(abs(ad), 1e-3 * ad_max)
        worst = max(worst, rel)
    print(f"C4 finite differences: worst relative error {worst:.3e} over 64 entries")
    assert worst <= 1e-6


def test_c5_mixed_precision_solve():
    tm = _tm()
    n, p = 64, 3
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    mesh = tm.Mesh(xyz, tets)
    op64 = tm.Operator(mesh, p, (qp, qw), bc="dirichlet")
    op32 = tm.Operator(mesh, p, (qp, qw), bc="dirichlet", precision="f32")
    b = op64.load_vector()
    x_ir, st_ir, ok_ir = op64.solve(b, inner=op32, rtol=1e-10, inner_rtol=1e-4)
    x_ru, st_ru, ok_ru = op64.solve(b, inner=op32, rtol=1e-10, inner_rtol=1e-2, method="reliable")
    x_cg, st_cg, ok_cg = op64.solve(b, rtol=1e-10, max_inner=20000)
    print(f"C5: FP32-inner IR {st_ir}; FP32 reliable updates {st_ru}; FP64 PCG {st_cg}")
    assert ok_ir and ok_ru and ok_cg
    assert max(st_ir["final_relres"], st_ru["final_relres"], st_cg["final_relres"]) <= 1e-10
    xi, xc = x_ir.cpu().numpy(), x_cg.cpu().numpy()
    assert np.linalg.norm(xi - xc) <= 1e-8 * np.linalg.norm(xc)
    assert np.linalg.norm(x_ru.cpu().numpy() - xc) <= 1e-8 * np.linalg.norm(xc)
    # residual of sampled free rows with the oracle: r_i = b_i - sum_j A_ij x_j
    _, dof_xyz, dof_cell = op64.numbering()
    tree = cKDTree(dof_xyz)
    rng = np.random.default_rng(3)
    rows = rng.choice(op64.n_free, 24, replace=False)
    ax, scale = cg_row_values(xyz, tets, p, qp, qw, rows, dof_xyz, dof_cell, xi, tree)
    bb = b.cpu().numpy()[rows]
    assert np.abs(bb - ax).max() <= 1e-9 * np.abs(bb).max() + 1e-12 * scale.max()
