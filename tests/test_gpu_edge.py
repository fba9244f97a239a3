"""Degenerate and ragged inputs on the GPU: a single tetrahedron (one
partial tile, every face on the boundary), one cube of six cells, the
five-tetrahedra cube split of the paper's throughput studies (Sec. 2.3),
and cell counts that end in a ragged tile and block."""
import numpy as np
import pytest

import oracle
import synth
from tests.tetmf_cases import cg_map, dg_map, rel_err, row_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ONE_TET = (np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.0, 0.1], [0.1, 0.2, 1.0]]),
           np.array([[0, 1, 2, 3]], dtype=np.int32))


def _cg_check(xyz, tets, p, h, bc="neumann", sigma=0.0, precision="f64", curved=False, ncomp=1):
    import paper_2509_10226_amd as tm
    qp, qw = synth.tet_rule(2 * p)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25) if curved else None
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, sigma=sigma, dirichlet=(bc == "dirichlet"), jac=jac)
    A = oracle.vector_operator(A, ncomp) if ncomp > 1 else A
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), bc=bc, sigma=sigma, precision=precision, q_jacobians=jac,
                     n_components=ncomp)
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], h)
    idx = np.concatenate([c * d["xyz"].shape[0] + idx for c in range(ncomp)])
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    u = synth.uniform(0, synth.STREAM_U, A.shape[0])
    if precision != "f64":
        u = u.astype(np.float32).astype(np.float64)
    v = op.apply(torch.from_numpy(u[idx]).to("cuda", op.dtype), kl).double().cpu().numpy()
    # the larger of the vector-norm error and the entry-wise error against
    # each row's scale sum_j |a_ij| |u_j|
    return max(rel_err(v, (A @ u)[idx]), row_err(v, A, u, idx))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_cg_single_tet(p, bc):
    xyz, tets = ONE_TET
    assert _cg_check(xyz, tets, p, 1.0, bc=bc, sigma=0.5) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_cg_one_cube(p):
    xyz, tets = synth.kuhn_cube_mesh(1, 0.0, 0)
    assert _cg_check(xyz, tets, p, 1.0) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_cg_five_tet_cube_mesh(precision, tol):
    xyz, tets = synth.five_tet_cube_mesh(3)
    assert _cg_check(xyz, tets, 3, 1.0 / 3, bc="dirichlet", precision=precision) <= tol


def test_cg_ragged_block():
    # 7^3 x 6 = 2058 cells: 8 full 256-cell blocks and a ragged ninth, ragged last tile
    xyz, tets = synth.kuhn_cube_mesh(7, 0.15, 1)
    assert tets.shape[0] % 256 != 0 and tets.shape[0] % 16 != 0
    assert _cg_check(xyz, tets, 3, 1.0 / 7, sigma=0.2) <= 1e-12


@pytest.mark.parametrize("mesh", ["one_tet", "one_cube"])
def test_dg_small(mesh):
    import paper_2509_10226_amd as tm
    xyz, tets = ONE_TET if mesh == "one_tet" else synth.kuhn_cube_mesh(1, 0.0, 0)
    p = 3
    qp, qw = synth.tet_rule(6)
    fp, fw = synth.tri_rule(6)
    m = tm.Mesh(xyz, tets)
    kc = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    kf = synth.lognormal(0, synth.STREAM_KAPPA_FACE, (m.n_face, fw.size), sigma=0.5)
    A, _ = oracle.assemble_dg(xyz, tets, p, qp, qw, fp, fw, kc, kf, bc="dirichlet")
    op = tm.Operator(m, p, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    _, dxyz, dcell = op.numbering()
    idx = dg_map(dxyz, dcell, xyz, tets, p)
    klc = op.cell_data_to_library(torch.from_numpy(kc).cuda())
    klf = torch.from_numpy(kf.T.copy()).cuda()
    u = synth.uniform(0, synth.STREAM_U, A.shape[0])
    v = op.apply(torch.from_numpy(u[idx]).cuda(), klc, klf).cpu().numpy()
    assert rel_err(v, (A @ u)[idx]) <= 1e-12
    assert row_err(v, A, u, idx) <= 1e-12


@pytest.mark.parametrize("mesh", ["one_tet", "ragged"])
@pytest.mark.parametrize("curved,ncomp", [(True, 1), (False, 3), (True, 3)])
def test_cg_curved_and_vector_edge_meshes(mesh, curved, ncomp):
    if mesh == "one_tet":
        xyz, tets = ONE_TET
        h = 1.0
    else:
        xyz, tets = synth.kuhn_cube_mesh(7, 0.15, 1)
        h = 1.0 / 7
    assert _cg_check(xyz, tets, 3, h, bc="dirichlet", sigma=0.3, curved=curved, ncomp=ncomp) <= 1e-12


@pytest.mark.parametrize("mesh", ["one_tet", "one_cube"])
def test_dg_backward_small(mesh):
    """SIPG coefficient gradients on meshes with only boundary faces (one
    tetrahedron) and with both kinds (one cube)."""
    import paper_2509_10226_amd as tm
    xyz, tets = ONE_TET if mesh == "one_tet" else synth.kuhn_cube_mesh(1, 0.0, 0)
    qp, qw = synth.tet_rule(4)
    fp, fw = synth.tri_rule(4)
    m = tm.Mesh(xyz, tets)
    op = tm.Operator(m, 2, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    _, dxyz, dcell = op.numbering()
    idx = dg_map(dxyz, dcell, xyz, tets, 2)
    n = op.n_dofs
    u = synth.uniform(1, synth.STREAM_U, n)
    g = synth.uniform(1, synth.STREAM_F, n)
    _, dk, dkf = op.backward(torch.from_numpy(u[idx]).cuda(), torch.from_numpy(g[idx]).cuda(), need_du=False,
                             need_dkappa_face=True)
    dkc_o, dkf_o = oracle.dg_kappa_grad(xyz, tets, 2, qp, qw, fp, fw, u, g, bc="dirichlet")
    assert rel_err(op.cell_data_to_user(dk).cpu().numpy(), dkc_o) <= 1e-12
    assert rel_err(dkf.cpu().numpy().T, dkf_o) <= 1e-12


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cell_data_layout_tiles(precision):
    """Per-point cell data in library layout: point q of library cell i at
    ((i / 16) n_q + q) 16 + i % 16, the padding of the partly used last tile
    zero, and the conversion back to user layout exact (3^3 x 6 = 162 cells:
    ten full tiles and one with two cells)."""
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(4)
    op = tm.Operator(tm.Mesh(xyz, tets), 2, (qp, qw), precision=precision)
    nc, nq = tets.shape[0], qw.size
    assert nc % 16 != 0
    assert op.n_cell_data == nq * 16 * ((nc + 15) // 16)
    data = synth.uniform(4, synth.STREAM_KAPPA_CELL, nc * nq).reshape(nc, nq)
    if precision != "f64":
        data = data.astype(np.float32).astype(np.float64)
    kl = op.cell_data_to_library(torch.from_numpy(data).cuda())
    assert kl.numel() == op.n_cell_data
    cp, _, _ = op.numbering()
    lib = kl.double().cpu().numpy()
    cells = np.arange(nc)
    expected = np.zeros(op.n_cell_data)
    for q in range(nq):
        expected[op.cell_data_index(q, cells)] = data[cp, q]
    assert np.array_equal(lib, expected)
    assert np.array_equal(op.cell_data_to_user(kl).cpu().numpy(), data)
