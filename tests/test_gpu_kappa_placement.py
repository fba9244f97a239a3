"""The HIP operators against closed forms with a coefficient field sampled at
the physical quadrature points (the pairing of coefficient values with
points documented in include/tetmf.h), and the manufactured-solution solve.

No oracle matrix is involved in the coefficient tests: the library's own DoF
coordinates give the nodal interpolants of the monomials, and the expected
values are the integrals of tests/test_oracle_kappa_placement.py (eq. (2)
cell term, eq. (3) face terms on a half box).  The solve tests compare the
GPU solution with the oracle's sparse direct solution and check the L2 rate
p + 1 (Sec. 4.1 states optimal convergence)."""
import numpy as np
import pytest

import oracle
import synth
from tests import test_oracle_kappa_placement as kp
from tests import test_oracle_mms as mms
from tests.tetmf_cases import cg_map

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda", 0)


@pytest.mark.parametrize("p,precision", [(2, "f64"), (3, "f64"), (3, "f32")])
def test_cg_cell_kappa_placement_closed_form(p, precision):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(3, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), precision=precision)
    kl = op.cell_data_to_library(torch.from_numpy(kp.kappa_at(kp.cell_points(xyz, tets, qp))).to(_dev()))
    _, X, _ = op.numbering()
    tol = 1e-12 if precision == "f64" else 2e-5
    for e1 in kp.monomials(p):
        for e2 in kp.monomials(p):
            ex = kp.cell_closed_form(kp.mono(e1), kp.mono(e2))
            v = op.apply(torch.from_numpy(kp.peval(kp.mono(e2), X)).to(_dev(), op.dtype), kl)
            got = kp.peval(kp.mono(e1), X) @ v.double().cpu().numpy()
            assert abs(got - ex) <= tol * max(1.0, abs(ex)), (e1, e2, got, ex)


@pytest.mark.parametrize("p", [2, 3])
def test_dg_face_kappa_placement_closed_form(p):
    import paper_2509_10226_amd as tm
    n = 2
    xyz, tets = synth.kuhn_cube_mesh(n, 0.0, 0)
    qp, qw = synth.tet_rule(2 * p)
    fp, fw = synth.tri_rule(2 * p)
    mesh = tm.Mesh(xyz, tets)
    op = tm.Operator(mesh, p, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    tri = kp.canonical_faces(tets)
    assert tri.shape[0] == mesh.n_face
    klc = op.cell_data_to_library(torch.from_numpy(kp.kappa_at(kp.cell_points(xyz, tets, qp))).to(_dev()))
    klf = torch.from_numpy(kp.kappa_at(kp.face_points(xyz, tri, fp)).T.copy()).to(_dev())
    _, X, dcell = op.numbering()
    cen = np.asarray(xyz)[np.asarray(tets)].mean(axis=1)
    left = cen[dcell, 0] < 0.5
    for e1, e2 in kp.half_box_pairs(p):
        u = np.where(left, kp.peval(kp.mono(e1), X), 0.0)
        v = kp.peval(kp.mono(e2), X)
        ex = kp.half_box_expected(p, n, e1, e2)
        scale = max(1.0, abs(ex), 3.0 * (p + 1) ** 2 * n)
        Av = op.apply(torch.from_numpy(v).to(_dev()), klc, klf).cpu().numpy()
        Au = op.apply(torch.from_numpy(u).to(_dev()), klc, klf).cpu().numpy()
        assert abs(u @ Av - ex) <= 1e-12 * scale, (e1, e2, u @ Av, ex)
        assert abs(v @ Au - ex) <= 1e-12 * scale, (e1, e2, v @ Au, ex)


def _gpu_mms(p, n, inner=None):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(2 * p)
    mesh = tm.Mesh(xyz, tets)
    op = tm.Operator(mesh, p, (qp, qw), bc="dirichlet")
    f = op.cell_data_to_library(torch.from_numpy(mms.source(xyz, tets, qp)).to(_dev()))
    b = op.load_vector(f)
    opi = tm.Operator(mesh, p, (qp, qw), bc="dirichlet", precision=inner) if inner else None
    x, st, ok = op.solve(b, inner=opi, rtol=1e-11, max_inner=20000)
    assert ok and st["final_relres"] <= 1e-11, st
    d = oracle.cg_dofs(xyz, tets, p)
    _, X, _ = op.numbering()
    idx = cg_map(X, d["xyz"], 1.0 / n)
    xo = np.zeros(d["xyz"].shape[0])
    xo[idx] = x.cpu().numpy()
    return xyz, tets, d, xo


@pytest.mark.parametrize("p,ns", [(2, (4, 8, 16)), (3, (4, 8))])
def test_mms_solve_rate_and_oracle_solution(p, ns):
    errs = []
    for n in ns:
        xyz, tets, d, x = _gpu_mms(p, n)
        errs.append(mms.l2_error(xyz, tets, p, x, d["dofmap"]))
        if n <= 8:
            _, _, do, xo = mms.oracle_solution(p, n)
            assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    for i in range(len(ns) - 1):
        rate = np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i])
        assert p + 1 - 0.25 <= rate <= p + 1 + 0.4, (errs, rate)


def test_mms_mixed_precision_solution_matches_fp64():
    """FP32-inner iterative refinement reaches the FP64 solution of the
    manufactured problem (both stop at a true FP64 residual of 1e-11)."""
    p, n = 3, 8
    _, _, _, x64 = _gpu_mms(p, n)
    xyz, tets, d, x32 = _gpu_mms(p, n, inner="f32")
    assert np.linalg.norm(x32 - x64) <= 1e-8 * np.linalg.norm(x64)
    e = mms.l2_error(xyz, tets, p, x32, d["dofmap"])
    assert e < 5e-5
