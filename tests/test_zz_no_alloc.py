"""The allocation-free apply (tetmf_apply_noalloc) through the C ABI: the
interface partial sums in the library's fixed device scratch give bitwise
the result of tetmf_apply (same kernels, same summation order), and both
match the oracle entry by entry.  Two calls in a row, the second on a
smaller operator (the scratch keeps the first call's contents), a vector
field in FP32, the largest scalar workload (64^3 x 6 P3 FP64, 40 MB of
partial sums) and the rejection of an operator whose partial sums exceed
the scratch."""
import numpy as np
import pytest

import oracle
import synth
from tests.tetmf_cases import cg_map, row_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _tm():
    import paper_2509_10226_amd as tm
    return tm


def _case(n, p, qdeg, sigma_kappa, precision="f64", bc="neumann", ncomp=1, with_oracle=True):
    tm = _tm()
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(qdeg)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=sigma_kappa)
    op = tm.Operator(tm.Mesh(xyz, tets), p, (qp, qw), precision=precision, bc=bc, n_components=ncomp)
    kl = op.cell_data_to_library(torch.from_numpy(kap).to(DEV))
    c = dict(op=op, kl=kl)
    if with_oracle:
        A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, kappa=kap, dirichlet=(bc == "dirichlet"))
        _, dxyz, _ = op.numbering()
        c.update(A=A, idx=cg_map(dxyz, d["xyz"], 1.0 / n))
    return c


def _both(c, u_lib):
    """(tetmf_apply result, tetmf_apply_noalloc result) for the same input."""
    op = c["op"]
    ut = torch.from_numpy(u_lib).to(DEV, op.dtype)
    v_ref = op.apply(ut, c["kl"])
    v_na = torch.full_like(v_ref, float("nan"))
    op.apply_noalloc(ut, v_na, c["kl"])
    torch.cuda.synchronize()
    return v_ref.cpu(), v_na.cpu()


def test_noalloc_two_calls_second_smaller():
    big = _case(6, 3, 6, 1.0)
    small = _case(4, 3, 6, 0.5, bc="dirichlet")
    # both use the scratch (several blocks), the second call less of it
    assert 0 < small["op"].info["n_partials"] < big["op"].info["n_partials"]
    for c in (big, small):
        u = synth.uniform(0, synth.STREAM_U, c["A"].shape[0])
        v_ref, v_na = _both(c, u[c["idx"]])
        assert torch.equal(v_ref, v_na), "noalloc apply differs from tetmf_apply"
        err = row_err(v_na.numpy(), c["A"], u, c["idx"])
        print(f"n_partials {c['op'].info['n_partials']}: entry-wise error vs oracle {err:.2e}")
        assert err <= 1e-12


def test_noalloc_vector_field_f32():
    c = _case(4, 3, 6, 1.0, precision="f32", ncomp=3, with_oracle=False)
    u = synth.uniform(0, synth.STREAM_U, c["op"].n_vec)
    v_ref, v_na = _both(c, u)
    assert torch.equal(v_ref, v_na)


def test_noalloc_largest_scalar_workload():
    c = _case(64, 3, 6, 1.0, with_oracle=False)
    need = c["op"].info["n_partials"] * 8
    assert need <= 64 << 20
    u = synth.uniform(0, synth.STREAM_U, c["op"].n_dofs)
    v_ref, v_na = _both(c, u)
    assert torch.equal(v_ref, v_na)


def test_noalloc_rejects_scratch_overflow():
    tm = _tm()
    c = _case(56, 3, 6, 1.0, ncomp=3, with_oracle=False)
    op = c["op"]
    assert op.info["n_partials"] * 3 * 8 > 64 << 20
    u = torch.zeros(op.n_vec, dtype=torch.float64, device=DEV)
    out = torch.full_like(u, 7.0)
    with pytest.raises(tm.TetmfError) as e:
        op.apply_noalloc(u, out, c["kl"])
    assert e.value.status == -4  # TETMF_ERR_UNSUPPORTED
    assert "fixed scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0), "a rejected call must launch nothing"
