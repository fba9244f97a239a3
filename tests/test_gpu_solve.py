"""GPU solver: Jacobi-PCG in FP64 and FP32-inner iterative refinement on a
Dirichlet Poisson problem, checked against the oracle's sparse direct
solution and its own true FP64 residual."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from tests.tetmf_cases import cg_map, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("inner,method", [(None, "refinement"), ("f32", "refinement"), ("f32", "reliable"),
                                          ("bf16in", "reliable")])
def test_solve_poisson_dirichlet(inner, method):
    import paper_2509_10226_amd as tm
    n, p = 6, 3
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    A, d = oracle.assemble_cg(xyz, tets, p, qp, qw, dirichlet=True)
    b = oracle.load_vector(xyz, tets, p, qp, qw, dirichlet=True, dofs=d)
    x_ref = spla.spsolve(A.tocsc(), b)
    mesh = tm.Mesh(xyz, tets)
    op = tm.Operator(mesh, p, (qp, qw), bc="dirichlet")
    _, dxyz, _ = op.numbering()
    idx = cg_map(dxyz, d["xyz"], 1.0 / n)
    bt = op.load_vector()
    assert rel_err(bt.cpu().numpy(), b[idx]) <= 1e-12
    opi = tm.Operator(mesh, p, (qp, qw), bc="dirichlet", precision=inner) if inner else None
    x, st, ok = op.solve(bt, inner=opi, rtol=1e-10, method=method)
    assert ok, st
    xs = x.cpu().numpy()
    # true residual with the oracle matrix in oracle order
    xo = np.empty_like(xs)
    xo[idx] = xs
    assert np.linalg.norm(b - A @ xo) <= 1.0001e-10 * np.linalg.norm(b)
    assert rel_err(xo, x_ref) <= 1e-8
    assert st["final_relres"] <= 1e-10
