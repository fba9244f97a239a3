"""Applies captured in a HIP graph (torch.cuda.graph on the current stream)
and replayed: every replay, with eager work on the same operator between
replays, must equal the eager result bitwise (the apply is deterministic and
records no memset or host synchronisation, so a replay is the same kernel
sequence)."""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _capture_and_check(op, args, n):
    u = torch.from_numpy(synth.uniform(5, synth.STREAM_U, n)).cuda().to(op.dtype)
    ref = op.apply(u, *args).clone()
    out = torch.empty_like(ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        op.apply(u, *args, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        op.apply(u, *args, out=out)
    for _ in range(4):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        op.apply(u * 2, *args)  # eager work on the same operator between the replays
        torch.cuda.synchronize()
    u.mul_(-1)  # the graph reads the captured buffers: a new input is seen by the next replay
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, op.apply(u, *args))


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16in"])
def test_graph_cg(precision):
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(8, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    op = tm.Operator(tm.Mesh(xyz, tets), 3, (qp, qw), precision=precision, bc="dirichlet", sigma=0.5)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=1.0)
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    _capture_and_check(op, (kl,), op.n_vec)


def test_graph_dg_and_vector():
    import paper_2509_10226_amd as tm
    xyz, tets = synth.kuhn_cube_mesh(6, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    fp, fw = synth.tri_rule(6)
    mesh = tm.Mesh(xyz, tets)
    op = tm.Operator(mesh, 3, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    _capture_and_check(op, (), op.n_vec)
    opv = tm.Operator(mesh, 3, (qp, qw), n_components=3, q_jacobians=synth.curved_jacobians(xyz, tets, qp, 0.25))
    _capture_and_check(opv, (), opv.n_vec)
