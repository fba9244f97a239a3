"""bench.py's roofline bookkeeping, on the host: the bound chosen by
arithmetic intensity, and which launches carry a measured HBM traffic
figure (only the kernel and mesh that the committed counter summary covers)."""
import bench


class _Op:
    """The two fields roofline() reads from an operator."""

    def __init__(self, n_cell, flops=1.0e10, nbytes=6.0e8):
        self.n_cell = n_cell
        self.info = {"flops_per_apply": flops, "bytes_per_apply": nbytes}


def test_bound_by_intensity():
    op = _Op(bench.PROFILED_CELLS)
    r64 = bench.roofline(op, "f64", 0.25)        # 16.7 flop/B > 78.6 T / 8 TB/s
    assert r64["bound"] == "mfma" and r64["unit"] == "TFLOP/s"
    assert abs(r64["achieved"] - 1.0e10 / 0.25e-3 / 1e12) < 1e-3
    assert abs(r64["frac"] - r64["achieved"] / 78.6) < 1e-4
    rbf = bench.roofline(op, "bf16in", 0.25)     # below the BF16 ridge
    assert rbf["bound"] == "hbm" and rbf["unit"] == "GB/s"
    assert abs(rbf["achieved"] - 6.0e8 / 0.25e-3 / 1e9) < 0.1


def test_traffic_only_for_profiled_kernel_and_mesh():
    full = _Op(bench.PROFILED_CELLS)
    for prec in ("f64", "f32", "bf16in"):
        assert bench.roofline(full, prec, 0.25, traffic_key="apply")["traffic"] == bench.read_traffic(prec)
        # no summary named (SIPG, P2, reduced rule, vector field): no figure
        assert bench.roofline(full, prec, 0.25)["traffic"] is None
        # another mesh size: the per-launch figure does not apply
        small = _Op(bench.PROFILED_CELLS // 8)
        assert bench.roofline(small, prec, 0.25, traffic_key="apply")["traffic"] is None
    for prec in ("f64", "f32"):
        assert (bench.roofline(full, prec, 0.25, traffic_key="curved")["traffic"]
                == bench.read_traffic(prec, bench.TRAFFIC_FILE_CURVED))
