#!/usr/bin/env python3
"""Throughput of the matrix-free operator apply (DoFs/s per apply) and its
roofline fraction on one MI355X.

Workload (one "step" = one application v = A(kappa) u, i.e. gather,
interpolate, point operator, integrate and scatter over the whole mesh):
continuous Galerkin P3 Poisson with a lognormal (mu = 0, sigma = 1)
coefficient per quadrature point on the unit cube split into 64^3 cubes x 6
Kuhn tetrahedra (1,572,864 cells, 7,189,057 DoFs), interior vertices
jittered by up to 0.15 h (seed 0), symmetric 24-point degree-6 cell rule,
random input vector.  ``value`` is the FP64 apply; the FP32 (matrix-core
f32) and BF16-operand applies on the same inputs are reported beside it.

Timing: each measurement starts after about 1 s of untimed calls (the GPU
leaves its idle clock state; the first launches after host-side set-up run
slower), and every timed loop runs its calls back to back (an event or a
host gap between calls measurably slows the next ones for tens of calls).
The apply (cell kernel + combine) is captured in a HIP graph and replayed;
``ms_per_step`` is the mean over the `steps` timed replays (after `warmup`
untimed ones) bracketed by device synchronisations, and ``step_ms`` gives
the median and 10th/90th percentiles over 10 further such loops.  The
roofline object refers to the dominant kernel (the cell kernel):
algorithmic flops (or bytes) per launch divided by the MEDIAN of its launch
durations, from the start and end timestamps of each dispatch (HIP events
attached to the launch on the stream it runs on) over at least 50
consecutive launches.
``traffic`` is the HBM byte count per launch from rocprofv3 FETCH_SIZE +
WRITE_SIZE counters scaled by a copy-kernel calibration (profiles/), or null
when the kernel source changed since the counters were taken.

The same line carries every other measured workload as a compact object:
``c2`` (SIPG P3 apply and backward), ``c4`` (P2 Helmholtz forward and
backward), ``c5`` (time to a 1e-10 residual, FP32-inner refinement against
FP64 PCG), ``f1`` (reduced cell rule), ``f2`` (3-component vector field),
``f3`` (curved cells), ``f4`` (Chebyshev-Jacobi smoothing) and ``order``
(randomly relabelled mesh); c2 and c4 also state a cold-cache apply (a
1 GiB buffer written between applies evicts L2 and the last-level cache).

The CPU baseline is the oracle's threaded CSR sparse matrix-vector product
(the matrix-based comparison of Sec. 3.2) on the host's cores, on a bounded
sample of the same workload (32^3 x 6 cells); assembly is reported apart.
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16in": 2500.0}   # MI355X dense matrix-core peaks
PEAK_HBM_GBS = 8000.0
METRIC = "DoFs/s per operator apply, p=3 CG, FP64 vs FP32-MFMA; % of roofline"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_apply_p3_n64_traffic.txt")
TRAFFIC_FILE_CURVED = os.path.join(ROOT, "profiles", "cg_curved_p3_n64_traffic.txt")
# The counter summaries cover the CG P3 cell kernel on the 64^3 x 6 mesh: the
# straight-sided apply ("apply") and the curved-cell apply ("curved").
TRAFFIC_FILES = {"apply": TRAFFIC_FILE, "curved": TRAFFIC_FILE_CURVED}
PROFILED_CELLS = 6 * 64 ** 3
KERNEL_SRC = os.path.join(ROOT, "paper_2509_10226_amd", "csrc", "kernels.hip")
STAT_SAMPLES = 50


def progress(msg):
    """One line on stderr per finished measurement (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(prec, path=TRAFFIC_FILE):
    """Calibrated HBM bytes per launch from the committed counter summary, or None."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_hash():
        return None
    key = f"traffic_bytes_per_launch_{prec}"
    return float(vals[key]) if key in vals else None


def stats(ms):
    """median, 10th and 90th percentile, mean and count of a list of times (ms)."""
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"median": round(float(np.median(a)), 5), "p10": round(float(np.percentile(a, 10)), 5),
            "p90": round(float(np.percentile(a, 90)), 5), "mean": round(float(a.mean()), 5), "n": int(a.size)}


def build_workload(n, seed=0, deg=6, sigma=1.0):
    import synth
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, seed)
    qp, qw = synth.tet_rule(deg)
    kap = synth.lognormal(seed, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), mu=0.0, sigma=sigma)
    return xyz, tets, qp, qw, kap


def rand_vec(n, dtype, seed=2):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    return (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).to("cuda", dtype)


SETTLE_S = 1.0


def settle(fn, seconds=None):
    """Untimed calls for about `seconds`: the GPU leaves its idle clock state
    (after host-side set-up the first launches run measurably slower), so the
    timed loops see the steady state a solver sees."""
    import torch
    seconds = SETTLE_S if seconds is None else seconds
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def loop_ms(fn, steps, warmup):
    """Mean milliseconds per call over `steps` calls after `warmup`, bracketed
    by device synchronisations (profiling off)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


_FLUSH = None


def flush_caches():
    """Write a 1 GiB buffer: evicts the L2 caches and the 256 MB last-level cache."""
    global _FLUSH
    import torch
    if _FLUSH is None:
        _FLUSH = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    _FLUSH.fill_(1.0)


def per_call_ms(fn, n, cold=False):
    """Single-call durations (ms) from HIP events on the current stream; cold:
    the cache-evicting write runs before each call, outside its event pair."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        if cold:
            flush_caches()
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def kernel_ms(op, fn, n):
    """Durations (ms) of the op's main kernel over n calls of fn, from the
    library's event pair around each launch."""
    import torch
    op.profile(True)
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    op.profile(False)
    t = op.profile_times(max(n, 1) * 4)
    return list(t)


def roofline(op, prec, ms, traffic_key=None, backward=False):
    """Roofline of the main kernel at the kernel time ms (the median launch),
    bound chosen by the algorithmic intensity against the ridge point peak
    flops / peak HBM bandwidth: straight-sided FP64 and FP32 are
    compute-bound; BF16 operands (16x the matrix-core peak) and curved cells
    (a geometry per point) are HBM-bound.  traffic: the calibrated HBM bytes
    per launch of the counter summary that traffic_key names, only on the
    mesh those counters were taken on; None for every other kernel."""
    flops = op.info["flops_per_backward" if backward else "flops_per_apply"]
    bytes_alg = op.info["bytes_per_backward" if backward else "bytes_per_apply"]
    tflops = flops / (ms * 1e-3) / 1e12
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    path = TRAFFIC_FILES.get(traffic_key)
    traffic = read_traffic(prec, path) if path and op.n_cell == PROFILED_CELLS else None
    ridge = PEAK_TFLOPS[prec] * 1e12 / (PEAK_HBM_GBS * 1e9)
    common = {"traffic": traffic, "algorithmic_flops": flops, "algorithmic_bytes": bytes_alg,
              "kernel_ms": round(ms, 5)}
    if flops / bytes_alg < ridge:
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), **common, "mfma_achieved_TFLOPs": round(tflops, 3)}
    return {"bound": "mfma", "achieved": round(tflops, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": round(tflops / PEAK_TFLOPS[prec], 4), **common, "hbm_achieved_GBs": round(gbs, 1),
            "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}


def graph_of(fn, ref, out):
    """A HIP graph of one call of fn (writing `out`), or None unless every
    checked replay equals the eager result `ref` bitwise (with eager work
    between the replays)."""
    import torch
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        for _ in range(3):
            out.zero_()
            graph.replay()
            torch.cuda.synchronize()
            if not torch.equal(out, ref):
                return None
            fn()
            torch.cuda.synchronize()
        return graph
    except Exception:  # capture unavailable: eager timing stands
        torch.cuda.synchronize()
        return None


def loop_stats(fn, steps, reps=10):
    """Mean ms per call of `reps` back-to-back loops of `steps` calls, each
    bracketed by a HIP event pair (no event between the calls of a loop)."""
    import torch
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b) / steps)
    return out


def measure_apply(op, kl, u, steps, warmup, prec, traffic_key=None, kf=None, graph=True, cold=False):
    """Apply throughput of an op, every timed loop back to back after a
    settle phase: kernel statistics from the dispatch timestamps of
    max(steps, 50) consecutive launches (median used for the roofline), the
    eager loop, then (when the capture reproduces the eager result bitwise) a
    HIP graph of one apply, replayed: 10 loops of `steps` replays for the
    step statistics and one loop of `steps` for ms_per_step."""
    import torch
    out = torch.empty(op.n_vec, dtype=op.dtype, device="cuda")

    def call():
        op.apply(u, kl, kf, out=out)
    call()
    torch.cuda.synchronize()
    ref = out.clone()
    nstat = max(steps, STAT_SAMPLES)
    settle(call)
    kt = stats(kernel_ms(op, call, nstat))
    settle(call)
    ms_eager = loop_ms(call, steps, warmup)
    g = graph_of(call, ref, out) if graph else None
    step_fn = g.replay if g is not None else call
    settle(step_fn)
    step = stats(loop_stats(step_fn, steps))
    ms_step = loop_ms(step_fn, steps, warmup)
    r = {"value": round(op.n_vec / (ms_step * 1e-3), 1), "ms_per_step": round(ms_step, 5),
         "ms_per_step_eager": round(ms_eager, 5), "timing": "graph" if g is not None else "eager",
         "step_ms": step, "kernel_ms": kt, "roofline": roofline(op, prec, kt["median"], traffic_key)}
    if cold:
        r["cold_step_ms"] = stats(per_call_ms(call, min(nstat, 20), cold=True))
    del g
    return r, ref


# ---------------------------------------------------------------------------
# the headline workload (C3) and the CPU baseline


def headline(args, keep_f64=False):
    import torch

    import paper_2509_10226_amd as tm
    xyz, tets, qp, qw, kap = build_workload(args.n)
    mesh = tm.Mesh(xyz, tets)
    results, outs, kept = {}, {}, None
    for prec in args.precisions.split(","):
        t0 = time.perf_counter()
        op = tm.Operator(mesh, 3, (qp, qw), precision=prec)
        setup_s = time.perf_counter() - t0
        kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
        u = rand_vec(op.n_dofs, op.dtype)
        r, out = measure_apply(op, kl, u, args.steps, args.warmup, prec, traffic_key="apply")
        r.update(n_dofs=op.n_dofs, n_cell=op.n_cell, setup_s=round(setup_s, 2),
                 blocks={"n_blocks": op.info["n_blocks"], "shared_dofs": op.info["n_shared"],
                         "partials": op.info["n_partials"]})
        outs[prec] = out.double()
        results[prec] = r
        progress(f"headline {prec}: {r['value'] / 1e9:.2f} GDoF/s, kernel median {r['kernel_ms']['median']:.4f} ms")
        if keep_f64 and prec == "f64":
            kept = (mesh, op, kl, u, kap, xyz, tets, qp, qw)
        else:
            del op
    return results, outs, kept


def host_cpu():
    """CPU model, sockets and physical cores of this host (lscpu), or {}."""
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name", platform.processor())
        sockets = int(kv.get("Socket(s)", "1"))
        cores = int(kv.get("Core(s) per socket", "0"))
        info["sockets"] = sockets
        info["physical_cores"] = sockets * cores
        info["logical_cpus"] = int(kv.get("CPU(s)", "0"))
    except Exception as e:  # lscpu missing: say so
        info["error"] = str(e)
    try:
        info["cpus_available_to_process"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return info


def cpu_baseline(n_sample=32):
    """The oracle's threaded FP64 CSR product on a sample of the workload,
    with the GPU operator's error against the oracle's product on it."""
    import numpy as np

    import oracle
    from oracle.cpu_spmv import CsrSpmv
    import synth
    xyz, tets, qp, qw, kap = build_workload(n_sample)
    t0 = time.perf_counter()
    A, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=kap)
    t_asm = time.perf_counter() - t0
    u = synth.uniform(0, synth.STREAM_U, A.shape[0])
    m = CsrSpmv(A, u)
    y = m.apply()
    times = m.time(3, 20)
    t_med = float(np.median(times))
    # scipy's single-threaded product as a floor
    t1 = time.perf_counter()
    for _ in range(3):
        ys = A @ u
    t_scipy = (time.perf_counter() - t1) / 3
    nd = A.shape[0]
    parity = {}
    try:
        import torch
        from scipy.spatial import cKDTree

        import paper_2509_10226_amd as tm
        mesh = tm.Mesh(xyz, tets)
        scale = abs(A) @ np.abs(u)
        for prec in ("f64", "f32", "bf16in"):
            op = tm.Operator(mesh, 3, (qp, qw), precision=prec)
            _, dxyz, _ = op.numbering()
            idx = cKDTree(d["xyz"]).query(dxyz)[1]
            kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
            v = op.apply(torch.from_numpy(u[idx]).cuda().to(op.dtype), kl).double().cpu().numpy()
            parity[prec] = {"rel_2norm": float(np.linalg.norm(v - y[idx]) / np.linalg.norm(y)),
                            "max_entry_vs_row_scale": float(np.max(np.abs(v - y[idx]) / scale[idx]))}
            del op
    except RuntimeError as e:  # no GPU: the oracle timing stands alone
        parity = {"error": str(e)}
    cpu = host_cpu()
    return {
        "value": round(nd / t_med, 1),
        "unit": "DoFs/s",
        "cores": CsrSpmv.threads(),
        "kind": "oracle",
        "sample": (f"CG P3 lognormal(0,1) kappa, {n_sample}^3x6 Kuhn tets ({tets.shape[0]} cells, {nd} DoFs, "
                   f"nnz {A.nnz}, CSR {(12 * A.nnz + 8 * nd) / 1e6:.0f} MB): the oracle's FP64 CSR product y = A u "
                   f"(C, OpenMP, {CsrSpmv.threads()} threads), median of 20 after 3 warm-ups; value = DoFs / median"),
        "spmv_ms": stats(times * 1e3),
        "assembly_s": round(t_asm, 3),
        "scipy_one_thread_DoFs_per_s": round(nd / t_scipy, 1),
        "host_cpu": cpu,
        "threads_note": "threads = OMP_NUM_THREADS when set (the process's CPU share), else the CPUs available",
        "max_abs_diff_vs_scipy": float(np.max(np.abs(y - ys))),
        "gpu_err_vs_oracle": parity,
    }


# ---------------------------------------------------------------------------
# the other workloads, each a compact object


def run_c2(args):
    """SIPG P3 apply and backward, 32^3 x 6 cells, lognormal(0, 0.5) cell and face coefficients, Dirichlet mirror."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = 32
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    fp, fw = synth.tri_rule(6)
    mesh = tm.Mesh(xyz, tets)
    kc = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    kf = synth.lognormal(0, synth.STREAM_KAPPA_FACE, (mesh.n_face, fw.size), sigma=0.5)
    op = tm.Operator(mesh, 3, (qp, qw), kind="dg", frule=(fp, fw), bc="dirichlet")
    klc = op.cell_data_to_library(torch.from_numpy(kc).cuda())
    klf = torch.from_numpy(kf.T.copy()).cuda()
    u = rand_vec(op.n_dofs, op.dtype)
    g = rand_vec(op.n_dofs, op.dtype, seed=3)
    r, _ = measure_apply(op, klc, u, args.steps, args.warmup, "f64", kf=klf, cold=True)

    def bwd():
        op.backward(u, g, klc, kappa_face=klf, need_dkappa_face=True)
    settle(bwd)
    bs = stats(loop_stats(bwd, args.steps))
    ms_b = loop_ms(bwd, args.steps, args.warmup)
    r["backward"] = {"what": "du = A g, dkappa_cell, dkappa_face", "ms_per_step": round(ms_b, 5), "step_ms": bs,
                     "roofline": roofline(op, "f64", bs["median"], backward=True)}
    r["workload"] = (f"DG SIPG P3, {n}^3x6 Kuhn tets ({op.n_cell} cells, {op.n_dofs} DoFs), lognormal(0,0.5) cell "
                     "and face kappa, Dirichlet mirror, 24/12-point rules; backward roofline over the whole "
                     "backward (two kernels) at its median step time")
    return r


def run_c4(args):
    """CG P2 Helmholtz (stiffness + 1.0 mass), 48^3 x 6 cells: forward and backward."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = 48
    xyz, tets, qp, qw, kap = build_workload(n, deg=4, sigma=0.5)
    op = tm.Operator(tm.Mesh(xyz, tets), 2, (qp, qw), sigma=1.0)
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    u = rand_vec(op.n_dofs, op.dtype)
    g = rand_vec(op.n_dofs, op.dtype, seed=3)
    r, _ = measure_apply(op, kl, u, args.steps, args.warmup, "f64", cold=True)

    def bwd():
        op.backward(u, g, kl)
    settle(bwd)
    kb = stats(kernel_ms(op, bwd, max(args.steps, STAT_SAMPLES)))
    ms_b = loop_ms(bwd, args.steps, args.warmup)
    r["backward"] = {"what": "du = A g and dkappa per point", "ms_per_step": round(ms_b, 5), "kernel_ms": kb,
                     "roofline": roofline(op, "f64", kb["median"], backward=True),
                     "cold_step_ms": stats(per_call_ms(bwd, 20, cold=True))}
    r["workload"] = (f"CG P2 stiffness + 1.0 mass, {n}^3x6 Kuhn tets ({op.n_cell} cells, {op.n_dofs} DoFs), "
                     "lognormal(0,0.5) kappa, 14-point rule")
    return r


def run_c5(args, include_bf16=True):
    """Time to a true relative residual of 1e-10: FP64 PCG against the mixed-precision solves (FP32 or
    BF16-operand inner PCG; iterative refinement and reliable updates)."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = 64
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    mesh = tm.Mesh(xyz, tets)
    op64 = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet")
    b = op64.load_vector()

    def timed(opi, method="refinement", inner_rtol=1e-4, warm=True):
        if warm:  # allocates the solver scratch
            op64.solve(b, inner=opi, rtol=1e-10, inner_rtol=inner_rtol, max_inner=20000, method=method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, ok = op64.solve(b, inner=opi, rtol=1e-10, inner_rtol=inner_rtol, max_inner=20000, method=method)
        torch.cuda.synchronize()
        return {"wall_s": round(time.perf_counter() - t0, 4), "converged": bool(ok), "outer_its": st["outer_its"],
                "inner_its": st["inner_its"], "final_relres": st["final_relres"]}

    res = {"fp64_pcg": timed(None)}
    ops = {"fp32": tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", precision="f32")}
    if include_bf16:
        ops["bf16"] = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", precision="bf16in")
    for name, opi in ops.items():
        res[f"{name}_inner_ir"] = timed(opi, "refinement", 1e-4)
        res[f"{name}_inner_reliable"] = timed(opi, "reliable", 1e-2)
    # sensitivity of the FP32-inner solves to the inner tolerance
    sweep_ir, sweep_ru = {}, {}
    for irt in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        sweep_ir[f"{irt:g}"] = timed(ops["fp32"], "refinement", irt, warm=False)
    for irt in (1e-1, 1e-2, 1e-3, 1e-4):
        sweep_ru[f"{irt:g}"] = timed(ops["fp32"], "reliable", irt, warm=False)
    del ops
    t64 = res["fp64_pcg"]["wall_s"]
    return {"value_s": res["fp32_inner_reliable"]["wall_s"], "unit": "s", "higher_is_better": False, **res,
            "fp32_inner_ir_by_inner_rtol": sweep_ir, "fp32_inner_reliable_by_inner_rtol": sweep_ru,
            "speedup_fp32_reliable_vs_fp64": round(t64 / res["fp32_inner_reliable"]["wall_s"], 3),
            "speedup_fp32_ir_vs_fp64": round(t64 / res["fp32_inner_ir"]["wall_s"], 3),
            "methods": "ir = iterative refinement (inner PCG restarted per FP64 residual, inner_rtol 1e-4); "
                       "reliable = one inner PCG with FP64 residual replacement every 1e-2 reduction, "
                       "search direction kept (FP32)",
            "workload": f"CG P3 Dirichlet Poisson f=1, kappa=1, {n}^3x6 Kuhn tets ({op64.n_free} free DoFs), "
                        "24-point rule, Jacobi-PCG; stop at true FP64 residual 1e-10"}, (mesh, op64, qp, qw)


def run_f1(args):
    """Reduced cell integration: P3 with the 14-point degree-4 rule."""
    import torch

    import paper_2509_10226_amd as tm
    xyz, tets, qp, qw, kap = build_workload(args.n, deg=4)
    op = tm.Operator(tm.Mesh(xyz, tets), 3, (qp, qw))
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    r, _ = measure_apply(op, kl, rand_vec(op.n_dofs, op.dtype), args.steps, args.warmup, "f64")
    r["workload"] = f"CG P3 Poisson, {args.n}^3x6, lognormal(0,1) kappa per point of the 14-point degree-4 rule"
    return r


def run_f2(args, scalar=None):
    """Vector field (3 components): one batched apply against three scalar applies."""
    import torch

    import paper_2509_10226_amd as tm
    if scalar is None:
        return {"error": "needs the FP64 headline operator"}
    mesh, ops, kl, u1, kap, xyz, tets, qp, qw = scalar
    opv = tm.Operator(mesh, 3, (qp, qw), n_components=3)
    assert torch.equal(opv.cell_data_to_library(torch.from_numpy(kap).cuda()), kl)  # same cell order
    u = rand_vec(opv.n_vec, opv.dtype)
    r, _ = measure_apply(opv, kl, u, args.steps, args.warmup, "f64")
    n = ops.n_dofs
    outs = [torch.empty(n, dtype=ops.dtype, device="cuda") for _ in range(3)]

    def three():
        for c in range(3):
            ops.apply(u[c * n:(c + 1) * n], kl, out=outs[c])
    settle(three)
    ms_three = loop_ms(three, args.steps, args.warmup)
    r["ms_three_scalar_applies"] = round(ms_three, 5)
    r["speedup_vs_three_scalar"] = round(ms_three / r["ms_per_step_eager"], 3)
    r["workload"] = f"vector Poisson, 3 components, CG P3, {args.n}^3x6, lognormal(0,1) kappa, straight cells"
    del opv
    return r


def run_f3(args, scalar=None):
    """Curved cells (per-point Jacobians), CG P3 FP64."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    if scalar is not None:
        mesh, _, _, u, kap, xyz, tets, qp, qw = scalar
    else:
        xyz, tets, qp, qw, kap = build_workload(args.n)
        mesh, u = tm.Mesh(xyz, tets), None
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25)
    op = tm.Operator(mesh, 3, (qp, qw), q_jacobians=jac)
    del jac
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    if u is None:
        u = rand_vec(op.n_dofs, op.dtype)
    r, _ = measure_apply(op, kl, u, args.steps, args.warmup, "f64", traffic_key="curved")
    r["workload"] = (f"CG P3 Poisson, {args.n}^3x6 mapped by (x + 0.25 y^2, y + 0.25 z^2, z + 0.25 x^2), "
                     "lognormal(0,1) kappa, 24-point rule")
    del op
    return r


def run_f4(args, solve_ctx=None):
    """Chebyshev-Jacobi smoothing of degree 5 on the solve workload, FP64."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    if solve_ctx is None:
        xyz, tets = synth.kuhn_cube_mesh(args.n, 0.15, 0)
        qp, qw = synth.tet_rule(6)
        op = tm.Operator(tm.Mesh(xyz, tets), 3, (qp, qw), bc="dirichlet")
    else:
        op = solve_ctx[1]
    inv = 1.0 / op.diagonal()
    t0 = time.perf_counter()
    lam = op.estimate_lambda_max(inv, n_iter=20)
    t_est = time.perf_counter() - t0
    lmax = 1.1 * lam
    b = op.load_vector()
    x = torch.zeros_like(b)

    def smooth():
        op.chebyshev(b, inv, 5, lmax / 15.0, lmax, x=x)
    settle(smooth)
    st = stats(loop_stats(smooth, args.steps))
    ms = loop_ms(smooth, args.steps, args.warmup)
    return {"ms_per_smoothing": round(ms, 5), "smoothing_ms": st, "steps": 5, "ms_per_step": round(ms / 5, 5),
            "DoFs_per_s_per_step": round(op.n_dofs * 5 / (ms * 1e-3), 1), "lambda_max_estimate": lam,
            "estimate_seconds_20_steps": round(t_est, 4),
            "workload": f"CG P3 Poisson, Dirichlet, kappa=1, {args.n}^3x6, FP64, degree 5, interval "
                        "[lambda_max/15, 1.1 lambda_max]"}


def run_order(args, native=None):
    """Randomly relabelled mesh: with the library's locality ordering and taken as given."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    xyz, tets, qp, qw, kap = build_workload(args.n)
    x, t = synth.shuffle_mesh(xyz, tets, 0)
    res = {}
    mesh = tm.Mesh(x, t)
    orderings = ("locality", "as_given") if args.order_variant == "both" else (args.order_variant,)
    for ordering in orderings:
        op = tm.Operator(mesh, 3, (qp, qw), ordering=ordering)
        kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
        u = rand_vec(op.n_dofs, op.dtype)
        r, _ = measure_apply(op, kl, u, args.steps, args.warmup, "f64", graph=False)
        res[f"shuffled_{ordering}"] = {"value": r["value"], "kernel_ms": r["kernel_ms"]["median"],
                                       "partials": op.info["n_partials"]}
        del op
    if native is not None:
        res["native_locality"] = {"value": native["value"], "kernel_ms": native["kernel_ms"]["median"],
                                  "partials": native["blocks"]["partials"]}
    res["workload"] = (f"CG P3 FP64, {args.n}^3x6 with cells and vertices relabelled by a seeded permutation "
                       "(kappa drawn per cell as numbered)")
    return res


CONFIGS = ("c2", "c4", "c5", "f1", "f2", "f3", "f4", "order")


def copy_calibration(mib=1024, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "reps": reps}), flush=True)


def main():
    global SETTLE_S
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64, help="cubes per axis (64 = the measured workload)")
    ap.add_argument("--precisions", default="f64,f32,bf16in")
    ap.add_argument("--config", default="all", choices=("all", "c3") + CONFIGS,
                    help="all (default): the headline line with every other workload inside it; c3: the "
                         "headline alone; c2 ... order: one workload, printed as its own JSON line")
    ap.add_argument("--order-variant", default="both", choices=("both", "locality", "as_given"),
                    help="order workload: the relabelled mesh with the locality ordering, taken as given, or both")
    ap.add_argument("--settle", type=float, default=SETTLE_S,
                    help="seconds of untimed calls before each measurement (0 under a counter profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    SETTLE_S = args.settle
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the operator shards by "
              "cell partition with one exchange of interface partial sums per apply; that path is not implemented).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2509_10226_amd  # noqa: F401  (fails loudly without libtetmf.so)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.config not in ("all", "c3"):
        fn = {"c2": run_c2, "c4": run_c4, "c5": lambda a: run_c5(a)[0], "f1": run_f1, "f2": None, "f3": run_f3,
              "f4": run_f4, "order": run_order}[args.config]
        if fn is None:
            _, _, kept = headline(argparse.Namespace(**{**vars(args), "precisions": "f64"}), keep_f64=True)
            out = run_f2(args, kept)
        else:
            out = fn(args)
        print(json.dumps({"config": args.config, **out}), flush=True)
        return
    t_start = time.perf_counter()
    everything = args.config == "all"
    results, outs, kept = headline(args, keep_f64=everything)
    main_prec = "f64" if "f64" in results else next(iter(results))
    r = results[main_prec]
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "ms_per_step_eager": r["ms_per_step_eager"],
        "step_ms": r["step_ms"],
        "timing": (("one apply (cell kernel + combine) captured in a HIP graph and replayed; replays checked "
                    "bitwise against the eager result; ms_per_step = mean of the timed replays, step_ms = "
                    "single replays; roofline at the median cell-kernel launch")
                   if r["timing"] == "graph" else "applies launched one by one"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {
            "workload": (f"CG P3 Poisson apply, lognormal(0,1) kappa per quadrature point, {args.n}^3x6 Kuhn tets "
                         f"jittered 0.15h seed 0 ({r['n_cell']} cells, {r['n_dofs']} DoFs), 24-point degree-6 rule"),
            "n_cell": r["n_cell"],
            "n_dofs": r["n_dofs"],
            "n_q": 24,
            "ordering": "locality (Morton)",
            "parallelism": "single GPU",
        },
        "roofline": r["roofline"],
        "kernel_ms": r["kernel_ms"],
    }
    for prec, rr in results.items():
        if prec != main_prec:
            line[prec] = {k: rr[k] for k in ("value", "ms_per_step", "ms_per_step_eager", "timing", "step_ms",
                                             "kernel_ms", "roofline")}
            if "f64" in outs:
                # same input (rounded to the operand precision); the FP64
                # operator matches the oracle to 1e-12 (tests)
                ref = outs["f64"]
                line[prec]["rel_diff_vs_f64_operator"] = float(torch.linalg.norm(outs[prec] - ref) /
                                                               torch.linalg.norm(ref))
    line["setup_s"] = r["setup_s"]
    line["blocks"] = r["blocks"]
    del outs
    if everything and args.n == 64:
        def guarded(name, fn):
            t0 = time.perf_counter()
            try:
                out = fn()
            except Exception as e:  # one workload failing does not hide the others
                out = {"error": f"{type(e).__name__}: {e}"}
            if isinstance(out, dict):
                out["wall_s"] = round(time.perf_counter() - t0, 1)
            torch.cuda.empty_cache()
            progress(f"{name} done in {time.perf_counter() - t0:.1f} s" + (f": {out['error']}" if "error" in out
                                                                          else ""))
            return out
        line["f2"] = guarded("f2", lambda: run_f2(args, kept))
        line["order"] = guarded("order", lambda: run_order(args, r))
        line["f3"] = guarded("f3", lambda: run_f3(args, kept))
        kept = None
        torch.cuda.empty_cache()
        line["f1"] = guarded("f1", lambda: run_f1(args))
        line["c2"] = guarded("c2", lambda: run_c2(args))
        line["c4"] = guarded("c4", lambda: run_c4(args))
        ctx = {}

        def c5():
            out, ctx["solve"] = run_c5(args)
            return out
        line["c5"] = guarded("c5", c5)
        line["f4"] = guarded("f4", lambda: run_f4(args, ctx.get("solve")))
        ctx.clear()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline and args.n == 64:
        progress("cpu baseline: oracle assembly and threaded SpMV on the 32^3 x 6 sample")
        cb = cpu_baseline()
        cb["gpu_over_cpu"] = round(line["value"] / cb["value"], 1)
        line["cpu_baseline"] = cb
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
