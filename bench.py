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
f32) apply on the same inputs is reported beside it.

The roofline object refers to the dominant kernel (the cell kernel of the
apply): algorithmic flops per launch (the paper's count, eq. (9), extended
to a per-point coefficient) divided by its average duration, measured with
HIP events on the stream the kernel runs on.  ``traffic`` is the HBM byte
count per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE counters scaled by a
copy-kernel calibration (profiles/), or null when the kernel source changed
since the counters were taken.

The CPU baseline is the oracle as it stands (FP64 sparse assembly plus one
sparse matrix-vector product) timed on a bounded sample of the same workload
(20^3 x 6 cells).
"""
import argparse
import hashlib
import json
import os
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


def build_workload(n, seed=0):
    import synth
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, seed)
    qp, qw = synth.tet_rule(6)
    kap = synth.lognormal(seed, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), mu=0.0, sigma=1.0)
    return xyz, tets, qp, qw, kap


def time_gpu(op, kl, u, steps, warmup):
    """(ms per apply, ms per cell-kernel launch, output).  The apply time is
    taken over `steps` launches with profiling off; the kernel time over a
    second `steps` launches with the HIP event pair on (the events add host
    work and dispatch latency to every call, so they are kept out of the
    first loop)."""
    import torch
    out = torch.empty_like(u)
    for _ in range(warmup):
        op.apply(u, kl, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.apply(u, kl, out=out)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    op.profile(True)
    for _ in range(steps):
        op.apply(u, kl, out=out)
    torch.cuda.synchronize()
    op.profile(False)
    ms_kernel, launches = op.profile_read()
    assert launches == steps
    return ms_step, ms_kernel / launches, out


def time_graph(op, kl, u, steps, warmup, ref):
    """ms per apply when one apply (cell kernel + combine) is captured in a
    HIP graph and replayed; None unless every checked replay equals the
    eager result `ref` bitwise (with eager work between the replays)."""
    import torch
    try:
        out = torch.empty_like(u)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                op.apply(u, kl, out=out)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            op.apply(u, kl, out=out)
        for _ in range(3):
            out.zero_()
            graph.replay()
            torch.cuda.synchronize()
            if not torch.equal(out, ref):
                return None
            op.apply(u, kl)
            torch.cuda.synchronize()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        del graph
        return ms
    except Exception:  # capture unavailable: the eager time stands
        torch.cuda.synchronize()
        return None


def roofline(op, prec, avg_ms, traffic_key=None):
    """Roofline of the cell kernel, bound chosen by the algorithmic intensity
    (flops per byte) against the ridge point peak flops / peak HBM bandwidth:
    straight-sided FP64 and FP32 are compute-bound; BF16 operands (16x the
    matrix-core peak) and curved cells (a geometry per point) are HBM-bound.
    traffic: the calibrated HBM bytes per launch of the counter summary that
    traffic_key names, only on the mesh those counters were taken on; None
    for every other kernel or workload."""
    flops = op.info["flops_per_apply"]
    bytes_alg = op.info["bytes_per_apply"]
    achieved = flops / (avg_ms * 1e-3) / 1e12
    path = TRAFFIC_FILES.get(traffic_key)
    traffic = read_traffic(prec, path) if path and op.n_cell == PROFILED_CELLS else None
    gbs = bytes_alg / (avg_ms * 1e-3) / 1e9
    ridge = PEAK_TFLOPS[prec] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops / bytes_alg < ridge:
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic, "algorithmic_flops": flops,
                "algorithmic_bytes": bytes_alg, "mfma_achieved_TFLOPs": round(achieved, 3),
                "kernel_ms": round(avg_ms, 5)}
    return {
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": PEAK_TFLOPS[prec],
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_TFLOPS[prec], 4),
        "traffic": traffic,
        "algorithmic_flops": flops,
        "algorithmic_bytes": bytes_alg,
        "hbm_achieved_GBs": round(bytes_alg / (avg_ms * 1e-3) / 1e9, 1),
        "hbm_frac": round(bytes_alg / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "kernel_ms": round(avg_ms, 5),
    }


def cpu_baseline(n_sample=20):
    """The oracle (sparse FP64 assembly + SpMV, numpy/scipy, one thread) on a sample."""
    import numpy as np

    import oracle
    import synth
    xyz, tets, qp, qw, kap = build_workload(n_sample)
    t0 = time.perf_counter()
    A, d = oracle.assemble_cg(xyz, tets, 3, qp, qw, kappa=kap)
    t1 = time.perf_counter()
    u = synth.uniform(0, synth.STREAM_U, A.shape[0])
    reps = 10
    for _ in range(reps):
        y = A @ u
    t2 = time.perf_counter()
    t_spmv = (t2 - t1) / reps
    nd = A.shape[0]
    # the GPU operator in each precision on the same sample, against the
    # oracle's product (DoFs matched by coordinates)
    parity = {}
    try:
        import torch
        from scipy.spatial import cKDTree

        import paper_2509_10226_amd as tm
        mesh = tm.Mesh(xyz, tets)
        for prec in ("f64", "f32", "bf16in"):
            op = tm.Operator(mesh, 3, (qp, qw), precision=prec)
            _, dxyz, _ = op.numbering()
            idx = cKDTree(d["xyz"]).query(dxyz)[1]
            kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
            v = op.apply(torch.from_numpy(u[idx]).cuda().to(op.dtype), kl).double().cpu().numpy()
            parity[prec] = float(np.linalg.norm(v - y[idx]) / np.linalg.norm(y))
            del op
    except RuntimeError as e:  # no GPU: the oracle timing stands alone
        parity = {"error": str(e)}
    return {
        "value": round(nd / ((t1 - t0) + t_spmv), 1),
        "unit": "DoFs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"CG P3 lognormal(0,1) kappa, {n_sample}^3x6 Kuhn tets ({tets.shape[0]} cells, {nd} DoFs): "
                   f"oracle FP64 assembly {t1 - t0:.2f} s + one CSR SpMV {t_spmv * 1e3:.2f} ms "
                   f"(nnz {A.nnz}); value = DoFs / (assembly + SpMV)"),
        "spmv_only_value": round(nd / t_spmv, 1),
        "assembly_s": round(t1 - t0, 3),
        "checksum": float(np.abs(y).sum()),
        "gpu_rel_err_vs_oracle": parity,
    }


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


def _time_call(fn, steps, warmup, op=None):
    """Milliseconds per call over `steps` timed calls after `warmup` calls,
    profiling off; with op, a second loop of `steps` calls with its kernel
    profiling on follows (read with op.profile_read())."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if op is not None:
        op.profile(True)
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        op.profile(False)
    return ms


def bench_c2(args):
    """SIPG P3 apply, 32^3 x 6 cells, lognormal(0, 0.5) cell and face coefficients, Dirichlet mirror."""
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
    u = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda") * 2 - 1
    out = torch.empty_like(u)
    ms = _time_call(lambda: op.apply(u, klc, klf, out=out), args.steps, args.warmup, op)
    kms, nl = op.profile_read()
    kms /= nl
    # backward: du = A g (one apply) plus the cell and face coefficient gradients
    g = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda") * 2 - 1
    ms_b = _time_call(lambda: op.backward(u, g, klc, kappa_face=klf, need_dkappa_face=True), args.steps, args.warmup)
    print(json.dumps({"metric": "DoFs/s per SIPG operator apply, P3, FP64", "value": round(op.n_dofs / (ms * 1e-3), 1),
                      "unit": "DoFs/s", "ms_per_step": round(ms, 5), "ms_backward": round(ms_b, 5), "dtype": "f64",
                      "config": {"workload": f"DG SIPG P3, {n}^3x6 Kuhn tets, lognormal(0,0.5) cell+face kappa, "
                                             f"Dirichlet mirror, 24/12-point rules", "n_dofs": op.n_dofs},
                      "roofline": roofline(op, "f64", kms)}), flush=True)


def bench_c4(args):
    """CG P2 Helmholtz (stiffness + 1.0 mass), 48^3 x 6 cells: forward and backward kernels."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = 48
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(4)
    kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), sigma=0.5)
    op = tm.Operator(tm.Mesh(xyz, tets), 2, (qp, qw), sigma=1.0)
    kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
    u = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda") * 2 - 1
    g = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda") * 2 - 1
    ms_f = _time_call(lambda: op.apply(u, kl), args.steps, args.warmup, op)
    kf, nf = op.profile_read()
    ms_b = _time_call(lambda: op.backward(u, g, kl), args.steps, args.warmup, op)
    kb, nb = op.profile_read()
    print(json.dumps({"metric": "DoFs/s per apply and per backward (du, dkappa), CG P2 Helmholtz, FP64",
                      "value": round(op.n_dofs / (ms_f * 1e-3), 1), "unit": "DoFs/s",
                      "ms_forward": round(ms_f, 5), "ms_backward": round(ms_b, 5),
                      "kernel_ms_forward": round(kf / nf, 5), "kernel_ms_backward": round(kb / nb, 5),
                      "backward_DoFs_per_s": round(op.n_dofs / (ms_b * 1e-3), 1), "dtype": "f64",
                      "config": {"workload": f"CG P2 stiffness + 1.0 mass, {n}^3x6 Kuhn tets, lognormal(0,0.5) kappa, "
                                             f"14-point rule", "n_dofs": op.n_dofs},
                      "roofline": roofline(op, "f64", kf / nf)}), flush=True)


def bench_c5(args):
    """Time to a true relative residual of 1e-10: FP32-inner iterative refinement vs FP64 PCG."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = 64
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    mesh = tm.Mesh(xyz, tets)
    op64 = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet")
    res = {}
    for inner in ("f32", "bf16in", None):
        opi = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", precision=inner) if inner else None
        b = op64.load_vector()
        op64.solve(b, inner=opi, rtol=1e-10, max_inner=20000)  # warm-up (allocates solver scratch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, ok = op64.solve(b, inner=opi, rtol=1e-10, max_inner=20000)
        torch.cuda.synchronize()
        st["solver_seconds"] = st.pop("seconds")
        res[inner or "f64"] = dict(wall_seconds=round(time.perf_counter() - t0, 4), converged=ok, **st)
    print(json.dumps({"metric": "time to relative residual 1e-10, CG P3 Dirichlet Poisson f=1",
                      "value": res["f32"]["wall_seconds"], "unit": "s", "higher_is_better": False,
                      "config": {"workload": f"CG P3, {n}^3x6 Kuhn tets, kappa=1, 24-point rule, Jacobi-PCG",
                                 "n_dofs": op64.n_dofs, "n_free": op64.n_free},
                      "fp32_inner_ir": res["f32"], "bf16_inner_ir": res["bf16in"], "fp64_pcg": res["f64"],
                      "speedup_fp32_ir_vs_fp64": round(res["f64"]["wall_seconds"] / res["f32"]["wall_seconds"], 3)}),
          flush=True)


def bench_order(args):
    """Cell and vertex order: the CG P3 FP64 apply of the measured workload on the
    mesh as generated, on a seeded random relabelling of its cells and vertices
    (the stand-in for an unordered mesh from a mesh generator) with the
    library's locality ordering, and on that relabelling taken as given."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    xyz, tets, qp, qw, kap = build_workload(args.n)
    variants = {"native_locality": (False, "locality"), "shuffled_locality": (True, "locality"),
                "shuffled_as_given": (True, "as_given")}
    if args.order_variant != "all":
        variants = {args.order_variant: variants[args.order_variant]}
    res = {}
    for name, (shuffle, ordering) in variants.items():
        # coefficients are drawn per cell of the mesh as numbered (same seed and
        # stream for both numberings)
        x, t = synth.shuffle_mesh(xyz, tets, 0) if shuffle else (xyz, tets)
        op = tm.Operator(tm.Mesh(x, t), 3, (qp, qw), ordering=ordering)
        kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
        g = torch.Generator(device="cpu").manual_seed(2)
        u = (torch.rand(op.n_dofs, generator=g, dtype=torch.float64) * 2 - 1).cuda()
        ms_step, ms_kernel, _ = time_gpu(op, kl, u, args.steps, args.warmup)
        res[name] = {"DoFs_per_s": round(op.n_dofs / (ms_step * 1e-3), 1), "ms_per_step": round(ms_step, 5),
                     "kernel_ms": round(ms_kernel, 5), "partials": op.info["n_partials"]}
        del op
    print(json.dumps({"metric": "DoFs/s per operator apply vs cell order, CG P3 FP64", "unit": "DoFs/s",
                      "dtype": "f64", "config": {"workload": f"CG P3 Poisson, {args.n}^3x6 Kuhn tets, lognormal(0,1) "
                                                             "kappa, 24-point rule; shuffle seed 0"},
                      "variants": res}), flush=True)


def bench_f1(args):
    """Reduced cell integration (a rule exact to degree 2p - 2 = 4, 14 points)
    against the degree-6 rule on the measured workload's mesh, FP64 and FP32."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    xyz, tets = synth.kuhn_cube_mesh(args.n, 0.15, 0)
    mesh = tm.Mesh(xyz, tets)
    res = {}
    for deg in (6, 4):
        qp, qw = synth.tet_rule(deg)
        kap = synth.lognormal(0, synth.STREAM_KAPPA_CELL, (tets.shape[0], qw.size), mu=0.0, sigma=1.0)
        for prec in ("f64", "f32"):
            op = tm.Operator(mesh, 3, (qp, qw), precision=prec)
            kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
            g = torch.Generator(device="cpu").manual_seed(2)
            u = (torch.rand(op.n_dofs, generator=g, dtype=torch.float64) * 2 - 1).to("cuda", op.dtype)
            ms_step, ms_kernel, _ = time_gpu(op, kl, u, args.steps, args.warmup)
            res[f"degree{deg}_{prec}"] = {"n_q": int(qw.size), "DoFs_per_s": round(op.n_dofs / (ms_step * 1e-3), 1),
                                          "ms_per_step": round(ms_step, 5), "kernel_ms": round(ms_kernel, 5),
                                          "roofline": roofline(op, prec, ms_kernel,
                                                               traffic_key="apply" if deg == 6 else None)}
            del op
    print(json.dumps({"metric": "DoFs/s per operator apply, CG P3, degree-4 (reduced) vs degree-6 cell rule",
                      "unit": "DoFs/s", "config": {"workload": f"CG P3 Poisson, {args.n}^3x6 Kuhn tets, lognormal(0,1) "
                                                                 "kappa per point of each rule"},
                      "variants": res,
                      "speedup_f64": round(res["degree4_f64"]["DoFs_per_s"] / res["degree6_f64"]["DoFs_per_s"], 3)}),
          flush=True)


def bench_f2(args):
    """Vector-valued Poisson (3 components without coupling, Sec. 3.2): one
    components-batched apply against three scalar applies of the same
    operator, CG P3 on the measured workload's mesh, straight-sided and
    curved cells, FP64 and FP32."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    xyz, tets, qp, qw, kap = build_workload(args.n)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25)
    mesh = tm.Mesh(xyz, tets)
    res = {}
    for geom in ("straight", "curved"):
        for prec in ("f64", "f32"):
            qj = jac if geom == "curved" else None
            opv = tm.Operator(mesh, 3, (qp, qw), precision=prec, q_jacobians=qj, n_components=3)
            kl = opv.cell_data_to_library(torch.from_numpy(kap).cuda())
            g = torch.Generator(device="cpu").manual_seed(2)
            u = (torch.rand(opv.n_vec, generator=g, dtype=torch.float64) * 2 - 1).to("cuda", opv.dtype)
            ms_v, k_v, _ = time_gpu(opv, kl, u, args.steps, args.warmup)
            rv = roofline(opv, prec, k_v)
            del opv
            ops = tm.Operator(mesh, 3, (qp, qw), precision=prec, q_jacobians=qj)
            n = ops.n_dofs
            outs = [torch.empty(n, dtype=ops.dtype, device="cuda") for _ in range(3)]

            def three():
                for c in range(3):
                    ops.apply(u[c * n:(c + 1) * n], kl, out=outs[c])
            ms_s = _time_call(three, args.steps, args.warmup)
            del ops
            res[f"{geom}_{prec}"] = {"DoFs_per_s": round(3 * n / (ms_v * 1e-3), 1), "ms_per_step": round(ms_v, 5),
                                     "kernel_ms": round(k_v, 5), "ms_three_scalar_applies": round(ms_s, 5),
                                     "speedup_vs_three_scalar": round(ms_s / ms_v, 3), "roofline": rv}
    print(json.dumps({"metric": "DoFs/s per vector operator apply (3 components), CG P3, components-batched",
                      "value": res["straight_f64"]["DoFs_per_s"], "unit": "DoFs/s", "dtype": "f64",
                      "config": {"workload": f"vector Poisson, 3 components, CG P3, {args.n}^3x6 Kuhn tets, "
                                             "lognormal(0,1) kappa, 24-point rule; curved: the f3 map"},
                      "variants": res}), flush=True)


def bench_f3(args):
    """Curved cells (a Jacobian per rule point, Sec. 3.2): the measured
    workload's mesh pushed through a smooth global map, CG P3 with the
    24-point rule, FP64 and FP32, next to the straight-sided operator."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    xyz, tets, qp, qw, kap = build_workload(args.n)
    jac = synth.curved_jacobians(xyz, tets, qp, 0.25)
    mesh = tm.Mesh(xyz, tets)
    res = {}
    for prec in ("f64", "f32"):
        for curved in (True, False):
            op = tm.Operator(mesh, 3, (qp, qw), precision=prec, q_jacobians=jac if curved else None)
            kl = op.cell_data_to_library(torch.from_numpy(kap).cuda())
            g = torch.Generator(device="cpu").manual_seed(2)
            u = (torch.rand(op.n_dofs, generator=g, dtype=torch.float64) * 2 - 1).to("cuda", op.dtype)
            ms_step, ms_kernel, _ = time_gpu(op, kl, u, args.steps, args.warmup)
            res[f"{'curved' if curved else 'straight'}_{prec}"] = {
                "DoFs_per_s": round(op.n_dofs / (ms_step * 1e-3), 1), "ms_per_step": round(ms_step, 5),
                "kernel_ms": round(ms_kernel, 5), "device_bytes": op.info["device_bytes"],
                "roofline": roofline(op, prec, ms_kernel, traffic_key="curved" if curved else "apply")}
            del op
    print(json.dumps({"metric": "DoFs/s per operator apply, CG P3 on curved cells (per-point Jacobians)",
                      "value": res["curved_f64"]["DoFs_per_s"], "unit": "DoFs/s", "dtype": "f64",
                      "config": {"workload": f"CG P3 Poisson, {args.n}^3x6 Kuhn tets mapped by "
                                             "(x + 0.25 y^2, y + 0.25 z^2, z + 0.25 x^2), lognormal(0,1) kappa, "
                                             "24-point rule"},
                      "variants": res}), flush=True)


def bench_f4(args):
    """Jacobi-preconditioned Chebyshev smoothing (degree 5, as in the
    multigrid of Sec. 4.1) on the solve workload, FP64 and FP32: time per
    smoother call and per step (one operator application plus the fused
    vector update), and the Lanczos estimate of lambda_max(D^-1 A)."""
    import torch

    import paper_2509_10226_amd as tm
    import synth
    n = args.n
    xyz, tets = synth.kuhn_cube_mesh(n, 0.15, 0)
    qp, qw = synth.tet_rule(6)
    mesh = tm.Mesh(xyz, tets)
    res = {}
    for prec in ("f64", "f32"):
        op = tm.Operator(mesh, 3, (qp, qw), bc="dirichlet", precision=prec)
        inv = 1.0 / op.diagonal()
        t0 = time.perf_counter()
        lam = op.estimate_lambda_max(inv, n_iter=20)
        t_est = time.perf_counter() - t0
        lmax = 1.1 * lam
        lmin = lmax / 15.0
        b = op.load_vector()
        x = torch.zeros_like(b)
        ms = _time_call(lambda: op.chebyshev(b, inv, 5, lmin, lmax, x=x), args.steps, args.warmup)
        u = torch.rand(op.n_dofs, dtype=op.dtype, device="cuda")
        ms_apply = _time_call(lambda: op.apply(u), args.steps, args.warmup)
        res[prec] = {"ms_per_smoothing": round(ms, 5), "steps": 5, "ms_per_step": round(ms / 5, 5),
                     "DoFs_per_s_per_step": round(op.n_dofs * 5 / (ms * 1e-3), 1),
                     "ms_per_apply": round(ms_apply, 5), "lambda_max_estimate": lam,
                     "estimate_seconds_20_steps": round(t_est, 4)}
        del op
    print(json.dumps({"metric": "DoFs/s per Chebyshev-Jacobi smoothing step, CG P3 (degree 5)", "unit": "DoFs/s",
                      "config": {"workload": f"CG P3 Poisson, Dirichlet, kappa=1, {n}^3x6 Kuhn tets, 24-point rule; "
                                             "interval [lambda_max/15, 1.1 lambda_max]"},
                      "variants": res}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64, help="cubes per axis (64 = the measured workload)")
    ap.add_argument("--precisions", default="f64,f32,bf16in")
    ap.add_argument("--config", default="c3", choices=["c3", "c2", "c4", "c5", "order", "f1", "f2", "f3", "f4"],
                    help="c3 (default): the measured workload; c2/c4/c5/order/f1/f2/f3/f4: secondary measurements, "
                         "each printed as its own JSON line")
    ap.add_argument("--order-variant", default="all",
                    choices=["all", "native_locality", "shuffled_locality", "shuffled_as_given"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the operator shards by "
              "cell partition with one halo exchange per apply, which this build does not run).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2509_10226_amd as tm
    if args.copy_calibration:
        copy_calibration()
        return
    if args.config != "c3":
        {"c2": bench_c2, "c4": bench_c4, "c5": bench_c5, "order": bench_order, "f1": bench_f1,
         "f2": bench_f2, "f3": bench_f3, "f4": bench_f4}[args.config](args)
        return
    dev = torch.device("cuda", 0)
    xyz, tets, qp, qw, kap = build_workload(args.n)
    t_setup = time.perf_counter()
    mesh = tm.Mesh(xyz, tets)
    results, outs = {}, {}
    for prec in args.precisions.split(","):
        op = tm.Operator(mesh, 3, (qp, qw), precision=prec)
        setup_s = time.perf_counter() - t_setup
        kl = op.cell_data_to_library(torch.from_numpy(kap).to(dev))
        g = torch.Generator(device="cpu").manual_seed(2)
        u = (torch.rand(op.n_dofs, generator=g, dtype=torch.float64) * 2 - 1).to(dev, op.dtype)
        ms_eager, ms_kernel, out = time_gpu(op, kl, u, args.steps, args.warmup)
        ms_graph = time_graph(op, kl, u, args.steps, args.warmup, out)
        ms_step = ms_graph if ms_graph is not None else ms_eager
        outs[prec] = out.double()
        results[prec] = {
            "value": op.n_dofs / (ms_step * 1e-3),
            "ms_per_step": ms_step,
            "ms_per_step_eager": ms_eager,
            "timing": "graph" if ms_graph is not None else "eager",
            "roofline": roofline(op, prec, ms_kernel, traffic_key="apply"),
            "n_dofs": op.n_dofs,
            "n_cell": op.n_cell,
            "setup_s": round(setup_s, 2),
            "blocks": op.info["n_blocks"],
            "shared_dofs": op.info["n_shared"],
            "partials": op.info["n_partials"],
        }
        del op
        t_setup = time.perf_counter()
    main_prec = "f64" if "f64" in results else next(iter(results))
    r = results[main_prec]
    line = {
        "metric": METRIC,
        "value": round(r["value"], 1),
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "ms_per_step_eager": round(r["ms_per_step_eager"], 5),
        "timing": (("one apply (cell kernel + combine) captured in a HIP graph and replayed; replays checked "
                    "bitwise against the eager result; ms_per_step_eager: the same calls launched one by one")
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
    }
    for prec, rr in results.items():
        if prec != main_prec:
            line[prec] = {"value": round(rr["value"], 1), "ms_per_step": round(rr["ms_per_step"], 5),
                          "ms_per_step_eager": round(rr["ms_per_step_eager"], 5), "timing": rr["timing"],
                          "roofline": rr["roofline"]}
            if "f64" in outs:
                # same input (rounded to the operand precision); the FP64
                # operator matches the oracle to 1e-12 (tests)
                ref = outs["f64"]
                line[prec]["rel_diff_vs_f64_operator"] = float(torch.linalg.norm(outs[prec] - ref) /
                                                               torch.linalg.norm(ref))
    line["setup_s"] = r["setup_s"]
    line["blocks"] = {"n_blocks": r["blocks"], "shared_dofs": r["shared_dofs"], "partials": r["partials"]}
    if not args.no_cpu_baseline and args.n == 64:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
