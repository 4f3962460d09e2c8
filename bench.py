#!/usr/bin/env python3
"""Benchmark: CGLS iterations/s (and A+A^T applies/s) on the 512x512 workload.

One step = one full CGLS solve on the GPU: r0 = y, s0 = A^T y, p0 = s0, then
50 iterations of (A p, ||q||^2, alpha, r update, A^T r with the x / s update,
||s||^2, beta, p update), captured once as a HIP graph and replayed.  Inputs
(y, geometry) are resident in HBM before timing starts.  The operator
throughputs (A, A^T and the A+A^T pair that one iteration contains) are timed
separately with HIP events on the stream the kernels run on.

The oracle (FP64 C on the host) runs only in the CPU-baseline leg at the end:
it is timed as the baseline, and every GPU result of the run is compared with
it there, on inputs generated from the seeded phantoms by the oracle itself.

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "A+A^T applies/s and CGLS iters/s, 512²×256 sensors; rel-L2 vs FP64 oracle"
WORKLOAD = ("512x512 image (0.05 mm pixels), ring of 256 sensors at 16 mm, 2048 samples at dt=12.5 ns, "
            "c=1500 m/s, 200-segment vessel tree, 1% noise, lambda=1e-3, 50 CGLS iterations, "
            "FP32 bulk with FP64 reductions")

# Algorithmic FP32 work of one (pixel, sensor) pair of the plain definition:
# difference vector (2), squared distance (3), clamp (1), sqrt (1),
# reciprocal (1), delay (2), floor and fraction (2), two weighted taps and the
# accumulation (6).  A fused multiply-add counts 2.
FLOP_PER_PAIR_2D = 18
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  The published FP32 vector
# peak (157.3 TFLOP/s) counts packed FP32 FMAs (2 per lane per clock); the
# build keeps packed FP32 off, so 78.6 TFLOP/s is the rate its code can issue.
VALU_LANES_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = VALU_LANES_PER_S * 2 / 1e12
COUNTERS = os.path.join(HERE, "profiles", "counters_512x512.json")
CSRC = os.path.join(HERE, "paper_2404_10928_amd", "csrc")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    for fn in ("pa_ops_dev.h", "pa_ops.hip", "pa_blas.hip", "pa_device.h"):
        with open(os.path.join(CSRC, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_summary():
    """The committed rocprofv3 counter summary of this workload's kernels, or
    None when the kernel sources changed since the counters were taken."""
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)
    except OSError:
        return None
    return rec if rec.get("kernel_sources_sha256") == kernel_sources_hash() else None


def gpu_clocks():
    """The current shader and memory clocks as rocm-smi reports them (empty when it is not there, or
    under a profiler, whose preloaded library would follow rocm-smi's own interpreter start)."""
    if "rocprof" in os.environ.get("LD_PRELOAD", "") or any(k.startswith("ROCPROF") for k in os.environ):
        return ""
    try:
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=15).stdout
    except (OSError, subprocess.SubprocessError):
        return ""
    keep = [ln.split(":", 2)[-1].strip() for ln in out.splitlines() if ("sclk" in ln or "mclk" in ln) and "GPU[" in ln]
    return "; ".join(keep)


def cpu_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        model = platform.processor()
    return {"nproc": os.cpu_count(), "model": model}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--op-reps", type=int, default=50, help="launches per operator timing")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (baseline and errors)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads for the baseline (the host share of one GPU); 1 is timed as well")
    ap.add_argument("--quick", action="store_true", help="CGLS steps only (profiling runs)")
    ap.add_argument("--no-extras", action="store_true", help="skip the legs beyond the 512x512 solve")
    ap.add_argument("--legs", default="all",
                    help="comma-separated extra legs: precisions, batched, volume, landweber, fista, dense, freq, "
                         "differentiable (default all)")
    ap.add_argument("--no-tune", action="store_true", help="plan by rule instead of running the autotuner")
    ap.add_argument("--tuning", default=None,
                    help="JSON tuning of the 512x512 workload to record instead of autotuning, e.g. "
                         "'{\"fwd_mode\": 3, \"fwd_tile\": [2, 2, 1], \"adj_lds_bytes\": 24576}' (profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=64,
                    help="size of a plain device copy run once (counter calibration for profiling runs)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        return 2

    import torch
    import paper_2404_10928_amd.ops as pa
    from synth import add_noise, make_config

    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        return 1
    dev = torch.device("cuda")
    w = make_config("C2")
    g = w.geom
    geom = pa.DeviceGeometry(g, dev)
    props = torch.cuda.get_device_properties(dev)
    gpu = {"name": props.name, "arch": getattr(props, "gcnArchName", ""), "cus": props.multi_processor_count,
           "clocks": gpu_clocks()}
    P, S, K = g.n_pixels, g.n_sensors, g.n_samples
    pairs = P * S

    # timing data: y = A x + 1% noise, generated on the GPU path itself
    x_true = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    y_clean = pa.forward(x_true, geom)
    torch.cuda.synchronize()
    y_np = add_noise(y_clean.double().cpu().numpy(), w.noise_rel, w.noise_seeds[0])
    y = torch.from_numpy(y_np.astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    log(f"workload ready: P={P} S={S} K={K}")
    if args.tuning:
        tuning = json.loads(args.tuning)
        pa.tuning_set(geom, tuning, torch.float32)
    else:
        tuning = pa.autotune(geom, torch.float32) if not args.no_tune else None
    log(f"tuning: {tuning}")

    # a plain copy of known size: HBM-counter calibration for profiling runs
    if args.calib_copy_mib > 0:
        a = torch.empty(args.calib_copy_mib * (1 << 18), dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ------------------------------------------------------------ CGLS steps
    solver = pa.CglsSolver(geom, torch.float32, w.iters, w.lam, graph=True, device=dev)
    x = torch.empty(g.image_shape, dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        solver.solve(y, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(y, x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    iters_per_s = w.iters * args.steps / (t1 - t0)
    log(f"CGLS: {ms_per_step:.3f} ms per {w.iters}-iteration solve, {iters_per_s:.1f} it/s")

    out = {
        "metric": METRIC, "value": iters_per_s, "unit": "CGLS iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded vessel-tree phantom, y = A x + 1% Gaussian noise)", "gpu": gpu,
        "config": {"workload": WORKLOAD, "image": [512, 512], "sensors": S, "samples": K,
                   "cgls_iterations": w.iters, "step": "one full CGLS solve (graph replay)",
                   "tuning": tuning},
    }
    if args.quick:
        print(json.dumps(out))
        return 0

    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        """Seconds per call from HIP events recorded on the stream the kernels run on."""
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    # -------------------------------------------------- operator timings
    xs = torch.rand(g.image_shape, dtype=torch.float32, device=dev)
    ys = torch.randn(g.data_shape, dtype=torch.float32, device=dev)
    yo = torch.empty_like(ys)
    xo = torch.empty_like(xs)
    op = pa.Operator(geom, torch.float32, dev)
    t_fwd = timed(lambda: op.forward_(xs, yo), args.op_reps)
    t_fwd_nows = timed(lambda: op.forward_no_workspace_(xs, yo), args.op_reps)
    t_adj = timed(lambda: op.adjoint_(ys, xo), args.op_reps)
    t_pair = timed(lambda: (op.forward_(xs, yo), op.adjoint_(yo, xo)), args.op_reps)
    fwd_method = "partial rows (two passes, workspace)" if tuning and tuning.get("fwd_mode") == 3 else \
        "sensor-major (one pass, no workspace)"
    out.update({
        "a_applies_per_s": 1.0 / t_fwd, "at_applies_per_s": 1.0 / t_adj, "a_plus_at_applies_per_s": 1.0 / t_pair,
        "us_per_apply": {"A": t_fwd * 1e6, "A_without_workspace": t_fwd_nows * 1e6, "AT": t_adj * 1e6,
                         "A+AT": t_pair * 1e6},
        "forward_method": fwd_method,
        "pairs_per_s": {"A": pairs / t_fwd, "AT": pairs / t_adj},
    })
    log(f"A {t_fwd * 1e6:.1f} us ({fwd_method}; {t_fwd_nows * 1e6:.1f} us without workspace), "
        f"A^T {t_adj * 1e6:.1f} us, A+A^T {t_pair * 1e6:.1f} us")

    # the roofline of the slower operator: plain VALU arithmetic
    if t_fwd >= t_adj:
        dom, t_dom, key = f"A ({fwd_method})", t_fwd, ("forward_two_pass" if "partial" in fwd_method else "forward")
    else:
        dom, t_dom, key = "A^T (bp_kernel)", t_adj, "adjoint"
    achieved = pairs * FLOP_PER_PAIR_2D / t_dom / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
            "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS, "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "work_per_launch": f"{pairs} pixel-sensor pairs x {FLOP_PER_PAIR_2D} FLOP"}
    cs = counter_summary()
    if cs is None:
        roof["traffic_note"] = "no counter summary for the current kernel sources"
    else:
        k = cs["per_apply"].get(key)
        if k:
            roof["traffic"] = k["hbm_bytes"]
            roof["hbm_GBps_at_measured_traffic"] = k["hbm_bytes"] / t_dom / 1e9
            roof["valu_instructions_per_pair"] = k["valu_per_pair"]
            # the pair rate the VALU can issue at that instruction count
            bound = VALU_LANES_PER_S / k["valu_per_pair"]
            roof["pair_rate_frac_of_valu_bound"] = (pairs / t_dom) / bound
            roof["valu_utilisation"] = k.get("valu_utilisation")
            roof["traffic_note"] = "FETCH_SIZE + WRITE_SIZE per apply, copy-calibrated (profiles/counters_512x512.json)"
    out["roofline"] = roof

    extras = {}
    if not args.no_extras:
        legs = set(args.legs.split(",")) if args.legs != "all" else None

        def want(name):
            return legs is None or name in legs
        if want("precisions"):
            out["precisions"] = precisions_leg(pa, torch, dev, geom, y, w)
        if want("batched"):
            out["batched_frames"] = batched_leg(pa, torch, dev, tune=not args.no_tune)
        if want("volume"):
            out["volume_3d"] = volume_leg(pa, torch, dev, tune=not args.no_tune)
        if want("landweber"):
            out["landweber"] = landweber_leg(pa, torch, dev, geom, y, w)
        if want("fista"):
            out["fista_l1_tv"] = fista_leg(pa, torch, dev, geom, y, w)
        if want("dense"):
            out["dense_matrix"] = dense_leg(pa, torch, dev)
        if want("freq"):
            out["frequency_domain"] = freq_leg(pa, torch, dev)
        if want("differentiable"):
            out["differentiable"] = autograd_leg(pa, torch, dev)
        extras = {k: v for k, v in out.items() if isinstance(v, dict) and "workload" in v}

    if not args.no_cpu_baseline:
        cpu_baseline_leg(pa, torch, dev, geom, w, args, out, extras)

    print(json.dumps(out))
    return 0


def _sync_time(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


# ------------------------------------------------------------------ legs
# Each leg times GPU work only; the oracle comparisons for it run in the
# CPU-baseline leg.

def precisions_leg(pa, torch, dev, geom, y32, w):
    """The 512x512 solve in PA_F64 and PA_MIXED (FP64 vectors around the
    FP32-arithmetic operator), and the 128x128 workload in PA_F64 (its
    configured precision), 50 and 20 iterations: CGLS iterations/s."""
    from synth import make_config
    res = {"workload": "512x512 ring solve (50 iterations) in PA_F64 and PA_MIXED; 128x128 ring solve "
                       "(20 iterations, 128 sensors, 512 samples) in PA_F64"}
    y64 = y32.double()
    for name, prec in (("c2_f64", None), ("c2_mixed", "mixed")):
        sv = pa.CglsSolver(geom, torch.float64, w.iters, w.lam, graph=True, device=dev, precision=prec)
        x = torch.empty(geom.image_shape, dtype=torch.float64, device=dev)
        sv.solve(y64, x)
        t = _sync_time(torch, lambda: sv.solve(y64, x), 3)
        res[name] = {"cgls_iterations_per_s": w.iters / t, "ms_per_solve": t * 1e3}
    w1 = make_config("C1")
    g1 = pa.DeviceGeometry(w1.geom, dev)
    x1 = torch.from_numpy(w1.x).to(dev)
    y1 = pa.forward(x1, g1)
    sv = pa.CglsSolver(g1, torch.float64, w1.iters, w1.lam, graph=True, device=dev)
    xo = torch.empty(g1.image_shape, dtype=torch.float64, device=dev)
    sv.solve(y1, xo)
    t = _sync_time(torch, lambda: sv.solve(y1, xo), 10)
    res["c1_f64"] = {"cgls_iterations_per_s": w1.iters / t, "ms_per_solve": t * 1e3}
    log(f"precisions: 512^2 f64 {res['c2_f64']['cgls_iterations_per_s']:.0f} it/s, "
        f"mixed {res['c2_mixed']['cgls_iterations_per_s']:.0f} it/s; 128^2 f64 {w1.iters / t:.0f} it/s")
    return res


def batched_leg(pa, torch, dev, tune=True):
    """64 uneven frames (images 128-512, 64-512 sensors, 512-2048 samples),
    50 CGLS iterations: one batched graph replay against 64 single-frame
    graph replays."""
    from synth import add_noise, make_config
    w = make_config("C4")
    geoms = [pa.DeviceGeometry(g, dev) for g in w.geoms]
    if tune:   # every frame shape (the single-frame plans use them), then the batch as a whole
        for g in geoms:
            pa.autotune(g, torch.float32)
    b = pa.Batch(geoms, torch.float32, dev)
    batch_tuned = b.autotune() if tune else False
    xp = b.pack_x([torch.from_numpy(x.astype(np.float32)).to(dev) for x in w.x_true])
    yc = b.unpack_y(b.forward(xp))
    ys = [torch.from_numpy(add_noise(y.double().cpu().numpy(), w.noise_rel, w.noise_seeds[i]).astype(np.float32)).to(dev)
          for i, y in enumerate(yc)]
    yp = b.pack_y(ys)
    xb = torch.empty(b.x_offsets[-1], dtype=torch.float32, device=dev)
    b.cgls(yp, w.iters, w.lam, xb)
    t_b = _sync_time(torch, lambda: b.cgls(yp, w.iters, w.lam, xb), 3)
    t_f = _sync_time(torch, lambda: b.forward(xp), 5)
    t_a = _sync_time(torch, lambda: b.adjoint(yp), 5)
    solvers = [pa.CglsSolver(g, torch.float32, w.iters, w.lam, graph=True, device=dev) for g in geoms]
    xs = [torch.empty(g.image_shape, dtype=torch.float32, device=dev) for g in geoms]

    def loop():
        for sv, yy, xx in zip(solvers, ys, xs):
            sv.solve(yy, xx)
    loop()
    t_s = _sync_time(torch, loop, 2)
    n = len(geoms)
    pairs = sum(g.n_pixels * g.n_sensors for g in geoms)
    log(f"batched {n} frames: {t_b * 1e3:.2f} ms per {w.iters}-iteration solve; single-frame loop "
        f"{t_s * 1e3:.2f} ms; batched A {t_f * 1e3:.2f} ms, A^T {t_a * 1e3:.2f} ms")
    return {"workload": f"{n} frames of 128-512 px square images, 64-512 sensors, 512-2048 samples, "
                        f"{w.iters} CGLS iterations, FP32", "pairs_per_apply": pairs,
            "frame_iterations_per_s_batched": n * w.iters / t_b,
            "frame_iterations_per_s_single_frame_loop": n * w.iters / t_s,
            "speedup": t_s / t_b,
            "ms_per_batched_apply": {"A": t_f * 1e3, "AT": t_a * 1e3},
            "pairs_per_s_batched": {"A": pairs / t_f, "AT": pairs / t_a},
            "batch_plans": "per-frame tuned" if batch_tuned else "planner rules (faster than the tuned set here)"}


def landweber_leg(pa, torch, dev, geom, y, w):
    """The gradient iteration on the 512x512 workload: 50 steps with the step
    size from 30 power-iteration steps, FP32, one graph replay per solve."""
    sv = pa.LandweberSolver(geom, torch.float32, w.iters, w.lam, omega=0.0, power_iters=30, graph=True, device=dev)
    x = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
    sv.solve(y, x)
    t = _sync_time(torch, lambda: sv.solve(y, x), 3)
    om, s2 = sv.step()
    return {"workload": f"512x512 ring workload, {w.iters} Landweber steps + 30 power-iteration steps, FP32",
            "ms_per_solve": t * 1e3, "solves_per_s": 1.0 / t, "sigma2": s2, "omega": om}


def fista_weights(adj_y_absmax):
    b = adj_y_absmax * 2.0
    return 1e-2 * b, 1e-4 * b, 1e-2


def fista_leg(pa, torch, dev, geom, y, w):
    """The l1 + TV objective of Eq. 8 on the 512x512 workload: 50 FISTA steps
    with the step from 30 power-iteration steps, x >= 0, FP32, one graph replay
    per solve.  Weights from the data: alpha = 1e-2 max|2 A^T y|,
    beta = 1e-4 max|2 A^T y|, eps = 1e-2."""
    alpha, beta, eps = fista_weights(float(pa.adjoint(y, geom).abs().max()))
    sv = pa.FistaSolver(geom, torch.float32, w.iters, w.lam, alpha, beta, eps, omega=0.0, power_iters=30,
                        nonneg=True, graph=True, device=dev)
    x = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
    sv.solve(y, x)
    t = _sync_time(torch, lambda: sv.solve(y, x), 3)
    om, s2 = sv.step()
    return {"workload": f"512x512 ring workload, {w.iters} FISTA steps + 30 power-iteration steps, "
                        f"l1 + TV (alpha {alpha:.3e}, beta {beta:.3e}, eps {eps}), x >= 0, FP32",
            "ms_per_solve": t * 1e3, "solves_per_s": 1.0 / t, "sigma2": s2, "omega": om,
            "zero_fraction": float((x == 0).double().mean())}


def table4_geometry():
    """The paper's dense shape (Table 4: 6144 measurements by 16384 pixels):
    a 128x128 image (0.1 mm) with 12 ring sensors at 10 mm and 512 samples at
    25 ns."""
    from synth import Geometry, ring_sensors
    return Geometry(2, 128, 128, 1, 1e-4, (0.0, 0.0, 0.0), ring_sensors(12, 10e-3), 512, 25e-9)


def dense_leg(pa, torch, dev):
    """The paper's own formulation: the dense FP64 matrix built on the GPU and
    applied as y = A x and x = A^T y, each reading the whole matrix from HBM;
    at Table 4's shape (6144 x 16384) and at the 128x128 ring workload
    (65536 x 16384), next to the matrix-free FP64 operators."""
    from synth import make_config
    res = {"workload": "dense FP64 matrix (the paper's kn layout, rows (sensor, sample), columns pixels): "
                       "Table 4's 6144 x 16384 and the 128x128 ring workload's 65536 x 16384"}
    stream = torch.cuda.current_stream(dev)

    def ev(fn, reps):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    for name, g0, x_np in (("table4_6144x16384", table4_geometry(), None),
                           ("ring_65536x16384", make_config("C1").geom, make_config("C1").x)):
        g = pa.DeviceGeometry(g0, dev)
        D = pa.DenseMatrix(g, torch.float64, dev)
        x = torch.from_numpy(x_np if x_np is not None else make_config("C1").x).to(dev)
        yv = torch.randn(g.data_shape, dtype=torch.float64, device=dev)
        yo = torch.empty_like(yv)
        xo = torch.empty_like(x)
        t_f = ev(lambda: D.forward(x, yo), 10)
        t_a = ev(lambda: D.adjoint(yv, xo), 10)
        op = pa.Operator(g, torch.float64, dev)
        t_mf = ev(lambda: op.forward_(x, yo), 50)
        t_ma = ev(lambda: op.adjoint_(yv, xo), 50)
        nbytes = D.matrix.numel()
        res[name] = {"rows": g.n_sensors * g.n_samples, "cols": g.n_pixels, "matrix_bytes": nbytes,
                     "us_per_apply": {"dense A": t_f * 1e6, "dense A^T": t_a * 1e6,
                                      "matrix-free A (FP64)": t_mf * 1e6, "matrix-free A^T (FP64)": t_ma * 1e6},
                     "roofline": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0,
                                  "achieved_A": nbytes / t_f / 1e9, "achieved_AT": nbytes / t_a / 1e9,
                                  "frac_A": nbytes / t_f / 8e12, "frac_AT": nbytes / t_a / 8e12,
                                  "bytes_per_launch": "the matrix once (x, y and the A^T partials are < 1 %)"}}
        log(f"dense {name}: A {t_f * 1e6:.0f} us ({nbytes / t_f / 1e9:.0f} GB/s), A^T {t_a * 1e6:.0f} us "
            f"({nbytes / t_a / 1e9:.0f} GB/s); matrix-free {t_mf * 1e6:.1f} / {t_ma * 1e6:.1f} us")
        del D
        torch.cuda.empty_cache()
    return res


def freq_setup(make_config):
    w = make_config("C1")
    g = w.geom
    nf = g.n_samples // 2
    df = 1.0 / (g.n_samples * g.dt)
    return w, g, nf, df


def freq_leg(pa, torch, dev):
    """The frequency-domain matrix of Eq. 7 on the 128x128 workload, at the
    DFT bins of its traces (f_n = (n + 1) / (K dt), 256 bins up to 20 MHz):
    Y = K x and x = Re(K^H Y), FP32 with FP64 phases and sums."""
    from synth import make_config
    w, g0, nf, df = freq_setup(make_config)
    g = pa.DeviceGeometry(g0, dev)
    op = pa.FreqOperator(g, df, df, nf, torch.float32, dev)
    x = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    Y = op.forward(x)
    xo = torch.empty_like(x)
    t_f = _sync_time(torch, lambda: op.forward(x, Y), 10)
    t_a = _sync_time(torch, lambda: op.adjoint(Y, xo), 10)
    terms = g.n_pixels * g.n_sensors * nf
    log(f"frequency domain 128^2 x 128 x {nf}: K {t_f * 1e6:.0f} us, K^H {t_a * 1e6:.0f} us")
    return {"workload": f"128x128 image, 128 sensors, {nf} frequencies f_n = (n+1)/(K dt), FP32",
            "terms_per_apply": terms, "us_per_apply": {"K": t_f * 1e6, "K^H": t_a * 1e6},
            "terms_per_s": {"K": terms / t_f, "K^H": terms / t_a}}


def autograd_leg(pa, torch, dev):
    """Loss ||A x - y||^2 + 1e-3 TV(x) over 16 images of 256x256 (128-sensor
    ring, 1024 samples), forward and backward through the autograd wrapper:
    one batched launch per operator pass."""
    import paper_2404_10928_amd.autograd as ag
    from synth import make_config
    w = make_config("C3")
    g = pa.DeviceGeometry(w.geom, dev)
    X = torch.from_numpy(np.stack(w.x_true).astype(np.float32)).to(dev).requires_grad_(True)
    Y = torch.zeros((len(w.x_true),) + g.data_shape, dtype=torch.float32, device=dev)
    with torch.no_grad():
        Y.copy_(ag.PAForward.apply(X, g))

    def step():
        X.grad = None
        loss = ag.data_term(X * 0.9, Y, g) + 1e-3 * ag.tv(X)
        loss.backward()

    step()
    t = _sync_time(torch, step, 5)
    return {"workload": "16 images of 256x256, 128-sensor ring, 1024 samples; loss ||Ax - y||^2 + 1e-3 TV(x), FP32",
            "ms_per_forward_backward": t * 1e3, "images_per_s": len(w.x_true) / t}


def volume_leg(pa, torch, dev, tune=True):
    """128^3 voxels, 1024-sensor hemisphere, 2048 samples, 30 CGLS iterations
    in PA_F32, PA_MIXED and PA_F64, timed."""
    from synth import add_noise, make_config
    w = make_config("C5")
    g = pa.DeviceGeometry(w.geom, dev)
    x_true = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    y32 = torch.from_numpy(add_noise(pa.forward(x_true, g).double().cpu().numpy(), w.noise_rel,
                                     w.noise_seeds[0]).astype(np.float32)).to(dev)
    res = {"workload": "128^3 voxels (0.1 mm), 1024-sensor Fibonacci hemisphere at 20 mm, 2048 samples at 20 ns, "
                       f"{w.iters} CGLS iterations"}
    for name, dt, prec in (("f32", torch.float32, None), ("mixed", torch.float64, "mixed"),
                           ("f64", torch.float64, None)):
        if tune:
            res[f"tuning_{name}"] = pa.autotune(g, dt, precision=prec)
        sv = pa.CglsSolver(g, dt, w.iters, w.lam, graph=True, device=dev, precision=prec)
        y = y32.to(dt)
        x = torch.empty(g.image_shape, dtype=dt, device=dev)
        sv.solve(y, x)
        t = _sync_time(torch, lambda: sv.solve(y, x), 2)
        op = pa.Operator(g, dt, dev, precision=prec)
        yo = torch.empty_like(y)
        xo = torch.empty_like(x)
        t_a = _sync_time(torch, lambda: op.forward_(x, yo), 5)
        t_at = _sync_time(torch, lambda: op.adjoint_(y, xo), 5)
        res[name] = {"cgls_iterations_per_s": w.iters / t, "us_per_A": t_a * 1e6, "us_per_AT": t_at * 1e6}
    log(f"3D: f32 {res['f32']['cgls_iterations_per_s']:.1f} it/s, mixed {res['mixed']['cgls_iterations_per_s']:.1f}, "
        f"f64 {res['f64']['cgls_iterations_per_s']:.1f} it/s")
    return res


# ------------------------------------------------------- CPU baseline leg

def cpu_baseline_leg(pa, torch, dev, geom, w, args, out, extras):
    """The FP64 oracle on the host: timed on the 512x512 solve (the baseline),
    and every GPU result above compared with it on inputs the oracle
    generates from the seeded phantoms."""
    import oracle
    from synth import add_noise, make_config
    threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
    g = w.geom
    errs = {}

    # the 512x512 solve: data from the oracle, then the oracle's own 50-iteration
    # CGLS (timed: the baseline) against the GPU solves of the same data
    y_o = add_noise(oracle.forward(g, w.x, threads=threads), w.noise_rel, w.noise_seeds[0])
    y32 = y_o.astype(np.float32)
    y64 = y32.astype(np.float64)
    ta = time.perf_counter()
    x_ref, h_ref, _ = oracle.cgls(g, y64, w.iters, w.lam, threads=threads)
    tb = time.perf_counter()
    it1 = 3
    oracle.cgls(g, y64, it1, w.lam, threads=1)
    tc = time.perf_counter()
    info = cpu_info()
    out["cpu_baseline"] = {
        "value": w.iters / (tb - ta), "unit": "CGLS iterations/s", "cores": threads, "kind": "oracle",
        "sample": f"FP64 C oracle, the whole 50-iteration CGLS of the 512x512 workload ({tb - ta:.1f} s on "
                  f"{threads} threads); 1 thread: {it1} iterations in {tc - tb:.1f} s",
        "one_thread_value": it1 / (tc - tb), "host": info}
    log(f"oracle CGLS: {w.iters / (tb - ta):.2f} it/s on {threads} threads, {it1 / (tc - tb):.3f} it/s on 1 "
        f"({info['model']}, nproc {info['nproc']})")

    def solve_err(x_gpu, h_gpu, xr, hr):
        return {"iterate_rel_l2": float(np.linalg.norm(x_gpu - xr) / np.linalg.norm(xr)),
                "final_F_rel": float(abs(h_gpu[-1, 2] / hr[-1, 2] - 1)),
                "final_r_rel": float(abs(h_gpu[-1, 0] / hr[-1, 0] - 1)),
                "max_F_rel_over_k": float(np.max(np.abs(h_gpu[:, 2] / hr[:, 2] - 1)))}

    dev_y32 = torch.from_numpy(y32).to(dev)
    sv = pa.CglsSolver(geom, torch.float32, w.iters, w.lam, graph=True, device=dev)
    xg = sv.solve(dev_y32)
    errs["cgls_512_f32"] = solve_err(xg.double().cpu().numpy(), sv.history.cpu().numpy(), x_ref, h_ref)
    if "precisions" in extras or "precisions" in out:
        for name, prec in (("cgls_512_f64", None), ("cgls_512_mixed", "mixed")):
            s2 = pa.CglsSolver(geom, torch.float64, w.iters, w.lam, graph=True, device=dev, precision=prec)
            xg = s2.solve(torch.from_numpy(y64).to(dev))
            errs[name] = solve_err(xg.cpu().numpy(), s2.history.cpu().numpy(), x_ref, h_ref)
        w1 = make_config("C1")
        y1 = add_noise(oracle.forward(w1.geom, w1.x, threads=threads), w1.noise_rel, w1.noise_seeds[0])
        xr1, hr1, _ = oracle.cgls(w1.geom, y1, w1.iters, w1.lam, threads=threads)
        x1, h1, _ = pa.cgls(torch.from_numpy(y1).to(dev), w1.geom, w1.iters, w1.lam)
        errs["cgls_128_f64"] = solve_err(x1.cpu().numpy(), h1.cpu().numpy(), xr1, hr1)
        errs["cgls_128_f64"]["oracle_band"] = oracle_band("c1")

    # per-apply errors on random inputs, both forward methods
    rng = np.random.default_rng([2002, 77])
    xv = rng.uniform(size=g.image_shape).astype(np.float32)
    yv = rng.normal(size=g.data_shape).astype(np.float32)
    yref = oracle.forward(g, xv.astype(np.float64), threads=threads)
    xref = oracle.adjoint(g, yv.astype(np.float64), threads=threads)
    op = pa.Operator(geom, torch.float32, dev)
    xt, yt = torch.from_numpy(xv).to(dev), torch.from_numpy(yv).to(dev)
    ya, yb, xa = torch.empty_like(yt), torch.empty_like(yt), torch.empty_like(xt)
    op.forward_(xt, ya)
    op.forward_no_workspace_(xt, yb)
    op.adjoint_(yt, xa)
    rel = lambda a, r: float(np.linalg.norm(a.double().cpu().numpy() - r) / np.linalg.norm(r))  # noqa: E731
    errs["apply_512_f32"] = {"A": rel(ya, yref), "A_without_workspace": rel(yb, yref), "AT": rel(xa, xref)}

    if "batched_frames" in extras:
        errs["batched_frames"] = batched_errors(pa, torch, dev, oracle, threads)
    if "volume_3d" in extras:
        errs["volume_3d"] = volume_errors(pa, torch, dev, oracle, threads)
    if "landweber" in extras:
        om = extras["landweber"]["omega"]
        xl, hl = oracle.landweber(g, y64, w.iters, w.lam, om, threads=threads)
        lw = pa.LandweberSolver(geom, torch.float32, w.iters, w.lam, omega=om, power_iters=0, graph=True, device=dev)
        xg = lw.solve(dev_y32)
        errs["landweber"] = {"iterate_rel_l2": float(np.linalg.norm(xg.double().cpu().numpy() - xl) / np.linalg.norm(xl)),
                             "max_F_rel_over_k": float(np.max(np.abs(lw.history.cpu().numpy() / hl - 1))),
                             "sigma2_rel": float(abs(extras["landweber"]["sigma2"] / oracle.power_sigma2(g, 30, threads=threads) - 1))}
    if "fista_l1_tv" in extras:
        alpha, beta, eps = fista_weights(float(np.abs(oracle.adjoint(g, y64, threads=threads)).max()))
        om = extras["fista_l1_tv"]["omega"]
        xf, hf, _ = oracle.fista(g, y64, w.iters, w.lam, alpha, beta, eps, om, nonneg=True, threads=threads)
        fs = pa.FistaSolver(geom, torch.float32, w.iters, w.lam, alpha, beta, eps, omega=om, power_iters=0,
                            nonneg=True, graph=True, device=dev)
        xg = fs.solve(dev_y32)
        errs["fista_l1_tv"] = {"iterate_rel_l2": float(np.linalg.norm(xg.double().cpu().numpy() - xf) / np.linalg.norm(xf)),
                               "max_F_rel_over_k": float(np.max(np.abs(fs.history.cpu().numpy() / hf - 1)))}
    if "dense_matrix" in extras:
        errs["dense_matrix"] = dense_errors(pa, torch, dev, oracle, threads)
    if "frequency_domain" in extras:
        errs["frequency_domain"] = freq_errors(pa, torch, dev, oracle, threads)
    if "differentiable" in extras:
        errs["differentiable"] = autograd_errors(pa, torch, dev, oracle, threads)
    out["rel_err_vs_fp64_oracle"] = errs
    log(f"errors vs oracle: {json.dumps(errs)}")


def batched_errors(pa, torch, dev, oracle, threads):
    """Three frames of the uneven batch (128^2, 256^2, 512^2), 50-iteration
    batched FP32 solve on oracle data, against the oracle's solves."""
    from synth import add_noise, make_config
    w = make_config("C4")
    frames = (58, 10, 7)
    geoms = [pa.DeviceGeometry(g, dev) for g in w.geoms]
    b = pa.Batch(geoms, torch.float32, dev)
    ys = [np.zeros(g.data_shape, dtype=np.float32) for g in w.geoms]
    refs = {}
    for i in frames:
        yo = add_noise(oracle.forward(w.geoms[i], w.x_true[i], threads=threads), w.noise_rel, w.noise_seeds[i])
        ys[i] = yo.astype(np.float32)
        refs[i] = oracle.cgls(w.geoms[i], ys[i].astype(np.float64), w.iters, w.lam, threads=threads)
    x = b.cgls(b.pack_y([torch.from_numpy(y).to(dev) for y in ys]), w.iters, w.lam)
    xs = b.unpack_x(x)
    hist = b.history.cpu().numpy()
    res = {}
    for i in frames:
        xr, hr, _ = refs[i]
        g = w.geoms[i]
        res[f"frame{i}_{g.nx}px_{g.n_sensors}s"] = {
            "iterate_rel_l2": float(np.linalg.norm(xs[i].double().cpu().numpy() - xr) / np.linalg.norm(xr)),
            "final_F_rel": float(abs(hist[i, -1, 2] / hr[-1, 2] - 1)),
            "final_r_rel": float(abs(hist[i, -1, 0] / hr[-1, 0] - 1)),
            "oracle_band": oracle_band(f"c4_{i}")}
    return res


def oracle_band(case):
    """How far the oracle's own solve of a case moves when every operator
    application is perturbed by a relative 1e-13 (f64) or 1e-6 (f32: FP32
    delays), largest over three seeds (tests/golden/solve_spread.json)."""
    try:
        with open(os.path.join(HERE, "tests", "golden", "solve_spread.json")) as f:
            b = json.load(f)[case]
    except (OSError, KeyError):
        return None
    out = {}
    for prec in ("f64", "f32"):
        out[prec] = {"eps": b[prec]["eps"], "F_final_rel": b[prec]["F_rel_by_k"][-1],
                     "iterate_rel_l2": b[prec]["x_rel_l2"]}
        if "x_sample_rel_l2" in b[prec]:
            out[prec]["x_sample_rel_l2"] = b[prec]["x_sample_rel_l2"]
    return out


def volume_errors(pa, torch, dev, oracle, threads):
    """The 128^3 solves on the oracle's data, against the oracle's solve stored
    in tests/golden (F_30, x_30 at 4096 voxels) and its measured spread."""
    sys.path.insert(0, os.path.join(HERE, "tests", "golden"))
    from make_c5_reference import c5_data
    with open(os.path.join(HERE, "tests", "golden", "c5_cgls_reference.json")) as f:
        ref = json.load(f)
    w, g, y = c5_data(threads=threads)
    h_ref = np.array(ref["history"])
    idx = np.array(ref["sample_index"])
    res = {"oracle_band": oracle_band("c5")}
    for name, dt, prec in (("f32", torch.float32, None), ("mixed", torch.float64, "mixed"),
                           ("f64", torch.float64, None)):
        x, h, _ = pa.cgls(torch.from_numpy(y).to(dev, dt), g, w.iters, w.lam, precision=prec)
        xs = x.double().cpu().numpy().reshape(-1)[idx]
        h = h.cpu().numpy()
        res[name] = {"final_F_rel": float(abs(h[-1, 2] / h_ref[-1, 2] - 1)),
                     "x_sample_rel_l2": float(np.linalg.norm(xs - ref["x_sample"]) / np.linalg.norm(ref["x_sample"]))}
    return res


def dense_errors(pa, torch, dev, oracle, threads):
    from synth import make_config
    res = {}
    for name, g0 in (("table4_6144x16384", table4_geometry()), ("ring_65536x16384", make_config("C1").geom)):
        g = pa.DeviceGeometry(g0, dev)
        D = pa.DenseMatrix(g, torch.float64, dev)
        rng = np.random.default_rng([1001, 7])
        xv = rng.uniform(size=g0.image_shape)
        yv = rng.normal(size=g0.data_shape)
        yd = D.forward(torch.from_numpy(xv).to(dev)).cpu().numpy()
        xd = D.adjoint(torch.from_numpy(yv).to(dev)).cpu().numpy()
        yr = oracle.forward(g0, xv, threads=threads)
        xr = oracle.adjoint(g0, yv, threads=threads)
        res[name] = {"A": float(np.linalg.norm(yd - yr) / np.linalg.norm(yr)),
                     "AT": float(np.linalg.norm(xd - xr) / np.linalg.norm(xr))}
        del D
        torch.cuda.empty_cache()
    return res


def freq_errors(pa, torch, dev, oracle, threads):
    from synth import make_config
    w, g0, nf, df = freq_setup(make_config)
    op = pa.FreqOperator(pa.DeviceGeometry(g0, dev), df, df, nf, torch.float32, dev)
    x32 = w.x.astype(np.float32)
    Y = op.forward(torch.from_numpy(x32).to(dev)).double().cpu().numpy()
    Yg = Y[..., 0] + 1j * Y[..., 1]
    Yr = oracle.freq_forward(g0, x32.astype(np.float64), df, df, nf, threads=threads)
    Yin = np.random.default_rng([1001, 8]).normal(size=(g0.n_sensors, nf, 2)).astype(np.float32)
    xg = op.adjoint(torch.from_numpy(Yin).to(dev)).double().cpu().numpy()
    xr = oracle.freq_adjoint(g0, Yin[..., 0].astype(np.float64) + 1j * Yin[..., 1].astype(np.float64), df, df, nf,
                             threads=threads)
    return {"K": float(np.linalg.norm(Yg - Yr) / np.linalg.norm(Yr)),
            "K^H": float(np.linalg.norm(xg - xr) / np.linalg.norm(xr))}


def autograd_errors(pa, torch, dev, oracle, threads):
    """The FP32 gradient of ||A x - y||^2 + 1e-3 TV(x) through the autograd
    wrapper against the FP64 oracle gradient, on one image of the
    differentiable workload."""
    import paper_2404_10928_amd.autograd as ag
    from synth import make_config
    w = make_config("C3")
    g0 = w.geom
    rng = np.random.default_rng([3003, 999])
    x = rng.uniform(size=g0.image_shape).astype(np.float32)
    y = oracle.forward(g0, w.x_true[0], threads=threads).astype(np.float32)
    _, grad_ref = oracle.loss_gradient(g0, x.astype(np.float64), y.astype(np.float64), 1e-3, threads=threads)
    g = pa.DeviceGeometry(g0, dev)
    X = torch.from_numpy(x).to(dev).requires_grad_(True)
    loss = ag.data_term(X, torch.from_numpy(y).to(dev), g) + 1e-3 * ag.tv(X)
    loss.backward()
    gg = X.grad.double().cpu().numpy()
    return {"gradient_rel_l2": float(np.linalg.norm(gg - grad_ref) / np.linalg.norm(grad_ref))}


if __name__ == "__main__":
    sys.exit(main())
