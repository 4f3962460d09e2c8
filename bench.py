#!/usr/bin/env python3
"""Benchmark: CGLS iterations/s (and A+A^T applies/s) on the 512x512 workload.

One step = one full CGLS solve on the GPU: r0 = y, s0 = A^T y, p0 = s0, then
50 iterations of (A p, ||q||^2, alpha, r update, A^T r with the x / s update,
||s||^2, beta, p update), captured once as a HIP graph and replayed.  Inputs
(y, geometry) are resident in HBM before timing starts.  The operator
throughputs (A, A^T and the A+A^T pair that one iteration contains) are timed
separately with HIP events on the same stream.

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
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
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 FLOP per FMA, without packed FP32
# (the build disables packed FP32 instructions).
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12


def measured_traffic(which: str):
    """HBM bytes per apply from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, or None when the operator kernels changed since it was taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", "traffic_512x512.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None, "no counter summary"
    h = hashlib.sha256()
    for fn in ("pa_ops_dev.h", "pa_ops.hip"):
        with open(os.path.join(HERE, "paper_2404_10928_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("kernel_sources_sha256"):
        return None, "kernels changed since the counters were taken"
    k = rec["per_launch_averages"]
    if which == "forward":
        return rec["forward_operator_hbm_bytes"], "FETCH_SIZE + WRITE_SIZE of both launches, copy-calibrated"
    return k["bp_kernel_cg"]["hbm_bytes"], "FETCH_SIZE + WRITE_SIZE, copy-calibrated (CG-epilogue instance)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--op-reps", type=int, default=50, help="launches per operator timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=4, help="oracle CGLS iterations timed on the host")
    ap.add_argument("--quick", action="store_true", help="skip operator and CPU legs (profiling runs)")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched-frames and 3D legs")
    ap.add_argument("--legs", default="all",
                    help="comma-separated extra legs to run: batched, volume, landweber, fista, dense, freq, "
                         "differentiable (default all)")
    ap.add_argument("--no-tune", action="store_true", help="plan by rule instead of running the autotuner")
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
    P, S, K = g.n_pixels, g.n_sensors, g.n_samples
    pairs = P * S

    # synthetic data: y = A x_true + 1% noise, generated on the GPU path itself
    x_true = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    y_clean = pa.forward(x_true, geom)
    torch.cuda.synchronize()
    y_np = add_noise(y_clean.double().cpu().numpy(), w.noise_rel, w.noise_seeds[0])
    y = torch.from_numpy(y_np.astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    print(f"[bench] workload ready: P={P} S={S} K={K}", file=sys.stderr, flush=True)
    # tilings for this shape from the autotuner (recorded for every later plan)
    tuning = pa.autotune(geom, torch.float32) if not args.no_tune else None
    print(f"[bench] tuning: {tuning}", file=sys.stderr, flush=True)

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
    hist_gpu = solver.history.cpu().numpy()
    print(f"[bench] CGLS: {ms_per_step:.3f} ms per {w.iters}-iteration solve, {iters_per_s:.1f} it/s",
          file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": iters_per_s, "unit": "CGLS iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded vessel-tree phantom, y = A x + 1% Gaussian noise)",
        "config": {"workload": WORKLOAD, "image": [512, 512], "sensors": S, "samples": K,
                   "cgls_iterations": w.iters, "step": "one full CGLS solve (graph replay)",
                   "tuning": tuning},
    }

    if not args.quick:
        # -------------------------------------------------- operator timings
        stream = torch.cuda.current_stream(dev)
        xs = torch.rand(g.image_shape, dtype=torch.float32, device=dev)
        ys = torch.randn(g.data_shape, dtype=torch.float32, device=dev)
        yo = torch.empty_like(ys)
        xo = torch.empty_like(xs)

        def timed(fn, reps):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps * 1e-3   # seconds per call

        op = pa.Operator(geom, torch.float32, dev)
        t_fwd = timed(lambda: op.forward_(xs, yo), args.op_reps)
        t_adj = timed(lambda: op.adjoint_(ys, xo), args.op_reps)
        t_pair = timed(lambda: (op.forward_(xs, yo), op.adjoint_(yo, xo)), args.op_reps)
        out.update({
            "a_applies_per_s": 1.0 / t_fwd, "at_applies_per_s": 1.0 / t_adj,
            "a_plus_at_applies_per_s": 1.0 / t_pair,
            "us_per_apply": {"A": t_fwd * 1e6, "AT": t_adj * 1e6, "A+AT": t_pair * 1e6},
            "pairs_per_s": {"A": pairs / t_fwd, "AT": pairs / t_adj},
        })
        # The dominant kernel of a CGLS iteration: the slower of the two
        # operators.  The forward operator is two launches per apply (the
        # per-sensor histogram scatter and the gather of its partial rows);
        # the adjoint is one.
        if t_fwd > t_adj:
            dom, t_dom, tkey = "A (fp_kernel + fp_gather_kernel, two launches per apply)", t_fwd, "forward"
        else:
            dom, t_dom, tkey = "A^T (bp_kernel)", t_adj, "adjoint"
        achieved = pairs * FLOP_PER_PAIR_2D / t_dom / 1e12
        traffic, traffic_note = measured_traffic(tkey)
        out["roofline"] = {
            "bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
            "work_per_launch": f"{pairs} pixel-sensor pairs x {FLOP_PER_PAIR_2D} FLOP",
            "traffic_note": traffic_note,
        }
        if traffic:
            out["roofline"]["hbm_GBps_at_measured_traffic"] = traffic / t_dom / 1e9
        print(f"[bench] A {t_fwd*1e6:.1f} us, A^T {t_adj*1e6:.1f} us, A+A^T {t_pair*1e6:.1f} us",
              file=sys.stderr, flush=True)

        # ------------------------------------------ parity of this run's applies
        if not args.no_cpu_baseline:
            import oracle
            threads = min(16, os.cpu_count() or 1)
            xs64 = xs.double().cpu().numpy()
            ys64 = ys.double().cpu().numpy()
            op.forward_(xs, yo)
            op.adjoint_(ys, xo)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            yref = oracle.forward(g, xs64, threads=threads)
            tb = time.perf_counter()
            xref = oracle.adjoint(g, ys64, threads=threads)
            tc = time.perf_counter()
            e_a = float(np.linalg.norm(yo.double().cpu().numpy() - yref) / np.linalg.norm(yref))
            e_at = float(np.linalg.norm(xo.double().cpu().numpy() - xref) / np.linalg.norm(xref))
            # the oracle's own CGLS on the same y (FP64 value of the FP32 data), a bounded sample
            it = args.cpu_iters
            td = time.perf_counter()
            _, hist_ref, _ = oracle.cgls(g, y.double().cpu().numpy(), it, w.lam, threads=threads)
            te = time.perf_counter()
            eF = float(np.max(np.abs(hist_gpu[: it + 1, 2] / hist_ref[:, 2] - 1)))
            eR = float(np.max(np.abs(hist_gpu[: it + 1, 0] / hist_ref[:, 0] - 1)))
            out["rel_l2_vs_fp64_oracle"] = {"A": e_a, "AT": e_at,
                                            f"cgls_F_k_max_rel_k<={it}": eF, f"cgls_r_k_max_rel_k<={it}": eR}
            out["cpu_baseline"] = {
                "value": it / (te - td), "unit": "CGLS iterations/s", "cores": threads, "kind": "oracle",
                "sample": f"FP64 C oracle CGLS, {it} iterations of the same 512x512x256x2048 problem "
                          f"({te - td:.1f} s); A apply {tb - ta:.2f} s, A^T apply {tc - tb:.2f} s",
                "a_plus_at_applies_per_s": 1.0 / ((tb - ta) + (tc - tb)),
            }
            print(f"[bench] parity A {e_a:.2e} A^T {e_at:.2e}; oracle {it} its in {te - td:.1f} s",
                  file=sys.stderr, flush=True)

    if not args.quick and not args.no_extras:
        legs = set(args.legs.split(",")) if args.legs != "all" else None
        def want(name):
            return legs is None or name in legs
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

    print(json.dumps(out))
    return 0


def _sync_time(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def batched_leg(pa, torch, dev, tune=True):
    """64 uneven frames (images 128-512, 64-512 sensors, 512-2048 samples),
    50 CGLS iterations: one batched graph replay against 64 single-frame
    graph replays, with the largest per-frame iterate difference."""
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
    solvers = [pa.CglsSolver(g, torch.float32, w.iters, w.lam, graph=True, device=dev) for g in geoms]
    xs = [torch.empty(g.image_shape, dtype=torch.float32, device=dev) for g in geoms]
    def loop():
        for sv, y, x in zip(solvers, ys, xs):
            sv.solve(y, x)
    loop()
    t_s = _sync_time(torch, loop, 2)
    diffs = [float(torch.linalg.norm((a.reshape(-1) - c.reshape(-1)).double()) / max(float(torch.linalg.norm(c.double())), 1e-300))
             for a, c in zip(b.unpack_x(xb), xs)]
    n = len(geoms)
    pairs = sum(g.n_pixels * g.n_sensors for g in geoms)
    print(f"[bench] batched {n} frames: {t_b * 1e3:.2f} ms per {w.iters}-iteration solve; "
          f"single-frame loop {t_s * 1e3:.2f} ms", file=sys.stderr, flush=True)
    return {"workload": f"{n} frames of 128-512 px square images, 64-512 sensors, 512-2048 samples, "
                        f"{w.iters} CGLS iterations, FP32", "pairs_per_apply": pairs,
            "frame_iterations_per_s_batched": n * w.iters / t_b,
            "frame_iterations_per_s_single_frame_loop": n * w.iters / t_s,
            "speedup": t_s / t_b,
            # equal bit for bit when both use the same plans; otherwise sums run in another order and CG amplifies it
            "max_rel_l2_batched_vs_single": max(diffs),
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
            "ms_per_solve": t * 1e3, "solves_per_s": 1.0 / t, "sigma2": s2, "omega": om,
            "F_first": float(sv.history[0]), "F_last": float(sv.history[-1])}


def fista_leg(pa, torch, dev, geom, y, w):
    """The l1 + TV objective of Eq. 8 on the 512x512 workload: 50 FISTA steps
    with the step from 30 power-iteration steps, x >= 0, FP32, one graph replay
    per solve.  Weights from the data: alpha = 1e-2 max|2 A^T y|,
    beta = 1e-4 max|2 A^T y|, eps = 1e-2."""
    b = float(pa.adjoint(y, geom).abs().max()) * 2.0
    alpha, beta, eps = 1e-2 * b, 1e-4 * b, 1e-2
    sv = pa.FistaSolver(geom, torch.float32, w.iters, w.lam, alpha, beta, eps, omega=0.0, power_iters=30,
                        nonneg=True, graph=True, device=dev)
    x = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
    sv.solve(y, x)
    t = _sync_time(torch, lambda: sv.solve(y, x), 3)
    om, s2 = sv.step()
    return {"workload": f"512x512 ring workload, {w.iters} FISTA steps + 30 power-iteration steps, "
                        f"l1 + TV (alpha {alpha:.3e}, beta {beta:.3e}, eps {eps}), x >= 0, FP32",
            "ms_per_solve": t * 1e3, "solves_per_s": 1.0 / t, "sigma2": s2, "omega": om,
            "F_first": float(sv.history[0]), "F_last": float(sv.history[-1]),
            "zero_fraction": float((x == 0).double().mean())}


def dense_leg(pa, torch, dev):
    """The paper's own formulation on the 128x128 workload: the dense FP64
    matrix (128 sensors x 512 samples by 16384 pixels, 8.6 GB) built on the
    GPU and applied as y = A x and x = A^T y, each reading the whole matrix
    from HBM; next to the matrix-free FP64 operators on the same geometry."""
    from synth import make_config
    w = make_config("C1")
    g = pa.DeviceGeometry(w.geom, dev)
    D = pa.DenseMatrix(g, torch.float64, dev)
    x = torch.from_numpy(w.x).to(dev)
    yv = torch.randn(g.data_shape, dtype=torch.float64, device=dev)
    yo = torch.empty_like(yv)
    xo = torch.empty_like(x)
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

    t_f = ev(lambda: D.forward(x, yo), 10)
    t_a = ev(lambda: D.adjoint(yv, xo), 10)
    op = pa.Operator(g, torch.float64, dev)
    t_mf = ev(lambda: op.forward_(x, yo), 50)
    t_ma = ev(lambda: op.adjoint_(yv, xo), 50)
    nbytes = D.matrix.numel()
    out = {"workload": "128x128 image, 128 sensors, 512 samples, dense FP64 matrix (the paper's kn layout: "
                       f"{g.n_sensors * g.n_samples} x {g.n_pixels})",
           "matrix_bytes": nbytes,
           "us_per_apply": {"dense A": t_f * 1e6, "dense A^T": t_a * 1e6,
                            "matrix-free A (FP64)": t_mf * 1e6, "matrix-free A^T (FP64)": t_ma * 1e6},
           "roofline": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0,
                        "achieved_A": nbytes / t_f / 1e9, "achieved_AT": nbytes / t_a / 1e9,
                        "frac_A": nbytes / t_f / 8e12, "frac_AT": nbytes / t_a / 8e12,
                        "bytes_per_launch": "the matrix once (x, y and the A^T partials are < 1 %)"}}
    del D
    torch.cuda.empty_cache()
    print(f"[bench] dense 128^2 FP64: A {t_f * 1e6:.0f} us ({nbytes / t_f / 1e9:.0f} GB/s), "
          f"A^T {t_a * 1e6:.0f} us; matrix-free {t_mf * 1e6:.1f} / {t_ma * 1e6:.1f} us", file=sys.stderr, flush=True)
    return out


def freq_leg(pa, torch, dev):
    """The frequency-domain matrix of Eq. 7 on the 128x128 workload, at the
    DFT bins of its traces (f_n = (n + 1) / (K dt), 256 bins up to 20 MHz):
    Y = K x and x = Re(K^H Y), FP32 with FP64 phases and sums."""
    from synth import make_config
    w = make_config("C1")
    g = pa.DeviceGeometry(w.geom, dev)
    nf = g.n_samples // 2
    df = 1.0 / (g.n_samples * g.dt)
    op = pa.FreqOperator(g, df, df, nf, torch.float32, dev)
    x = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    Y = op.forward(x)
    xo = torch.empty_like(x)
    t_f = _sync_time(torch, lambda: op.forward(x, Y), 10)
    t_a = _sync_time(torch, lambda: op.adjoint(Y, xo), 10)
    terms = g.n_pixels * g.n_sensors * nf
    print(f"[bench] frequency domain 128^2 x 128 x {nf}: K {t_f * 1e6:.0f} us, K^H {t_a * 1e6:.0f} us",
          file=sys.stderr, flush=True)
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
    in FP32 (FP64 reductions) and in FP64, timed, with their iterate gap."""
    from synth import add_noise, make_config
    w = make_config("C5")
    g = pa.DeviceGeometry(w.geom, dev)
    x_true = torch.from_numpy(w.x.astype(np.float32)).to(dev)
    y32 = torch.from_numpy(add_noise(pa.forward(x_true, g).double().cpu().numpy(), w.noise_rel,
                                     w.noise_seeds[0]).astype(np.float32)).to(dev)
    res = {"workload": "128^3 voxels (0.1 mm), 1024-sensor Fibonacci hemisphere at 20 mm, 2048 samples at 20 ns, "
                       f"{w.iters} CGLS iterations"}
    xs = {}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        if tune:
            res[f"tuning_{name}"] = pa.autotune(g, dt)
        sv = pa.CglsSolver(g, dt, w.iters, w.lam, graph=True, device=dev)
        y = y32.to(dt)
        x = torch.empty(g.image_shape, dtype=dt, device=dev)
        sv.solve(y, x)
        t = _sync_time(torch, lambda: sv.solve(y, x), 2)
        op = pa.Operator(g, dt, dev)
        yo = torch.empty_like(y)
        xo = torch.empty_like(x)
        t_a = _sync_time(torch, lambda: op.forward_(x, yo), 5)
        t_at = _sync_time(torch, lambda: op.adjoint_(y, xo), 5)
        res[name] = {"cgls_iterations_per_s": w.iters / t, "us_per_A": t_a * 1e6, "us_per_AT": t_at * 1e6,
                     "final_F": float(sv.history[-1, 2])}
        xs[name] = x.double()
    res["iterate_rel_l2_f32_vs_f64"] = float(torch.linalg.norm(xs["f32"] - xs["f64"]) / torch.linalg.norm(xs["f64"]))
    res["final_F_rel_f32_vs_f64"] = abs(res["f32"]["final_F"] / res["f64"]["final_F"] - 1)
    print(f"[bench] 3D: f32 {res['f32']['cgls_iterations_per_s']:.1f} it/s, f64 {res['f64']['cgls_iterations_per_s']:.1f} it/s, "
          f"iterate gap {res['iterate_rel_l2_f32_vs_f64']:.2e}", file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    sys.exit(main())
