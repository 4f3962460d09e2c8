"""Writes solve_spread.json: how far the FP64 oracle's own CGLS moves when
every operator application is perturbed by noise of the size of a GPU
solve's rounding.

CG amplifies rounding.  On the ring and hemisphere workloads there are
stretches of iterations where a change in the 13th digit of one operator
application grows to a 1e-3 .. 1e-1 change of F(x_k) a few iterations later
(and, on some workloads, shrinks back again).  A GPU solve rounds differently
from the oracle in every application: its sums run in another order, and
under PA_F32 / PA_MIXED the delays and weights are formed in FP32.  Past the
stable iterations such a solve follows another, equally valid, trajectory,
so a gate after the solve has to come from the band those trajectories
span.  This script measures the band with the oracle itself:

  CGLS in FP64 (the same recurrences as oracle.cgls), written out with numpy
  around oracle.forward / oracle.adjoint, where the output v of every
  application becomes v + eps * (||v|| / sqrt(n)) * u, u ~ N(0, 1) from a
  seeded generator, i.e. a relative L2 change of eps per application.

eps is the per-application relative L2 error measured for each GPU
precision on these workloads:
  f64: 1e-13   (FP64 taps and sums in another order)
  f32: 1e-6    (FP32 delays and weights: PA_F32 and PA_MIXED)
Three seeds per eps, plus, for f64, the unperturbed numpy solve (its inner
products and updates round in another order than the C oracle's).  Stored
per case and eps: the largest relative change of F_k and of ||r_k|| at every
k, and of the final iterate (relative L2; for the 3D case also over the 4096
voxels of c5_cgls_reference.json).

Only the oracle and the seeded input generators are called.  Run from the
repository root:
    python tests/golden/make_solve_spread.py [threads] [case ...]
cases: c1 c4_58 c4_10 c4_7 c5 (default: all; the 3D case takes about an hour
on 8 threads).  Cases already in the file and not named are kept.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from synth import add_noise, make_config  # noqa: E402

OUT = os.path.join(HERE, "solve_spread.json")
EPS = {"f64": 1e-13, "f32": 1e-6}
SEEDS = 3


def case_problem(name, threads):
    """(geometry, y, iters, lambda, sample index or None) of each case, with
    the data the GPU tests solve."""
    if name == "c1":
        w = make_config("C1")
        y = add_noise(oracle.forward(w.geom, w.x, threads=threads), w.noise_rel, w.noise_seeds[0])
        return w.geom, y, w.iters, w.lam, None
    if name.startswith("c4_"):
        i = int(name[3:])
        w = make_config("C4")
        g = w.geoms[i]
        y = add_noise(oracle.forward(g, w.x_true[i], threads=threads), w.noise_rel, w.noise_seeds[i])
        return g, y.astype(np.float32).astype(np.float64), w.iters, w.lam, None
    if name == "c5":
        from make_c5_reference import c5_data, sample_indices
        w, g, y = c5_data(threads)
        return g, y, w.iters, w.lam, sample_indices(g.n_pixels)
    raise ValueError(name)


def cgls_perturbed(g, y, iters, lam, eps, rng, threads):
    """CGLS from x0 = 0 with every application of A and A^T perturbed by a
    relative L2 amount eps (eps = 0: no perturbation).  Returns (x, hist)."""
    def noisy(v):
        if eps == 0.0:
            return v
        scale = eps * np.linalg.norm(v) / np.sqrt(v.size)
        return v + scale * rng.standard_normal(v.shape)

    def A(v):
        return noisy(oracle.forward(g, v, threads=threads))

    def At(v):
        return noisy(oracle.adjoint(g, v, threads=threads))

    x = np.zeros(g.image_shape)
    r = np.array(y, dtype=np.float64).reshape(g.data_shape).copy()
    s = At(r) - lam * x
    p = s.copy()
    gamma = float(np.vdot(s, s))
    hist = np.zeros((iters + 1, 3))

    def record(k):
        rr = float(np.vdot(r, r))
        hist[k] = (np.sqrt(rr), np.sqrt(gamma), rr + lam * float(np.vdot(x, x)))
    record(0)
    for k in range(iters):
        q = A(p)
        delta = float(np.vdot(q, q)) + lam * float(np.vdot(p, p))
        alpha = gamma / delta
        x += alpha * p
        r -= alpha * q
        s = At(r) - lam * x
        gamma1 = float(np.vdot(s, s))
        beta = gamma1 / gamma
        gamma = gamma1
        p = s + beta * p
        record(k + 1)
    return x, hist


def run_case(name, threads):
    g, y, iters, lam, idx = case_problem(name, threads)
    t0 = time.time()
    x0, h0, stop = oracle.cgls(g, y, iters, lam, threads=threads)
    assert stop == iters, f"{name}: the oracle solve stopped at {stop}"
    print(f"{name}: oracle solve {time.time() - t0:.0f} s", flush=True)
    out = {"iters": iters, "lam": lam, "shape": list(g.image_shape), "sensors": g.n_sensors,
           "samples": g.n_samples, "F_oracle": h0[:, 2].tolist()}
    for pi, (prec, eps) in enumerate(EPS.items()):
        runs = [(eps, s) for s in range(SEEDS)] + ([(0.0, -1)] if prec == "f64" else [])
        per = []
        for e, seed in runs:
            rng = np.random.default_rng([9009, pi, max(seed, 0)])
            t0 = time.time()
            x, h = cgls_perturbed(g, y, iters, lam, e, rng, threads)
            dF = np.abs(h[:, 2] / h0[:, 2] - 1)
            dr = np.abs(h[:, 0] / h0[:, 0] - 1)
            rec = {"eps": e, "seed": seed, "F_rel_by_k": dF.tolist(), "r_rel_by_k": dr.tolist(),
                   "x_rel_l2": float(np.linalg.norm(x - x0) / np.linalg.norm(x0))}
            if idx is not None:
                xs, x0s = x.reshape(-1)[idx], x0.reshape(-1)[idx]
                rec["x_sample_rel_l2"] = float(np.linalg.norm(xs - x0s) / np.linalg.norm(x0s))
            per.append(rec)
            print(f"{name} {prec} eps {e:g} seed {seed}: {time.time() - t0:.0f} s, F_N {dF[-1]:.2e}, "
                  f"max_k F {dF.max():.2e}, x_N {rec['x_rel_l2']:.2e}", flush=True)
        band = {"eps": eps,
                "F_rel_by_k": np.max([p["F_rel_by_k"] for p in per], axis=0).tolist(),
                "r_rel_by_k": np.max([p["r_rel_by_k"] for p in per], axis=0).tolist(),
                "x_rel_l2": max(p["x_rel_l2"] for p in per), "runs": per}
        if idx is not None:
            band["x_sample_rel_l2"] = max(p["x_sample_rel_l2"] for p in per)
        out[prec] = band
    return out


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else None
    cases = sys.argv[2:] or ["c1", "c4_58", "c4_10", "c4_7", "c5"]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["what"] = ("band of the FP64 oracle's CGLS under per-application relative L2 perturbations eps "
                    "(f64: 1e-13, f32: 1e-6), largest change over three seeds (and, for f64, the unperturbed "
                    "numpy solve) relative to oracle.cgls")
    for c in cases:
        data[c] = run_case(c, threads)
        with open(OUT, "w") as f:
            json.dump(data, f)


if __name__ == "__main__":
    main()
