"""Writes c5_cgls_spread.json: how far the FP64 oracle's own 30-iteration CGLS
on the 128^3-voxel hemisphere workload moves when its data y is perturbed.

The solve amplifies small changes of its inputs (the iterates of CG are
sensitive to rounding once the residual has fallen a few decades), so an
after-solve gate for a solve that rounds differently from the oracle has to
be set from the spread between equally valid solves.  Two perturbations are
measured, each as y_i (1 + eps u_i) with u_i ~ N(0, 1) drawn from a fixed seed:
  eps = 1e-12  (far below any FP64 summation-order effect on y)
  eps = 6e-8   (half an FP32 ulp: the size of FP32 rounding of the data)
For each: F_k of the perturbed solve relative to the unperturbed one at
every k, the relative L2 distance of x_30 from the unperturbed x_30, and the
same distance over the 4096 voxels stored in c5_cgls_reference.json.

Only the oracle and the seeded input generators are called.  Run from the
repository root:
    python tests/golden/make_c5_spread.py [threads]
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
from make_c5_reference import c5_data, sample_indices  # noqa: E402

EPS = (1e-12, 6e-8)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else None
    w, g, y = c5_data(threads)
    t0 = time.time()
    x0, h0, _ = oracle.cgls(g, y, w.iters, w.lam, threads=threads)
    print(f"unperturbed solve {time.time() - t0:.0f} s", flush=True)
    idx = sample_indices(g.n_pixels)
    out = {"what": "spread of the FP64 oracle's 30-iteration CGLS (128^3 hemisphere workload) under relative "
                   "perturbations y (1 + eps u), u ~ N(0, 1)",
           "F_unperturbed": h0[:, 2].tolist(), "perturbations": {}}
    for j, eps in enumerate(EPS):
        u = np.random.default_rng([5005, 90 + j]).standard_normal(y.shape)
        t0 = time.time()
        x, h, _ = oracle.cgls(g, y * (1.0 + eps * u), w.iters, w.lam, threads=threads)
        dF = np.abs(h[:, 2] / h0[:, 2] - 1.0)
        dx = float(np.linalg.norm(x - x0) / np.linalg.norm(x0))
        xs, x0s = x.reshape(-1)[idx], x0.reshape(-1)[idx]
        dxs = float(np.linalg.norm(xs - x0s) / np.linalg.norm(x0s))
        out["perturbations"][f"{eps:g}"] = {"eps": eps, "F_rel_by_k": dF.tolist(), "F_final_rel": float(dF[-1]),
                                           "F_max_rel": float(dF.max()), "x_final_rel_l2": dx,
                                           "x_sample_rel_l2": dxs}
        print(f"eps {eps:g}: {time.time() - t0:.0f} s, F_30 {dF[-1]:.3e}, max_k F {dF.max():.3e}, "
              f"x_30 {dx:.3e} (sampled {dxs:.3e})", flush=True)
    with open(os.path.join(HERE, "c5_cgls_spread.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
