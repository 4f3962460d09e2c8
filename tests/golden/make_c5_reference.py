"""Writes c5_cgls_reference.json: the FP64 oracle's CGLS on the 128^3-voxel,
1024-sensor hemisphere workload (30 iterations, lambda 1e-3) from data
y = A x_true + 1% noise rounded to float32, i.e. the data an FP32 solve sees.

Stored: the history (||r_k||, ||s_k||, F_k) at every k, ||x_30||, and x_30 at
4096 voxels drawn with a fixed seed.  Only the oracle and the seeded input
generators are called.  Run from the repository root:
    python tests/golden/make_c5_reference.py [threads]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import add_noise, make_config  # noqa: E402

N_SAMPLE = 4096


def c5_data(threads=None):
    w = make_config("C5")
    g = w.geom
    y = add_noise(oracle.forward(g, w.x, threads=threads), w.noise_rel, w.noise_seeds[0])
    return w, g, y.astype(np.float32).astype(np.float64)


def sample_indices(n_pixels):
    return np.sort(np.random.default_rng([5005, 77]).choice(n_pixels, N_SAMPLE, replace=False))


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else None
    w, g, y = c5_data(threads)
    x, hist, stop = oracle.cgls(g, y, w.iters, w.lam, threads=threads)
    idx = sample_indices(g.n_pixels)
    out = {
        "what": "FP64 oracle CGLS, 128^3 voxels, 1024-sensor hemisphere, 2048 samples, 30 iterations, lambda 1e-3",
        "iters": w.iters, "lam": w.lam, "stop": int(stop),
        "history": hist.tolist(),
        "x_norm": float(np.linalg.norm(x)),
        "sample_index": idx.tolist(),
        "x_sample": x.reshape(-1)[idx].tolist(),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_cgls_reference.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
