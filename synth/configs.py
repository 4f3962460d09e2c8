"""The five seeded workloads (C1..C5) the operator and solver are exercised on.

Missing geometry (pitch, ring radius, dt) for the differentiable and batched
workloads is filled in by a fixed rule so every arrival fits in its trace:
h = 0.1 mm; batched frames use ring radius 1.1 * half-diagonal and
dt = (radius + half-diagonal) / (c * (K - 2)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .geometry import Geometry, ring_sensors, fibonacci_hemisphere
from .phantoms import segment_phantom, vessel_tree


@dataclasses.dataclass
class Workload:
    name: str
    geoms: list              # one Geometry per frame
    x_true: list             # one float64 image per frame
    lam: float
    iters: int
    dtype: str               # "f32" (FP32 bulk + FP64 reductions) or "f64"
    noise_rel: float
    noise_seeds: list

    @property
    def geom(self) -> Geometry:
        return self.geoms[0]

    @property
    def x(self) -> np.ndarray:
        """Phantom of the first (for single-frame workloads, the only) frame."""
        return self.x_true[0]


def _c1(seed_base=1001):
    n, h = 128, 1e-4
    g = Geometry(2, n, n, 1, h, (0.0, 0.0, 0.0), ring_sensors(128, 10e-3), 512, 25e-9)
    x = segment_phantom((n, n), 12, [seed_base, 0])
    return Workload("C1", [g], [x], 1e-3, 20, "f64", 0.01, [[seed_base, 1]])


def _c2(seed_base=2002):
    n, h = 512, 5e-5
    g = Geometry(2, n, n, 1, h, (0.0, 0.0, 0.0), ring_sensors(256, 16e-3), 2048, 12.5e-9)
    x = vessel_tree((n, n), 200, [seed_base, 0])
    return Workload("C2", [g], [x], 1e-3, 50, "f32", 0.01, [[seed_base, 1]])


def _c3(seed_base=3003, batch=16):
    n, h = 256, 1e-4
    sens = ring_sensors(128, 20e-3)
    geoms, xs, seeds = [], [], []
    for i in range(batch):
        geoms.append(Geometry(2, n, n, 1, h, (0.0, 0.0, 0.0), sens, 1024, 25e-9))
        xs.append(segment_phantom((n, n), 12, [seed_base, i]))
        seeds.append([seed_base, 100 + i])
    return Workload("C3", geoms, xs, 1e-3, 0, "f32", 0.01, seeds)


def batched_frame(f, seed_base=4004):
    rng = np.random.default_rng([seed_base, f])
    n = int(rng.choice([128, 256, 384, 512]))
    s = int(rng.integers(64, 513))
    k = int(rng.integers(512, 2049))
    h = 1e-4
    half_diag = math.sqrt(2.0) * (n - 1) * h / 2.0
    radius = 1.1 * half_diag
    c = 1500.0
    dt = (radius + half_diag) / (c * (k - 2))
    g = Geometry(2, n, n, 1, h, (0.0, 0.0, 0.0), ring_sensors(s, radius), k, dt)
    x = segment_phantom((n, n), 12, [seed_base, f, 0])
    return g, x


def _c4(seed_base=4004, frames=64):
    geoms, xs, seeds = [], [], []
    for f in range(frames):
        g, x = batched_frame(f, seed_base)
        geoms.append(g)
        xs.append(x)
        seeds.append([seed_base, f, 1])
    return Workload("C4", geoms, xs, 1e-3, 50, "f32", 0.01, seeds)


def _c5(seed_base=5005):
    n, h = 128, 1e-4
    g = Geometry(3, n, n, n, h, (0.0, 0.0, 0.0), fibonacci_hemisphere(1024, 20e-3), 2048, 20e-9)
    x = vessel_tree((n, n, n), 300, [seed_base, 0])
    return Workload("C5", [g], [x], 1e-3, 30, "f32", 0.01, [[seed_base, 1]])


CONFIGS = {"C1": _c1, "C2": _c2, "C3": _c3, "C4": _c4, "C5": _c5}


def make_config(name: str, **kw) -> Workload:
    return CONFIGS[name](**kw)
