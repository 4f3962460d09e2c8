"""Shared helpers for the GPU parity tests (loaded only by tests marked gpu)."""
import math

import numpy as np

from synth import Geometry, ring_sensors, fibonacci_hemisphere


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def ring_geom(n=(37, 29), S=70, K=300, h=1e-4, radius=None, t0=0.0, dt=None, center=(0.0, 0.0), r_min=0.0):
    nx, ny = n
    half_diag = math.hypot(nx - 1, ny - 1) * h / 2
    if radius is None:
        radius = 1.2 * half_diag
    if dt is None:
        dt = (radius + half_diag) / (1500.0 * (K - 4))
    sens = ring_sensors(S, radius, center)
    return Geometry(2, nx, ny, 1, h, (center[0], center[1], 0.0), sens, K, dt, t0, 1500.0, r_min)


def hemi_geom(n=(19, 13, 11), S=90, K=260, h=1e-4, radius=None, t0=0.0, dt=None):
    nx, ny, nz = n
    half_diag = math.sqrt((nx - 1) ** 2 + (ny - 1) ** 2 + (nz - 1) ** 2) * h / 2
    if radius is None:
        radius = 1.3 * half_diag
    if dt is None:
        dt = (radius + half_diag) / (1500.0 * (K - 4))
    sens = fibonacci_hemisphere(S, radius)
    return Geometry(3, nx, ny, nz, h, (0.0, 0.0, 0.0), sens, K, dt, t0, 1500.0)


def rounded(x, dtype):
    """The value the GPU sees (dtype) and its exact FP64 image for the oracle."""
    xd = np.asarray(x, dtype=dtype)
    return xd, xd.astype(np.float64)
