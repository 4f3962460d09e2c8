"""Image-grid and sensor-array descriptions (inputs only).

The paper's time-domain measurement matrix (Section "Principle of Iterative
Reconstruction", Eq. 6) is indexed by a pixel position r_ij and a probe
position r_m.  This module fixes how those positions are laid out:

* the grid is centred on ``center``; pixel (ix, iy[, iz]) sits at
  center + (i - (n-1)/2) * h on each axis, images are stored [nz][ny][nx]
  with ix fastest;
* sensor m of an S-sensor ring sits at angle 2*pi*m/S from +x;
* the hemisphere is a Fibonacci lattice on the lower half sphere.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Geometry:
    ndim: int
    nx: int
    ny: int
    nz: int
    h: float                      # pixel pitch [m]
    center: tuple                 # grid centre [m], 3 entries (z ignored in 2D)
    sensors: np.ndarray           # float64 [S][ndim], metres
    n_samples: int                # K
    dt: float                     # sample interval [s]
    t0: float = 0.0               # time of sample 0 [s]
    c: float = 1500.0             # speed of sound [m/s]
    r_min: float = 0.0            # distance clamp [m]; 0 selects h/2

    @property
    def n_sensors(self) -> int:
        return int(self.sensors.shape[0])

    @property
    def n_pixels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def image_shape(self) -> tuple:
        return (self.ny, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def data_shape(self) -> tuple:
        return (self.n_sensors, self.n_samples)

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def ring_sensors(n: int, radius: float, center=(0.0, 0.0)) -> np.ndarray:
    """S point sensors on a circle; sensor m at angle 2*pi*m/S from +x."""
    m = np.arange(n, dtype=np.float64)
    ang = 2.0 * math.pi * m / n
    out = np.empty((n, 2), dtype=np.float64)
    out[:, 0] = center[0] + radius * np.cos(ang)
    out[:, 1] = center[1] + radius * np.sin(ang)
    return out


def fibonacci_hemisphere(n: int, radius: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Fibonacci lattice on the lower hemisphere (z < 0) of a sphere.

    z_i = -(i + 1/2)/n, rho_i = sqrt(1 - z_i^2), phi_i = i * pi * (3 - sqrt 5).
    """
    i = np.arange(n, dtype=np.float64)
    z = -(i + 0.5) / n
    rho = np.sqrt(1.0 - z * z)
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    out = np.empty((n, 3), dtype=np.float64)
    out[:, 0] = center[0] + radius * rho * np.cos(phi)
    out[:, 1] = center[1] + radius * rho * np.sin(phi)
    out[:, 2] = center[2] + radius * z
    return out
