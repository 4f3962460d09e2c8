"""Seeded synthetic inputs for the photoacoustic operator workloads.

This package holds only input generation: sensor layouts, grid descriptions,
vessel-like phantoms and measurement noise.  It contains none of the
forward/adjoint arithmetic, so the FP64 oracle and the GPU path can both use
it without sharing any of the method's code.
"""
from .geometry import Geometry, ring_sensors, fibonacci_hemisphere
from .phantoms import segment_phantom, vessel_tree
from .noise import add_noise
from .configs import CONFIGS, make_config, Workload

__all__ = ["Geometry", "ring_sensors", "fibonacci_hemisphere", "segment_phantom",
           "vessel_tree", "add_noise", "CONFIGS", "make_config", "Workload"]
