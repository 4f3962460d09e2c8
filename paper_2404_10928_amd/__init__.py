"""MI355X-native matrix-free photoacoustic operator library.

y = A x is the time-domain measurement matrix of the paper (Eq. 6) with 1/R
spreading and linear interpolation on the sample grid; A^T is its exact
adjoint (delay-and-interpolate back-projection); cgls() solves
min ||A x - y||^2 + lambda ||x||^2 entirely on the GPU.  All arithmetic runs
in hand-written HIP kernels for gfx950 behind the C ABI in include/pa.h.

Importing the package does not touch the GPU; the first call loads
libpa_mi355x.so and raises if it has not been built.
"""
from .build import build, LIB as LIB_PATH

__all__ = ["build", "LIB_PATH", "DeviceGeometry", "forward", "adjoint", "cgls", "CglsSolver",
           "cgls_workspace_bytes", "PAForward", "tv"]


def __getattr__(name):
    if name in ("DeviceGeometry", "forward", "adjoint", "cgls", "CglsSolver", "cgls_workspace_bytes"):
        from . import ops
        return getattr(ops, name)
    if name in ("PAForward", "tv"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
