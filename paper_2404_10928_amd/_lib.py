"""ctypes marshalling for libpa_mi355x.so (the C ABI declared in include/pa.h).

Nothing here computes: every step runs in the HIP kernels behind the C ABI.
torch supplies device memory and the current stream.  If the shared library
is missing the import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa_mi355x.so")

PA_OK = 0
PA_ERR_INVALID_ARGUMENT = 1
PA_ERR_UNSUPPORTED = 2
PA_ERR_WORKSPACE = 3
PA_ERR_HIP = 4
PA_ERR_BREAKDOWN = 5
STATUS_NAMES = {0: "PA_OK", 1: "PA_ERR_INVALID_ARGUMENT", 2: "PA_ERR_UNSUPPORTED", 3: "PA_ERR_WORKSPACE",
                4: "PA_ERR_HIP", 5: "PA_ERR_BREAKDOWN"}

PA_F32 = 0
PA_F64 = 1
PA_MIXED = 2
PA_X0_ZERO = 1
PA_USE_GRAPH = 2
PA_NONNEG = 4

EXPORTS = ["pa_validate_geometry", "pa_forward", "pa_forward_workspace_bytes", "pa_forward_ws", "pa_forward_noalloc", "pa_adjoint",
           "pa_autotune_workspace_bytes", "pa_cgls_workspace_bytes", "pa_cgls_solve",
           "pa_cgls_stop_iteration", "pa_last_error", "pa_abi_version", "pa_batch_create", "pa_batch_destroy",
           "pa_batch_offsets", "pa_batch_workspace_bytes", "pa_batch_cgls_workspace_bytes", "pa_batch_forward",
           "pa_batch_adjoint", "pa_batch_cgls_solve", "pa_batch_stop_iterations", "pa_autotune", "pa_tuning_set", "pa_tuning_clear",
           "pa_landweber_workspace_bytes", "pa_landweber_solve", "pa_landweber_step",
           "pa_batch_autotune_workspace_bytes", "pa_batch_autotune", "pa_fista_workspace_bytes", "pa_fista_solve",
           "pa_fista_step", "pa_dense_matrix_bytes", "pa_dense_build", "pa_dense_forward",
           "pa_dense_adjoint_workspace_bytes", "pa_dense_adjoint",
           "pa_freq_workspace_bytes", "pa_freq_forward", "pa_freq_adjoint"]


class PaTuning(ctypes.Structure):
    _fields_ = [("fwd_seg", ctypes.c_int32), ("adj_lds_bytes", ctypes.c_int32), ("fwd_mode", ctypes.c_int32),
                ("fwd_tile", ctypes.c_int32 * 3), ("fwd_us", ctypes.c_double), ("adj_us", ctypes.c_double)]


class PaGeometry(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("center", ctypes.c_double * 3), ("n_sensors", ctypes.c_int32),
                ("sensors", ctypes.c_void_p), ("n_samples", ctypes.c_int32), ("dt", ctypes.c_double),
                ("t0", ctypes.c_double), ("c", ctypes.c_double), ("r_min", ctypes.c_double)]


class PaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2404_10928_amd.build.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, gp = ctypes.c_void_p, ctypes.POINTER(PaGeometry)
    lib.pa_validate_geometry.argtypes = [gp, ctypes.c_int]
    lib.pa_validate_geometry.restype = ctypes.c_int
    lib.pa_forward.argtypes = [gp, ctypes.c_int, vp, vp, vp]
    lib.pa_forward.restype = ctypes.c_int
    lib.pa_forward_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_forward_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_forward_ws.argtypes = [gp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pa_forward_ws.restype = ctypes.c_int
    lib.pa_forward_noalloc.argtypes = [gp, ctypes.c_int, vp, vp, vp]
    lib.pa_forward_noalloc.restype = ctypes.c_int
    lib.pa_adjoint.argtypes = [gp, ctypes.c_int, vp, vp, vp]
    lib.pa_adjoint.restype = ctypes.c_int
    lib.pa_cgls_workspace_bytes.argtypes = [gp, ctypes.c_int, ctypes.c_int32]
    lib.pa_cgls_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_cgls_solve.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, vp,
                                  ctypes.c_size_t, vp, vp]
    lib.pa_cgls_solve.restype = ctypes.c_int
    lib.pa_cgls_stop_iteration.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.pa_cgls_stop_iteration.restype = ctypes.c_int
    lib.pa_last_error.argtypes = []
    lib.pa_last_error.restype = ctypes.c_char_p
    lib.pa_abi_version.argtypes = []
    lib.pa_abi_version.restype = ctypes.c_int32
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.pa_batch_create.argtypes = [gp, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(vp)]
    lib.pa_batch_create.restype = ctypes.c_int
    lib.pa_batch_destroy.argtypes = [vp]
    lib.pa_batch_destroy.restype = ctypes.c_int
    lib.pa_batch_offsets.argtypes = [vp, i64p, i64p]
    lib.pa_batch_offsets.restype = ctypes.c_int
    lib.pa_batch_workspace_bytes.argtypes = [vp]
    lib.pa_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_batch_cgls_workspace_bytes.argtypes = [vp, ctypes.c_int32]
    lib.pa_batch_cgls_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_batch_forward.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pa_batch_forward.restype = ctypes.c_int
    lib.pa_batch_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pa_batch_adjoint.restype = ctypes.c_int
    lib.pa_batch_cgls_solve.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, vp,
                                        ctypes.c_size_t, vp, vp]
    lib.pa_batch_cgls_solve.restype = ctypes.c_int
    lib.pa_batch_stop_iterations.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.pa_batch_stop_iterations.restype = ctypes.c_int
    lib.pa_autotune_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_autotune_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_autotune.argtypes = [gp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(PaTuning)]
    lib.pa_autotune.restype = ctypes.c_int
    lib.pa_tuning_set.argtypes = [gp, ctypes.c_int, ctypes.POINTER(PaTuning)]
    lib.pa_tuning_set.restype = ctypes.c_int
    lib.pa_tuning_clear.argtypes = []
    lib.pa_tuning_clear.restype = ctypes.c_int
    lib.pa_landweber_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_landweber_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_landweber_solve.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_uint32, vp, ctypes.c_size_t, vp, vp]
    lib.pa_landweber_solve.restype = ctypes.c_int
    dpp = ctypes.POINTER(ctypes.c_double)
    lib.pa_landweber_step.argtypes = [vp, dpp, dpp]
    lib.pa_landweber_step.restype = ctypes.c_int
    lib.pa_batch_autotune_workspace_bytes.argtypes = [vp]
    lib.pa_batch_autotune_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_batch_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.pa_batch_autotune.restype = ctypes.c_int
    lib.pa_fista_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_fista_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_fista_solve.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                   vp, ctypes.c_size_t, vp, vp]
    lib.pa_fista_solve.restype = ctypes.c_int
    lib.pa_fista_step.argtypes = [vp, dpp, dpp]
    lib.pa_fista_step.restype = ctypes.c_int
    lib.pa_dense_matrix_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_dense_matrix_bytes.restype = ctypes.c_size_t
    lib.pa_dense_adjoint_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_dense_adjoint_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_dense_build.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp]
    lib.pa_dense_build.restype = ctypes.c_int
    lib.pa_dense_forward.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp, vp, vp]
    lib.pa_dense_forward.restype = ctypes.c_int
    lib.pa_dense_adjoint.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pa_dense_adjoint.restype = ctypes.c_int
    lib.pa_freq_workspace_bytes.argtypes = [gp, ctypes.c_int, ctypes.c_int32]
    lib.pa_freq_workspace_bytes.restype = ctypes.c_size_t
    for name in ("pa_freq_forward", "pa_freq_adjoint"):
        fn = getattr(lib, name)
        fn.argtypes = [gp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp, vp,
                       ctypes.c_size_t, vp]
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().pa_last_error().decode()


def check(status: int, allow=(PA_OK,)) -> int:
    if status not in allow:
        raise PaError(status, last_error())
    return status
