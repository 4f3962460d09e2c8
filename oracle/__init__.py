"""FP64 CPU oracle for the photoacoustic operator A, its adjoint and CGLS.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports, links or
calls anything here, and this package imports nothing from the product.

The arithmetic lives in ``pa_oracle.c`` (plain C, FP64, OpenMP over output
rows); this module is ctypes marshalling plus ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "libpa_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("h", ctypes.c_double), ("center", ctypes.c_double * 3),
                ("n_sensors", ctypes.c_int32), ("sensors", ctypes.c_void_p),
                ("n_samples", ctypes.c_int32), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
                ("c", ctypes.c_double), ("r_min", ctypes.c_double)]


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    if True:
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Geom)
        lib.or_forward.argtypes = [gp, dp, dp, ctypes.c_int]
        lib.or_adjoint.argtypes = [gp, dp, dp, ctypes.c_int]
        lib.or_forward_at.argtypes = [gp, dp, ctypes.c_int32, ctypes.c_int32]
        lib.or_forward_at.restype = ctypes.c_double
        lib.or_adjoint_at.argtypes = [gp, dp, ctypes.c_int64]
        lib.or_adjoint_at.restype = ctypes.c_double
        lib.or_cgls.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp,
                                ctypes.c_int]
        lib.or_landweber.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     dp, ctypes.c_int]
        lib.or_power_sigma2.argtypes = [gp, ctypes.c_int, ctypes.c_int]
        lib.or_power_sigma2.restype = ctypes.c_double
        lib.or_tv2d.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, dp]
        lib.or_tv2d.restype = ctypes.c_double
        lib.or_freq_forward.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp, dp,
                                        ctypes.c_int]
        lib.or_freq_adjoint.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp, dp,
                                        ctypes.c_int]
        lib.or_fista.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 dp, dp, ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _geom(g):
    sens = np.ascontiguousarray(g.sensors, dtype=np.float64)
    c = _Geom()
    c.ndim, c.nx, c.ny, c.nz = g.ndim, g.nx, g.ny, g.nz
    c.h = g.h
    ctr = list(g.center) + [0.0] * (3 - len(g.center))
    c.center = (ctypes.c_double * 3)(*ctr[:3])
    c.n_sensors = sens.shape[0]
    c.sensors = sens.ctypes.data if sens.size else None
    c.n_samples = g.n_samples
    c.dt, c.t0, c.c, c.r_min = g.dt, g.t0, g.c, g.r_min
    return c, sens   # keep sens alive alongside the struct


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _threads(threads):
    return int(threads) if threads else 0


def forward(g, x, threads=None) -> np.ndarray:
    """y := A x in FP64; x has g.image_shape, y has (S, K)."""
    lib = _load()
    cg, keep = _geom(g)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    assert x.size == g.n_pixels
    y = np.empty(g.data_shape, dtype=np.float64)
    if lib.or_forward(ctypes.byref(cg), _dp(x), _dp(y), _threads(threads)) != 0:
        raise ValueError("oracle: bad geometry")
    return y


def adjoint(g, y, threads=None) -> np.ndarray:
    lib = _load()
    cg, keep = _geom(g)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    assert y.size == g.n_sensors * g.n_samples
    x = np.empty(g.image_shape, dtype=np.float64)
    if lib.or_adjoint(ctypes.byref(cg), _dp(y), _dp(x), _threads(threads)) != 0:
        raise ValueError("oracle: bad geometry")
    return x


def forward_at(g, x, s, k) -> float:
    lib = _load()
    cg, keep = _geom(g)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    return lib.or_forward_at(ctypes.byref(cg), _dp(x), int(s), int(k))


def adjoint_at(g, y, p) -> float:
    lib = _load()
    cg, keep = _geom(g)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    return lib.or_adjoint_at(ctypes.byref(cg), _dp(y), int(p))


def cgls(g, y, iters, lam, x0=None, threads=None):
    """Returns (x_N, hist[iters+1][3] = (||r_k||, ||s_k||, F_k), stop_iteration)."""
    lib = _load()
    cg, keep = _geom(g)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    x = np.zeros(g.image_shape, dtype=np.float64) if x0 is None else \
        np.array(x0, dtype=np.float64).reshape(g.image_shape).copy()
    hist = np.zeros((iters + 1, 3), dtype=np.float64)
    stop = lib.or_cgls(ctypes.byref(cg), _dp(y), _dp(x), int(iters), float(lam),
                       1 if x0 is None else 0, _dp(hist), _threads(threads))
    if stop < 0:
        raise ValueError("oracle: bad arguments")
    return x, hist, stop


def landweber(g, y, iters, lam, omega, threads=None):
    lib = _load()
    cg, keep = _geom(g)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    x = np.zeros(g.image_shape, dtype=np.float64)
    hist = np.zeros(iters + 1, dtype=np.float64)
    if lib.or_landweber(ctypes.byref(cg), _dp(y), _dp(x), int(iters), float(lam), float(omega),
                        _dp(hist), _threads(threads)) != 0:
        raise ValueError("oracle: bad arguments")
    return x, hist


def power_sigma2(g, iters=30, threads=None):
    """Largest eigenvalue of A^T A after `iters` power-iteration steps from the
    all-ones vector (the gradient iteration's step-size estimate)."""
    lib = _load()
    cg, keep = _geom(g)
    v = lib.or_power_sigma2(ctypes.byref(cg), int(iters), _threads(threads))
    if v < 0:
        raise ValueError("oracle: bad arguments")
    return float(v)


def fista(g, y, iters, lam, alpha, beta, eps, omega, nonneg=False, x_history=False, threads=None):
    """FISTA on ||A x - y||^2 + lam ||x||^2 + beta TV_eps(x) + alpha ||x||_1 from x0 = 0.
    Returns (x_N, hz, hx): hz[k] = F(z_k) for k < N, hz[N] = F(x_N); hx[k] = F(x_k)
    (None unless x_history, which costs one more forward per iteration)."""
    lib = _load()
    cg, keep = _geom(g)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    x = np.zeros(g.image_shape, dtype=np.float64)
    hz = np.zeros(iters + 1, dtype=np.float64)
    hx = np.zeros(iters + 1, dtype=np.float64) if x_history else None
    if lib.or_fista(ctypes.byref(cg), _dp(y), _dp(x), int(iters), float(lam), float(alpha), float(beta),
                    float(eps), float(omega), 1 if nonneg else 0, _dp(hz),
                    _dp(hx) if hx is not None else None, _threads(threads)) != 0:
        raise ValueError("oracle: bad arguments")
    return x, hz, hx


def freq_forward(g, x, f0, df, nf, threads=None) -> np.ndarray:
    """Y = K x for the frequency-domain matrix of Eq. 7; Y is complex [S][nf]."""
    lib = _load()
    cg, keep = _geom(g)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    assert x.size == g.n_pixels
    Y = np.empty((g.n_sensors, int(nf), 2), dtype=np.float64)
    if lib.or_freq_forward(ctypes.byref(cg), float(f0), float(df), int(nf), _dp(x), _dp(Y), _threads(threads)) != 0:
        raise ValueError("oracle: bad arguments")
    return Y[..., 0] + 1j * Y[..., 1]


def freq_adjoint(g, Y, f0, df, nf, threads=None) -> np.ndarray:
    """x = Re(K^H Y) for complex Y [S][nf]."""
    lib = _load()
    cg, keep = _geom(g)
    Y = np.asarray(Y, dtype=np.complex128).reshape(g.n_sensors, int(nf))
    Yi = np.ascontiguousarray(np.stack([Y.real, Y.imag], -1))
    x = np.empty(g.image_shape, dtype=np.float64)
    if lib.or_freq_adjoint(ctypes.byref(cg), float(f0), float(df), int(nf), _dp(Yi), _dp(x), _threads(threads)) != 0:
        raise ValueError("oracle: bad arguments")
    return x


def tv2d(x, eps=1e-8):
    """(TV_eps(x), dTV/dx) of one 2D image in FP64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.ndim == 2
    g = np.empty_like(x)
    v = lib.or_tv2d(_dp(x), x.shape[1], x.shape[0], float(eps), _dp(g))
    return v, g


def loss_gradient(g, x, y, tv_weight, eps=1e-8, threads=None):
    """FP64 value and gradient of ||A x - y||^2 + tv_weight * TV_eps(x) for one 2D frame:
    gradient = 2 A^T (A x - y) + tv_weight * dTV/dx."""
    r = forward(g, x, threads) - np.asarray(y, dtype=np.float64).reshape(g.data_shape)
    tvv, tvg = tv2d(np.asarray(x, dtype=np.float64).reshape(g.image_shape), eps)
    val = float(np.sum(r * r)) + tv_weight * tvv
    grad = 2.0 * adjoint(g, r, threads) + tv_weight * tvg
    return val, grad
