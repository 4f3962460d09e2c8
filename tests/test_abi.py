"""The C ABI library loads, exports every function include/pa.h declares, and
rejects bad arguments on the host before touching a GPU (CPU-only test)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")
LIB = os.path.join(ROOT, "paper_2404_10928_amd", "libpa_mi355x.so")


class Geom(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("center", ctypes.c_double * 3), ("n_sensors", ctypes.c_int32),
                ("sensors", ctypes.c_void_p), ("n_samples", ctypes.c_int32), ("dt", ctypes.c_double),
                ("t0", ctypes.c_double), ("c", ctypes.c_double), ("r_min", ctypes.c_double)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2404_10928_amd.build import build
        build()
    l = ctypes.CDLL(LIB)
    gp = ctypes.POINTER(Geom)
    l.pa_validate_geometry.argtypes = [gp, ctypes.c_int]
    l.pa_forward.argtypes = [gp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    l.pa_adjoint.argtypes = [gp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    l.pa_cgls_workspace_bytes.argtypes = [gp, ctypes.c_int, ctypes.c_int32]
    l.pa_cgls_workspace_bytes.restype = ctypes.c_size_t
    l.pa_cgls_solve.argtypes = [gp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    l.pa_last_error.restype = ctypes.c_char_p
    l.pa_cgls_stop_iteration.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
    return l


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pa_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"pa_forward", "pa_adjoint", "pa_cgls_solve", "pa_cgls_workspace_bytes"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.pa_abi_version() == 2


def good():
    g = Geom()
    g.ndim, g.nx, g.ny, g.nz = 2, 64, 48, 1
    g.h = 1e-4
    g.center = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    g.n_sensors = 32
    g.sensors = 4096          # never dereferenced on the host
    g.n_samples = 300
    g.dt, g.t0, g.c, g.r_min = 25e-9, 0.0, 1500.0, 0.0
    return g


BAD = [
    ("ndim", 4, 1), ("nz", 3, 1), ("nx", -1, 1), ("n_sensors", -2, 1), ("n_samples", -1, 1),
    ("h", 0.0, 1), ("h", float("nan"), 1), ("dt", -1e-9, 1), ("c", float("inf"), 1), ("t0", float("nan"), 1),
    ("r_min", -1e-6, 1), ("sensors", 0, 1), ("sensors", 4097, 1), ("n_samples", (1 << 22) + 1, 2),
    ("dt", 1e-15, 2),  # h / (c dt) so large a single tile's window cannot fit in LDS
]


@pytest.mark.parametrize("field,value,code", BAD, ids=[f"{f}={v}" for f, v, _ in BAD])
def test_invalid_geometry_rejected_on_host(lib, field, value, code):
    g = good()
    setattr(g, field, value)
    assert lib.pa_validate_geometry(ctypes.byref(g), 0) == code
    assert lib.pa_last_error()
    # the operator entry points fail the same way, before any HIP call
    assert lib.pa_forward(ctypes.byref(g), 0, 256, 1 << 20, None) == code
    assert lib.pa_adjoint(ctypes.byref(g), 0, 1 << 20, 256, None) == code
    assert lib.pa_cgls_workspace_bytes(ctypes.byref(g), 0, 10) == 0


def test_valid_geometry_and_workspace(lib):
    g = good()
    assert lib.pa_validate_geometry(ctypes.byref(g), 0) == 0
    assert lib.pa_last_error() == b""
    n32 = lib.pa_cgls_workspace_bytes(ctypes.byref(g), 0, 20)
    n64 = lib.pa_cgls_workspace_bytes(ctypes.byref(g), 1, 20)
    P, M = 64 * 48, 32 * 300
    assert n32 >= 4 * (2 * P + 2 * M) and n64 >= 8 * (2 * P + 2 * M) and n64 > n32
    assert lib.pa_validate_geometry(None, 0) == 1
    assert lib.pa_validate_geometry(ctypes.byref(g), 7) == 1


def test_pointer_and_argument_checks_on_host(lib):
    g = good()
    # NULL / misaligned / overlapping buffers
    assert lib.pa_forward(ctypes.byref(g), 0, None, 1 << 20, None) == 1
    assert lib.pa_forward(ctypes.byref(g), 0, 256 + 2, 1 << 20, None) == 1
    assert lib.pa_forward(ctypes.byref(g), 0, 1 << 20, (1 << 20) + 64, None) == 1
    assert lib.pa_adjoint(ctypes.byref(g), 1, 1 << 20, 256 + 4, None) == 1
    ws = lib.pa_cgls_workspace_bytes(ctypes.byref(g), 0, 5)
    base = 1 << 30
    args = lambda **kw: dict(dict(it=5, lam=1e-3, flags=1, ws=base, wsb=ws), **kw)
    def solve(a):
        return lib.pa_cgls_solve(ctypes.byref(g), 0, 1 << 20, 1 << 24, a["it"], a["lam"], a["flags"], a["ws"],
                                 a["wsb"], None, None)
    assert solve(args(it=-1)) == 1
    assert solve(args(lam=-1.0)) == 1
    assert solve(args(lam=float("nan"))) == 1
    assert solve(args(flags=8)) == 1
    assert solve(args(ws=None)) == 3
    assert solve(args(ws=base + 16)) == 3
    assert solve(args(wsb=ws - 1)) == 3
    stop = ctypes.c_int32()
    assert lib.pa_cgls_stop_iteration(None, ctypes.byref(stop)) == 1


def batch_lib(lib):
    vp = ctypes.c_void_p
    gp = ctypes.POINTER(Geom)
    lib.pa_batch_create.argtypes = [gp, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(vp)]
    lib.pa_batch_destroy.argtypes = [vp]
    lib.pa_batch_offsets.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.pa_batch_workspace_bytes.argtypes = [vp]
    lib.pa_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_batch_cgls_workspace_bytes.argtypes = [vp, ctypes.c_int32]
    lib.pa_batch_cgls_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_batch_forward.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.pa_batch_cgls_solve.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, vp,
                                        ctypes.c_size_t, vp, vp]
    return lib


def test_batch_planning_on_host(lib):
    lib = batch_lib(lib)
    frames = (Geom * 3)(good(), good(), good())
    frames[1].nx, frames[1].n_sensors, frames[1].n_samples = 100, 17, 450
    frames[2].ny, frames[2].dt = 7, 40e-9
    h = ctypes.c_void_p()
    assert lib.pa_batch_create(frames, 3, 0, ctypes.byref(h)) == 0 and h.value
    xo = (ctypes.c_int64 * 4)()
    yo = (ctypes.c_int64 * 4)()
    assert lib.pa_batch_offsets(h, xo, yo) == 0
    P = [64 * 48, 100 * 48, 64 * 7]
    M = [32 * 300, 17 * 450, 32 * 300]
    assert list(xo) == [0, P[0], P[0] + P[1], sum(P)]
    assert list(yo) == [0, M[0], M[0] + M[1], sum(M)]
    n_op = lib.pa_batch_workspace_bytes(h)
    n_cg = lib.pa_batch_cgls_workspace_bytes(h, 20)
    assert n_op > 0 and n_cg >= n_op + 4 * 2 * (sum(P) + sum(M))
    # workspace and buffer checks fail on the host, before any HIP call
    assert lib.pa_batch_forward(h, 1 << 20, 1 << 28, None, 0, None) == 3
    assert lib.pa_batch_forward(h, 1 << 20, 1 << 28, (1 << 32) + 16, n_op, None) == 3
    assert lib.pa_batch_forward(h, 1 << 20, 1 << 28, 1 << 32, n_op - 1, None) == 3
    assert lib.pa_batch_forward(h, None, 1 << 28, 1 << 32, n_op, None) == 1
    assert lib.pa_batch_cgls_solve(h, 1 << 28, 1 << 20, 5, -1.0, 1, 1 << 32, n_cg, None, None) == 1
    assert lib.pa_batch_cgls_solve(h, 1 << 28, 1 << 20, 5, 1e-3, 8, 1 << 32, n_cg, None, None) == 1
    assert lib.pa_batch_destroy(h) == 0


def test_batch_rejects_bad_frames_on_host(lib):
    lib = batch_lib(lib)
    h = ctypes.c_void_p()
    frames = (Geom * 2)(good(), good())
    assert lib.pa_batch_create(frames, 0, 0, ctypes.byref(h)) == 1
    frames[1].dt = -1.0
    assert lib.pa_batch_create(frames, 2, 0, ctypes.byref(h)) == 1
    assert b"frame 1" in lib.pa_last_error()
    frames[1] = good()
    frames[1].ndim, frames[1].nz = 3, 4
    frames[1].sensors = 4096 * 3
    assert lib.pa_batch_create(frames, 2, 0, ctypes.byref(h)) == 1
    assert b"ndim" in lib.pa_last_error()


def test_autotune_argument_checks_on_host(lib):
    vp = ctypes.c_void_p
    lib.pa_autotune.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp, vp]
    lib.pa_autotune_workspace_bytes.argtypes = [ctypes.POINTER(Geom), ctypes.c_int]
    lib.pa_autotune_workspace_bytes.restype = ctypes.c_size_t
    g = good()
    # FP32: the partial-row candidates need a workspace; FP64 times the sensor-major method only
    assert lib.pa_autotune_workspace_bytes(ctypes.byref(g), 0) > 0
    assert lib.pa_autotune_workspace_bytes(ctypes.byref(g), 1) == 0
    assert lib.pa_autotune(ctypes.byref(g), 0, None, 1 << 20, None, 0, None, None) == 1
    assert lib.pa_autotune(ctypes.byref(g), 0, 1 << 20, (1 << 20) + 64, None, 0, None, None) == 1
    # a misaligned workspace and one that overlaps x
    assert lib.pa_autotune(ctypes.byref(g), 0, 1 << 20, 1 << 28, (1 << 30) + 8, 4096, None, None) == 3
    assert lib.pa_autotune(ctypes.byref(g), 0, 1 << 20, 1 << 28, 1 << 20, 4096, None, None) == 1
    g.dt = -1.0
    assert lib.pa_autotune(ctypes.byref(g), 0, 1 << 20, 1 << 28, None, 0, None, None) == 1
    assert lib.pa_tuning_clear() == 0


def test_forward_workspace_checks_on_host(lib):
    vp = ctypes.c_void_p
    lib.pa_forward_workspace_bytes.argtypes = [ctypes.POINTER(Geom), ctypes.c_int]
    lib.pa_forward_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_forward_ws.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    g = good()
    # by rule the forward operator is the sensor-major one, which needs no workspace
    assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 0) == 0
    assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 2) == 0
    assert lib.pa_forward_ws(ctypes.byref(g), 0, None, 1 << 20, None, 0, None) == 1
    assert lib.pa_forward_ws(ctypes.byref(g), 0, 1 << 20, (1 << 20) + 64, None, 0, None) == 1
    g.dt = -1.0
    assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 0) == 0


def test_landweber_argument_checks_on_host(lib):
    vp = ctypes.c_void_p
    lib.pa_landweber_workspace_bytes.argtypes = [ctypes.POINTER(Geom), ctypes.c_int]
    lib.pa_landweber_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_landweber_solve.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, vp, vp, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_uint32, vp, ctypes.c_size_t, vp, vp]
    g = good()
    n = lib.pa_landweber_workspace_bytes(ctypes.byref(g), 0)
    P, M = 64 * 48, 32 * 300
    assert n >= 4 * (2 * P + 2 * M)
    def solve(it=5, lam=1e-3, om=0.0, pw=30, flags=1, ws=1 << 32, wsb=n):
        return lib.pa_landweber_solve(ctypes.byref(g), 0, 1 << 20, 1 << 24, it, lam, om, pw, flags, ws, wsb, None, None)
    assert solve(it=-1) == 1
    assert solve(lam=-1.0) == 1
    assert solve(om=-0.5) == 1
    assert solve(om=0.0, pw=0) == 1
    assert solve(flags=4) == 1
    assert solve(ws=None) == 3
    assert solve(wsb=n - 1) == 3
    assert solve(ws=(1 << 32) + 8) == 3


def test_fista_argument_checks_on_host(lib):
    vp = ctypes.c_void_p
    d = ctypes.c_double
    lib.pa_fista_workspace_bytes.argtypes = [ctypes.POINTER(Geom), ctypes.c_int]
    lib.pa_fista_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_fista_solve.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, vp, vp, ctypes.c_int32, d, d, d, d, d,
                                   ctypes.c_int32, ctypes.c_uint32, vp, ctypes.c_size_t, vp, vp]
    g = good()
    n = lib.pa_fista_workspace_bytes(ctypes.byref(g), 0)
    P, M = 64 * 48, 32 * 300
    assert n >= 4 * (4 * P + 2 * M) and n > lib.pa_landweber_workspace_bytes(ctypes.byref(g), 0)

    def solve(it=5, lam=1e-3, al=1.0, be=1e-3, eps=1e-2, om=0.0, pw=30, flags=4, ws=1 << 32, wsb=n, geom=g):
        return lib.pa_fista_solve(ctypes.byref(geom), 0, 1 << 20, 1 << 24, it, lam, al, be, eps, om, pw, flags, ws,
                                  wsb, None, None)
    assert solve(it=-1) == 1
    assert solve(lam=-1.0) == 1
    assert solve(al=-1.0) == 1
    assert solve(al=float("nan")) == 1
    assert solve(be=-1.0) == 1
    assert solve(eps=0.0) == 1
    assert solve(om=-0.5) == 1
    assert solve(om=0.0, pw=0) == 1
    assert solve(flags=1) == 1          # PA_X0_ZERO is not a FISTA flag: it always starts from 0
    assert solve(flags=8) == 1
    assert solve(ws=None) == 3
    assert solve(wsb=n - 1) == 3
    assert solve(ws=(1 << 32) + 8) == 3
    # the TV term needs a 2D image; without it a volume is accepted up to the workspace check
    g3 = good()
    g3.ndim, g3.nz = 3, 8
    sens3 = (ctypes.c_double * (3 * 32))()
    g3.sensors = ctypes.cast(sens3, vp)
    assert solve(geom=g3, be=1e-3) == 2
    n3 = lib.pa_fista_workspace_bytes(ctypes.byref(g3), 0)
    assert n3 > 0 and solve(geom=g3, be=0.0, ws=None, wsb=n3) == 3


def test_dense_argument_checks_on_host(lib):
    vp = ctypes.c_void_p
    gp = ctypes.POINTER(Geom)
    lib.pa_dense_matrix_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_dense_matrix_bytes.restype = ctypes.c_size_t
    lib.pa_dense_adjoint_workspace_bytes.argtypes = [gp, ctypes.c_int]
    lib.pa_dense_adjoint_workspace_bytes.restype = ctypes.c_size_t
    lib.pa_dense_build.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp]
    lib.pa_dense_forward.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp, vp, vp]
    lib.pa_dense_adjoint.argtypes = [gp, ctypes.c_int, vp, ctypes.c_size_t, vp, vp, vp, ctypes.c_size_t, vp]
    g = good()
    M, P = 32 * 300, 64 * 48
    assert lib.pa_dense_matrix_bytes(ctypes.byref(g), 1) == M * P * 8        # P is a multiple of 32
    assert lib.pa_dense_matrix_bytes(ctypes.byref(g), 0) == M * P * 4
    g.nx = 63                                                                # ld rounds 63 * 48 up to 3040
    assert lib.pa_dense_matrix_bytes(ctypes.byref(g), 1) == M * 3040 * 8
    w = lib.pa_dense_adjoint_workspace_bytes(ctypes.byref(g), 1)
    assert w >= 8 * 3040 and w % (8 * 3040) == 0
    n = lib.pa_dense_matrix_bytes(ctypes.byref(g), 1)
    assert lib.pa_dense_build(ctypes.byref(g), 1, None, n, None) == 1
    assert lib.pa_dense_build(ctypes.byref(g), 1, (1 << 32) + 8, n, None) == 1      # alignment
    assert lib.pa_dense_build(ctypes.byref(g), 1, 1 << 32, n - 1, None) == 3
    assert lib.pa_dense_forward(ctypes.byref(g), 1, 1 << 36, n, None, 1 << 20, None) == 1
    assert lib.pa_dense_forward(ctypes.byref(g), 1, 1 << 36, n, 1 << 20, (1 << 36) + 64, None) == 1   # y inside A
    assert lib.pa_dense_adjoint(ctypes.byref(g), 1, 1 << 36, n, 1 << 20, 1 << 24, None, w, None) == 3
    assert lib.pa_dense_adjoint(ctypes.byref(g), 1, 1 << 36, n, 1 << 20, 1 << 24, 1 << 30, w - 8, None) == 3
    g.dt = -1.0
    assert lib.pa_dense_matrix_bytes(ctypes.byref(g), 1) == 0
    g = good()
    g.nx, g.ny, g.n_sensors, g.n_samples = 4096, 4096, 1024, 4096          # ~5e14 bytes
    assert lib.pa_dense_matrix_bytes(ctypes.byref(g), 1) == 0


def test_freq_argument_checks_on_host(lib):
    vp = ctypes.c_void_p
    d = ctypes.c_double
    gp = ctypes.POINTER(Geom)
    lib.pa_freq_workspace_bytes.argtypes = [gp, ctypes.c_int, ctypes.c_int32]
    lib.pa_freq_workspace_bytes.restype = ctypes.c_size_t
    for name in ("pa_freq_forward", "pa_freq_adjoint"):
        getattr(lib, name).argtypes = [gp, ctypes.c_int, d, d, ctypes.c_int32, vp, vp, vp, ctypes.c_size_t, vp]
    g = good()
    w = lib.pa_freq_workspace_bytes(ctypes.byref(g), 0, 256)
    # forward partials dominate here: 12 chunks of 256 pixels x 32 sensors x 256 frequencies, complex FP64
    assert w == 16 * 12 * 32 * 256
    assert lib.pa_freq_workspace_bytes(ctypes.byref(g), 0, -1) == 0
    assert lib.pa_freq_workspace_bytes(ctypes.byref(g), 0, 65537) == 0
    for fn in (lib.pa_freq_forward, lib.pa_freq_adjoint):
        assert fn(ctypes.byref(g), 0, -1.0, 1e5, 256, 1 << 20, 1 << 24, 1 << 30, w, None) == 1
        assert fn(ctypes.byref(g), 0, 1e5, float("inf"), 256, 1 << 20, 1 << 24, 1 << 30, w, None) == 1
        assert fn(ctypes.byref(g), 0, 1e5, 1e5, 256, None, 1 << 24, 1 << 30, w, None) == 1
        assert fn(ctypes.byref(g), 0, 1e5, 1e5, 256, 1 << 20, 1 << 24, None, w, None) == 3
        assert fn(ctypes.byref(g), 0, 1e5, 1e5, 256, 1 << 20, 1 << 24, 1 << 30, w - 8, None) == 3
        assert fn(ctypes.byref(g), 0, 1e5, 1e5, 256, 1 << 20, (1 << 20) + 64, 1 << 30, w, None) == 1   # x, Y overlap


def test_tuning_set_checks_on_host(lib):
    from paper_2404_10928_amd._lib import PaTuning
    lib.pa_tuning_set.argtypes = [ctypes.POINTER(Geom), ctypes.c_int, ctypes.POINTER(PaTuning)]
    lib.pa_forward_workspace_bytes.argtypes = [ctypes.POINTER(Geom), ctypes.c_int]
    lib.pa_forward_workspace_bytes.restype = ctypes.c_size_t
    g = good()
    t = PaTuning()
    try:
        assert lib.pa_tuning_set(ctypes.byref(g), 0, None) == 1
        t.fwd_mode = 4
        assert lib.pa_tuning_set(ctypes.byref(g), 0, ctypes.byref(t)) == 1
        t.fwd_mode = 3                       # partial rows need a tile
        assert lib.pa_tuning_set(ctypes.byref(g), 0, ctypes.byref(t)) == 1
        t.fwd_tile[0], t.fwd_tile[1], t.fwd_tile[2] = 2, 2, 1
        assert lib.pa_tuning_set(ctypes.byref(g), 1, ctypes.byref(t)) == 2   # PA_F32 only
        assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 0) == 0
        assert lib.pa_tuning_set(ctypes.byref(g), 0, ctypes.byref(t)) == 0
        # now the partial-row forward is planned, and it needs a workspace
        n = lib.pa_forward_workspace_bytes(ctypes.byref(g), 0)
        assert n >= 64 * 48 * 4
        t.fwd_tile[2] = 2                    # a 2D geometry has one tile along z
        assert lib.pa_tuning_set(ctypes.byref(g), 0, ctypes.byref(t)) == 2
        assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 0) == n       # unchanged after a refusal
    finally:
        assert lib.pa_tuning_clear() == 0
    assert lib.pa_forward_workspace_bytes(ctypes.byref(g), 0) == 0
