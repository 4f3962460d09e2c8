"""Python entry points over the C ABI: forward (A), adjoint (A^T) and CGLS.

Argument marshalling only: tensors must already live on the HIP device; the
kernels run on the current torch stream.  Image tensors have shape
(ny, nx) or (nz, ny, nx) (or flat), measurement tensors (S, K); float32 selects
PA_F32, float64 selects PA_F64.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


class DeviceGeometry:
    """Grid, sensor array and timing, with the sensor table on the device.

    Accepts any object exposing ndim, nx, ny, nz, h, center, sensors
    ([S][ndim] metres), n_samples, dt, t0, c, r_min.
    """

    def __init__(self, g, device=None):
        device = torch.device("cuda") if device is None else torch.device(device)
        self.ndim = int(g.ndim)
        self.nx, self.ny, self.nz = int(g.nx), int(g.ny), int(g.nz)
        self.h = float(g.h)
        ctr = list(g.center) + [0.0] * (3 - len(g.center))
        self.center = tuple(float(v) for v in ctr[:3])
        sens = g.sensors
        if not isinstance(sens, torch.Tensor):
            sens = torch.from_numpy(np.ascontiguousarray(np.asarray(sens, dtype=np.float64)))
        self.sensors = sens.to(device=device, dtype=torch.float64).contiguous().reshape(-1, self.ndim)
        self.n_samples = int(g.n_samples)
        self.dt, self.t0, self.c, self.r_min = float(g.dt), float(g.t0), float(g.c), float(g.r_min)
        self.device = device

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

    def c_struct(self) -> _lib.PaGeometry:
        s = _lib.PaGeometry()
        s.ndim, s.nx, s.ny, s.nz = self.ndim, self.nx, self.ny, self.nz
        s.h = self.h
        s.center = (ctypes.c_double * 3)(*self.center)
        s.n_sensors = self.n_sensors
        s.sensors = self.sensors.data_ptr() if self.n_sensors else None
        s.n_samples = self.n_samples
        s.dt, s.t0, s.c, s.r_min = self.dt, self.t0, self.c, self.r_min
        return s


def as_device_geometry(g, device=None) -> DeviceGeometry:
    return g if isinstance(g, DeviceGeometry) else DeviceGeometry(g, device)


PRECISIONS = ("f32", "f64", "mixed")


def dtype_code(dtype: torch.dtype, precision: str | None = None) -> int:
    """The C ABI's dtype for tensors of `dtype`: float32 -> PA_F32, float64 ->
    PA_F64; precision="mixed" (float64 tensors) -> PA_MIXED, FP32 delay
    arithmetic with every vector and sum in FP64."""
    if precision is not None and precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {PRECISIONS}")
    if dtype == torch.float32:
        if precision not in (None, "f32"):
            raise TypeError(f"precision {precision!r} needs float64 tensors")
        return _lib.PA_F32
    if dtype == torch.float64:
        if precision == "f32":
            raise TypeError("precision 'f32' needs float32 tensors")
        return _lib.PA_MIXED if precision == "mixed" else _lib.PA_F64
    raise TypeError(f"unsupported dtype {dtype}; use float32 or float64")


def _code(t: torch.Tensor, precision: str | None = None) -> int:
    return dtype_code(t.dtype, precision)


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _check_tensor(t: torch.Tensor, numel: int, name: str):
    if not (t.is_cuda or t.numel() == 0):
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _frames(t: torch.Tensor, per: int):
    """Split a contiguous tensor into frames of `per` elements (one frame if it holds exactly one)."""
    if per == 0:
        return [t.reshape(-1)], ()
    if t.numel() % per != 0:
        raise ValueError(f"tensor with {t.numel()} elements is not a whole number of frames of {per}")
    nb = t.numel() // per
    return list(t.reshape(nb, per)), nb


_BATCHES: dict = {}


def _frames_batch(g: "DeviceGeometry", n: int, dtype: torch.dtype, precision: str | None = None) -> "Batch":
    """A cached batch of n copies of one geometry (frames of a leading batch dimension)."""
    key = (id(g), n, dtype, precision)
    b = _BATCHES.get(key)
    if b is None or b.geoms[0] is not g:
        if len(_BATCHES) > 32:
            _BATCHES.clear()
        b = _BATCHES[key] = Batch([g] * n, dtype, g.device, precision=precision)
    return b


def forward(x: torch.Tensor, geom, out: torch.Tensor | None = None, precision: str | None = None) -> torch.Tensor:
    """y := A x.  Leading batch dimensions of x are frames, applied in one
    batched launch per pass (the single-frame result for every frame)."""
    g = as_device_geometry(geom, x.device)
    P, M = g.n_pixels, g.n_sensors * g.n_samples
    x = x.contiguous()
    batch = tuple(x.shape[: x.dim() - len(g.image_shape)]) if x.dim() > len(g.image_shape) else ()
    if out is None:
        out = torch.empty(batch + g.data_shape, dtype=x.dtype, device=x.device)
    _check_tensor(out, out.numel(), "y")
    xs, nb = _frames(x, P)
    ys, nb2 = _frames(out, M) if M else ([out.reshape(-1)] * len(xs), nb)
    if M and len(xs) != len(ys):
        raise ValueError("x and y hold different numbers of frames")
    if len(xs) > 1 and P and M:
        _frames_batch(g, len(xs), x.dtype, precision).forward(x.reshape(-1), out.reshape(-1))
        return out
    lib = _lib.load()
    cg = g.c_struct()
    code = _code(x, precision)
    ws = _forward_workspace(lib, cg, code, x.device)
    for xb, yb in zip(xs, ys):
        _lib.check(lib.pa_forward_ws(ctypes.byref(cg), code, xb.data_ptr() or None, yb.data_ptr() or None,
                                     ws.data_ptr() if ws is not None else None, ws.numel() if ws is not None else 0,
                                     _stream(x.device)))
    return out


def _forward_workspace(lib, cg, code, device):
    """A torch-owned workspace for pa_forward_ws (None when the plan needs none)."""
    n = int(lib.pa_forward_workspace_bytes(ctypes.byref(cg), code))
    if n == 0:
        _lib.check(lib.pa_validate_geometry(ctypes.byref(cg), code))
        return None
    return torch.empty(n, dtype=torch.uint8, device=device)


def adjoint(y: torch.Tensor, geom, out: torch.Tensor | None = None, precision: str | None = None) -> torch.Tensor:
    """x := A^T y.  Leading batch dimensions of y are frames, applied in one
    batched launch (the single-frame result for every frame)."""
    g = as_device_geometry(geom, y.device)
    P, M = g.n_pixels, g.n_sensors * g.n_samples
    y = y.contiguous()
    batch = tuple(y.shape[:-2]) if y.dim() > 2 else ()
    if out is None:
        out = torch.empty(batch + g.image_shape, dtype=y.dtype, device=y.device)
    _check_tensor(out, out.numel(), "x")
    ys, nb = _frames(y, M)
    xs, nb2 = _frames(out, P) if P else ([out.reshape(-1)] * len(ys), nb)
    if P and len(xs) != len(ys):
        raise ValueError("x and y hold different numbers of frames")
    if len(ys) > 1 and P and M:
        _frames_batch(g, len(ys), y.dtype, precision).adjoint(y.reshape(-1), out.reshape(-1))
        return out
    lib = _lib.load()
    cg = g.c_struct()
    for yb, xb in zip(ys, xs):
        _lib.check(lib.pa_adjoint(ctypes.byref(cg), _code(y, precision), yb.data_ptr() or None,
                                  xb.data_ptr() or None, _stream(y.device)))
    return out


class Operator:
    """A and A^T on one geometry with the argument struct built once (low call overhead).

    forward_(x, y) and adjoint_(y, x) write into preallocated contiguous device
    tensors of the operator's dtype and skip the shape bookkeeping of
    forward()/adjoint().
    """

    def __init__(self, geom, dtype: torch.dtype = torch.float32, device=None, precision: str | None = None):
        self.geom = as_device_geometry(geom, device)
        self.dtype = dtype
        self._code = dtype_code(dtype, precision)
        self._cg = self.geom.c_struct()
        self._ref = ctypes.byref(self._cg)
        self._lib = _lib.load()
        _lib.check(self._lib.pa_validate_geometry(self._ref, self._code))
        self._ws = None

    def forward_(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        n = int(self._lib.pa_forward_workspace_bytes(self._ref, self._code))   # follows later tunings
        if n > (0 if self._ws is None else self._ws.numel()):
            self._ws = torch.empty(n, dtype=torch.uint8, device=self.geom.device)
        ws = self._ws
        _lib.check(self._lib.pa_forward_ws(self._ref, self._code, x.data_ptr() or None, y.data_ptr() or None,
                                           ws.data_ptr() if (n and ws is not None) else None, n,
                                           torch.cuda.current_stream(x.device).cuda_stream))
        return y

    def forward_no_workspace_(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        """y := A x through pa_forward (the sensor-major method, no workspace)."""
        _lib.check(self._lib.pa_forward(self._ref, self._code, x.data_ptr() or None, y.data_ptr() or None,
                                        torch.cuda.current_stream(x.device).cuda_stream))
        return y

    def adjoint_(self, y: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
        _lib.check(self._lib.pa_adjoint(self._ref, self._code, y.data_ptr() or None, x.data_ptr() or None,
                                        torch.cuda.current_stream(y.device).cuda_stream))
        return x


def cgls_workspace_bytes(geom, dtype: torch.dtype, iters: int, precision: str | None = None) -> int:
    g = as_device_geometry(geom)
    lib = _lib.load()
    code = dtype_code(dtype, precision)
    n = lib.pa_cgls_workspace_bytes(ctypes.byref(g.c_struct()), code, int(iters))
    if n == 0:
        raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
    return int(n)


class CglsSolver:
    """Owns the device workspace and history of repeated solves on one geometry."""

    def __init__(self, geom, dtype: torch.dtype, iters: int, lam: float, graph: bool = True, device=None,
                 precision: str | None = None):
        self.geom = as_device_geometry(geom, device)
        self.dtype = dtype
        self.precision = precision
        self._code = dtype_code(dtype, precision)
        self.iters = int(iters)
        self.lam = float(lam)
        self.graph = graph
        dev = self.geom.device
        nbytes = cgls_workspace_bytes(self.geom, dtype, self.iters, precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.history = torch.zeros((self.iters + 1, 3), dtype=torch.float64, device=dev)
        self._cg = self.geom.c_struct()

    def solve(self, y: torch.Tensor, x: torch.Tensor | None = None, x0_zero: bool = True) -> torch.Tensor:
        g = self.geom
        if x is None:
            x = torch.empty(g.image_shape, dtype=self.dtype, device=y.device)
            x0_zero = True
        _check_tensor(y, g.n_sensors * g.n_samples, "y")
        _check_tensor(x, g.n_pixels, "x")
        if y.dtype != self.dtype or x.dtype != self.dtype:
            raise TypeError("y and x must match the solver dtype")
        flags = (_lib.PA_X0_ZERO if x0_zero else 0) | (_lib.PA_USE_GRAPH if self.graph else 0)
        lib = _lib.load()
        _lib.check(lib.pa_cgls_solve(ctypes.byref(self._cg), self._code, y.data_ptr() or None, x.data_ptr() or None,
                                     self.iters, self.lam, flags, self.workspace.data_ptr(),
                                     self.workspace.numel(), self.history.data_ptr(), _stream(y.device)))
        return x

    def stop_iteration(self) -> int:
        """-1 if the last solve ran every iteration, else the iteration it stopped at (synchronises)."""
        torch.cuda.synchronize(self.geom.device)
        out = ctypes.c_int32(-1)
        _lib.check(_lib.load().pa_cgls_stop_iteration(self.workspace.data_ptr(), ctypes.byref(out)),
                   allow=(_lib.PA_OK, _lib.PA_ERR_BREAKDOWN))
        return int(out.value)


def cgls(y: torch.Tensor, geom, iters: int, lam: float, x0: torch.Tensor | None = None, graph: bool = True,
         precision: str | None = None):
    """CGLS on ||A x - y||^2 + lam ||x||^2.  Returns (x, history[iters+1][3], stop_iteration).
    precision="mixed" (float64 y): FP64 vectors and sums around the FP32-arithmetic operator."""
    solver = CglsSolver(geom, y.dtype, iters, lam, graph=graph, device=y.device, precision=precision)
    if x0 is None:
        x = solver.solve(y.contiguous())
    else:
        x = x0.detach().clone().contiguous()
        solver.solve(y.contiguous(), x, x0_zero=False)
    stop = solver.stop_iteration()
    return x, solver.history.clone(), stop


class Batch:
    """Many frames of uneven size under one plan: one launch per step for all frames.

    geoms: frame geometries (objects accepted by DeviceGeometry), all with the
    same ndim.  Packed buffers hold the frames one after another in the given
    order; `x_offsets` / `y_offsets` (length n + 1) give each frame's element
    range, and pack_x / unpack_x / pack_y / unpack_y convert from and to
    per-frame tensors.
    """

    def __init__(self, geoms, dtype: torch.dtype = torch.float32, device=None, precision: str | None = None):
        self.geoms = [as_device_geometry(g, device) for g in geoms]
        if not self.geoms:
            raise ValueError("a batch needs at least one frame")
        self.device = self.geoms[0].device
        self.dtype = dtype
        self._code = dtype_code(dtype, precision)
        self._structs = (_lib.PaGeometry * len(self.geoms))(*[g.c_struct() for g in self.geoms])
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self._lib.pa_batch_create(self._structs, len(self.geoms), self._code, ctypes.byref(h)))
        self._h = h
        n = len(self.geoms)
        xo = (ctypes.c_int64 * (n + 1))()
        yo = (ctypes.c_int64 * (n + 1))()
        _lib.check(self._lib.pa_batch_offsets(self._h, xo, yo))
        self.x_offsets = [int(v) for v in xo]
        self.y_offsets = [int(v) for v in yo]
        self._ws = None
        self._ws_cg = {}
        self.history = None

    def __len__(self):
        return len(self.geoms)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            torch.cuda.synchronize(self.device)
            self._lib.pa_batch_destroy(h)
            self._h = None

    # packing helpers (torch copies; no arithmetic)
    def pack_x(self, xs):
        return torch.cat([x.reshape(-1).to(self.dtype) for x in xs]).contiguous()

    def pack_y(self, ys):
        return torch.cat([y.reshape(-1).to(self.dtype) for y in ys]).contiguous()

    def unpack_x(self, x):
        return [x[self.x_offsets[i]:self.x_offsets[i + 1]].reshape(g.image_shape) for i, g in enumerate(self.geoms)]

    def unpack_y(self, y):
        return [y[self.y_offsets[i]:self.y_offsets[i + 1]].reshape(g.data_shape) for i, g in enumerate(self.geoms)]

    def _workspace(self):
        if self._ws is None:
            n = self._lib.pa_batch_workspace_bytes(self._h)
            self._ws = torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def _check(self, t, n, name):
        _check_tensor(t, n, name)
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}")

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Packed y := A x, frame by frame."""
        self._check(x, self.x_offsets[-1], "x")
        if out is None:
            out = torch.empty(self.y_offsets[-1], dtype=self.dtype, device=self.device)
        self._check(out, self.y_offsets[-1], "y")
        ws = self._workspace()
        _lib.check(self._lib.pa_batch_forward(self._h, x.data_ptr() or None, out.data_ptr() or None, ws.data_ptr(),
                                              ws.numel(), _stream(self.device)))
        return out

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Packed x := A^T y, frame by frame."""
        self._check(y, self.y_offsets[-1], "y")
        if out is None:
            out = torch.empty(self.x_offsets[-1], dtype=self.dtype, device=self.device)
        self._check(out, self.x_offsets[-1], "x")
        ws = self._workspace()
        _lib.check(self._lib.pa_batch_adjoint(self._h, y.data_ptr() or None, out.data_ptr() or None, ws.data_ptr(),
                                              ws.numel(), _stream(self.device)))
        return out

    def cgls(self, y: torch.Tensor, iters: int, lam: float, x: torch.Tensor | None = None, x0_zero: bool = True,
             graph: bool = True) -> torch.Tensor:
        """CGLS on every frame; x (packed) is the start (unless x0_zero) and the result.
        self.history becomes [n_frames][iters + 1][3] (||r_k||, ||s_k||, F_k) on the device."""
        iters = int(iters)
        self._check(y, self.y_offsets[-1], "y")
        if x is None:
            x = torch.empty(self.x_offsets[-1], dtype=self.dtype, device=self.device)
            x0_zero = True
        self._check(x, self.x_offsets[-1], "x")
        ws = self._ws_cg.get(iters)
        if ws is None:
            n = self._lib.pa_batch_cgls_workspace_bytes(self._h, iters)
            if n == 0:
                raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
            ws = self._ws_cg[iters] = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        if self.history is None or self.history.shape != (len(self), iters + 1, 3):
            self.history = torch.zeros((len(self), iters + 1, 3), dtype=torch.float64, device=self.device)
        flags = (_lib.PA_X0_ZERO if x0_zero else 0) | (_lib.PA_USE_GRAPH if graph else 0)
        _lib.check(self._lib.pa_batch_cgls_solve(self._h, y.data_ptr() or None, x.data_ptr() or None, iters,
                                                 float(lam), flags, ws.data_ptr(), ws.numel(),
                                                 self.history.data_ptr(), _stream(self.device)))
        self._last_iters = iters
        return x

    def autotune(self) -> bool:
        """Times the batched operators under rule plans and under the frames'
        recorded tunings and keeps the faster; True if the tuned plans won."""
        n = int(self._lib.pa_batch_autotune_workspace_bytes(self._h))
        if n == 0:
            raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
        ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        x = torch.zeros(self.x_offsets[-1], dtype=self.dtype, device=self.device)
        y = torch.zeros(self.y_offsets[-1], dtype=self.dtype, device=self.device)
        out = ctypes.c_int32(0)
        _lib.check(self._lib.pa_batch_autotune(self._h, x.data_ptr() or None, y.data_ptr() or None, ws.data_ptr(),
                                               ws.numel(), _stream(self.device), ctypes.byref(out)))
        self._ws = None       # the plan may need other workspace sizes now
        self._ws_cg = {}
        return bool(out.value)

    def stop_iterations(self) -> list:
        """Per frame: the iteration its last solve stopped at, or -1 (synchronises)."""
        torch.cuda.synchronize(self.device)
        iters = self._last_iters
        out = (ctypes.c_int32 * len(self))()
        _lib.check(self._lib.pa_batch_stop_iterations(self._h, self._ws_cg[iters].data_ptr(), iters, out),
                   allow=(_lib.PA_OK, _lib.PA_ERR_BREAKDOWN))
        return [int(v) for v in out]


def autotune(geom, dtype: torch.dtype = torch.float32, device=None, precision: str | None = None) -> dict:
    """Times the candidate tilings of A and A^T on this geometry and records the
    fastest for every later plan of the same shape (process-wide).  Returns the
    choice and its measured times."""
    g = as_device_geometry(geom, device)
    x = torch.zeros(g.image_shape, dtype=dtype, device=g.device)
    y = torch.zeros(g.data_shape, dtype=dtype, device=g.device)
    t = _lib.PaTuning()
    lib = _lib.load()
    cg = g.c_struct()
    code = _code(x, precision)
    n = int(lib.pa_autotune_workspace_bytes(ctypes.byref(cg), code))
    ws = torch.empty(n, dtype=torch.uint8, device=g.device) if n else None
    _lib.check(lib.pa_autotune(ctypes.byref(cg), code, x.data_ptr() or None, y.data_ptr() or None,
                               ws.data_ptr() if ws is not None else None, n, _stream(g.device), ctypes.byref(t)))
    return {"fwd_seg": int(t.fwd_seg), "fwd_mode": int(t.fwd_mode), "fwd_tile": tuple(int(v) for v in t.fwd_tile),
            "adj_lds_bytes": int(t.adj_lds_bytes),
            "fwd_us": float(t.fwd_us), "adj_us": float(t.adj_us)}


def tuning_set(geom, tuning: dict, dtype: torch.dtype = torch.float32, device=None,
               precision: str | None = None) -> None:
    """Records a tuning for this geometry's shape (e.g. a dict autotune returned
    in an earlier process); missing keys keep the planner's rule."""
    g = as_device_geometry(geom, device)
    t = _lib.PaTuning()
    t.fwd_seg = int(tuning.get("fwd_seg", 0))
    t.fwd_mode = int(tuning.get("fwd_mode", 0))
    for a, v in enumerate(tuning.get("fwd_tile", (0, 0, 0))):
        t.fwd_tile[a] = int(v)
    t.adj_lds_bytes = int(tuning.get("adj_lds_bytes", 0))
    cg = g.c_struct()
    _lib.check(_lib.load().pa_tuning_set(ctypes.byref(cg), dtype_code(dtype, precision), ctypes.byref(t)))


def tuning_clear() -> None:
    """Forgets every recorded tiling."""
    _lib.check(_lib.load().pa_tuning_clear())


class LandweberSolver:
    """Workspace and history of repeated Landweber solves on one geometry.

    omega > 0 fixes the step; omega == 0 estimates it on the GPU with
    power_iters power-iteration steps (omega = 1 / (sigma2 + lam))."""

    def __init__(self, geom, dtype: torch.dtype, iters: int, lam: float, omega: float = 0.0, power_iters: int = 30,
                 graph: bool = True, device=None, precision: str | None = None):
        self.geom = as_device_geometry(geom, device)
        self.dtype = dtype
        self.iters, self.lam, self.omega, self.power_iters = int(iters), float(lam), float(omega), int(power_iters)
        self.graph = graph
        self._code = dtype_code(dtype, precision)
        self._cg = self.geom.c_struct()
        lib = _lib.load()
        n = lib.pa_landweber_workspace_bytes(ctypes.byref(self._cg), self._code)
        if n == 0:
            raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
        self.workspace = torch.empty(int(n), dtype=torch.uint8, device=self.geom.device)
        self.history = torch.zeros(self.iters + 1, dtype=torch.float64, device=self.geom.device)

    def solve(self, y: torch.Tensor, x: torch.Tensor | None = None, x0_zero: bool = True) -> torch.Tensor:
        g = self.geom
        if x is None:
            x = torch.empty(g.image_shape, dtype=self.dtype, device=y.device)
            x0_zero = True
        _check_tensor(y, g.n_sensors * g.n_samples, "y")
        _check_tensor(x, g.n_pixels, "x")
        if y.dtype != self.dtype or x.dtype != self.dtype:
            raise TypeError("y and x must match the solver dtype")
        flags = (_lib.PA_X0_ZERO if x0_zero else 0) | (_lib.PA_USE_GRAPH if self.graph else 0)
        _lib.check(_lib.load().pa_landweber_solve(ctypes.byref(self._cg), self._code, y.data_ptr() or None,
                                                  x.data_ptr() or None, self.iters, self.lam, self.omega,
                                                  self.power_iters, flags, self.workspace.data_ptr(),
                                                  self.workspace.numel(), self.history.data_ptr(),
                                                  _stream(y.device)))
        return x

    def step(self):
        """(omega used, sigma2 estimate) of the last solve (synchronises)."""
        torch.cuda.synchronize(self.geom.device)
        om, s2 = ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().pa_landweber_step(self.workspace.data_ptr(), ctypes.byref(om), ctypes.byref(s2)))
        return om.value, s2.value


def landweber(y: torch.Tensor, geom, iters: int, lam: float, omega: float = 0.0, power_iters: int = 30,
              x0: torch.Tensor | None = None, graph: bool = True):
    """Landweber on ||A x - y||^2 + lam ||x||^2.  Returns (x, history[iters+1], omega, sigma2)."""
    sv = LandweberSolver(geom, y.dtype, iters, lam, omega, power_iters, graph=graph, device=y.device)
    if x0 is None:
        x = sv.solve(y.contiguous())
    else:
        x = x0.detach().clone().contiguous()
        sv.solve(y.contiguous(), x, x0_zero=False)
    om, s2 = sv.step()
    return x, sv.history.clone(), om, s2


class FistaSolver:
    """Workspace and history of repeated FISTA solves of
    ||A x - y||^2 + lam ||x||^2 + beta TV_eps(x) + alpha ||x||_1 on one geometry.

    omega > 0 fixes the step; omega == 0 estimates it on the GPU with
    power_iters power-iteration steps (omega = 1 / (sigma2 + lam + 4 beta / eps)).
    nonneg adds the constraint x >= 0.  history[k] = F(z_k) for k < iters and
    F(x_iters) last."""

    def __init__(self, geom, dtype: torch.dtype, iters: int, lam: float, alpha: float, beta: float,
                 eps: float = 1e-2, omega: float = 0.0, power_iters: int = 30, nonneg: bool = False,
                 graph: bool = True, device=None, precision: str | None = None):
        self.geom = as_device_geometry(geom, device)
        self.dtype = dtype
        self.iters, self.lam, self.alpha, self.beta = int(iters), float(lam), float(alpha), float(beta)
        self.eps, self.omega, self.power_iters = float(eps), float(omega), int(power_iters)
        self.nonneg, self.graph = bool(nonneg), graph
        self._code = dtype_code(dtype, precision)
        self._cg = self.geom.c_struct()
        lib = _lib.load()
        n = lib.pa_fista_workspace_bytes(ctypes.byref(self._cg), self._code)
        if n == 0:
            raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
        self.workspace = torch.empty(int(n), dtype=torch.uint8, device=self.geom.device)
        self.history = torch.zeros(self.iters + 1, dtype=torch.float64, device=self.geom.device)

    def solve(self, y: torch.Tensor, x: torch.Tensor | None = None) -> torch.Tensor:
        g = self.geom
        if x is None:
            x = torch.empty(g.image_shape, dtype=self.dtype, device=y.device)
        _check_tensor(y, g.n_sensors * g.n_samples, "y")
        _check_tensor(x, g.n_pixels, "x")
        if y.dtype != self.dtype or x.dtype != self.dtype:
            raise TypeError("y and x must match the solver dtype")
        flags = (_lib.PA_NONNEG if self.nonneg else 0) | (_lib.PA_USE_GRAPH if self.graph else 0)
        _lib.check(_lib.load().pa_fista_solve(ctypes.byref(self._cg), self._code, y.data_ptr() or None,
                                              x.data_ptr() or None, self.iters, self.lam, self.alpha, self.beta,
                                              self.eps, self.omega, self.power_iters, flags,
                                              self.workspace.data_ptr(), self.workspace.numel(),
                                              self.history.data_ptr(), _stream(y.device)))
        return x

    def step(self):
        """(omega used, sigma2 estimate) of the last solve (synchronises)."""
        torch.cuda.synchronize(self.geom.device)
        om, s2 = ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().pa_fista_step(self.workspace.data_ptr(), ctypes.byref(om), ctypes.byref(s2)))
        return om.value, s2.value


def fista(y: torch.Tensor, geom, iters: int, lam: float, alpha: float, beta: float, eps: float = 1e-2,
          omega: float = 0.0, power_iters: int = 30, nonneg: bool = False, graph: bool = True):
    """FISTA on the l1 + TV objective from x0 = 0.  Returns (x, history[iters+1], omega, sigma2)."""
    sv = FistaSolver(geom, y.dtype, iters, lam, alpha, beta, eps, omega, power_iters, nonneg, graph=graph,
                     device=y.device)
    x = sv.solve(y.contiguous())
    om, s2 = sv.step()
    return x, sv.history.clone(), om, s2


class DenseMatrix:
    """The dense time-domain matrix of a geometry (the paper's kn), built on
    the GPU and applied by HBM-bound matrix-vector products.  Holds
    S * K * round_up(P, 32) elements of device memory."""

    def __init__(self, geom, dtype: torch.dtype = torch.float64, device=None):
        self.geom = as_device_geometry(geom, device)
        self.dtype = dtype
        self._code = _lib.PA_F32 if dtype == torch.float32 else _lib.PA_F64
        self._cg = self.geom.c_struct()
        lib = _lib.load()
        n = lib.pa_dense_matrix_bytes(ctypes.byref(self._cg), self._code)
        if n == 0:
            raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
        w = lib.pa_dense_adjoint_workspace_bytes(ctypes.byref(self._cg), self._code)
        self.matrix = torch.empty(int(n), dtype=torch.uint8, device=self.geom.device)
        self.workspace = torch.empty(int(w), dtype=torch.uint8, device=self.geom.device)
        self.ld = (self.geom.n_pixels + 31) // 32 * 32
        _lib.check(lib.pa_dense_build(ctypes.byref(self._cg), self._code, self.matrix.data_ptr(), self.matrix.numel(),
                                      _stream(self.geom.device)))

    def view(self) -> torch.Tensor:
        """The matrix as a [S*K][ld] tensor (a view of the same memory)."""
        g = self.geom
        return self.matrix.view(self.dtype).view(g.n_sensors * g.n_samples, self.ld)

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        g = self.geom
        _check_tensor(x, g.n_pixels, "x")
        if x.dtype != self.dtype:
            raise TypeError("x must match the matrix dtype")
        y = torch.empty(g.data_shape, dtype=self.dtype, device=x.device) if out is None else out
        _check_tensor(y, g.n_sensors * g.n_samples, "y")
        _lib.check(_lib.load().pa_dense_forward(ctypes.byref(self._cg), self._code, self.matrix.data_ptr(),
                                                self.matrix.numel(), x.data_ptr() or None, y.data_ptr() or None,
                                                _stream(x.device)))
        return y

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        g = self.geom
        _check_tensor(y, g.n_sensors * g.n_samples, "y")
        if y.dtype != self.dtype:
            raise TypeError("y must match the matrix dtype")
        x = torch.empty(g.image_shape, dtype=self.dtype, device=y.device) if out is None else out
        _check_tensor(x, g.n_pixels, "x")
        _lib.check(_lib.load().pa_dense_adjoint(ctypes.byref(self._cg), self._code, self.matrix.data_ptr(),
                                                self.matrix.numel(), y.data_ptr() or None, x.data_ptr() or None,
                                                self.workspace.data_ptr(), self.workspace.numel(),
                                                _stream(y.device)))
        return x


class FreqOperator:
    """The frequency-domain matrix of Eq. 7 on one geometry and frequency grid
    f_n = f0 + n df (n < nf): forward(x) -> complex Y [S][nf] (stored as real
    pairs), adjoint(Y) -> x = Re(K^H Y)."""

    def __init__(self, geom, f0: float, df: float, nf: int, dtype: torch.dtype = torch.float32, device=None):
        self.geom = as_device_geometry(geom, device)
        self.f0, self.df, self.nf = float(f0), float(df), int(nf)
        self.dtype = dtype
        self._code = _lib.PA_F32 if dtype == torch.float32 else _lib.PA_F64
        self._cg = self.geom.c_struct()
        n = _lib.load().pa_freq_workspace_bytes(ctypes.byref(self._cg), self._code, self.nf)
        if n == 0:
            raise _lib.PaError(_lib.PA_ERR_INVALID_ARGUMENT, _lib.last_error())
        self.workspace = torch.empty(int(n), dtype=torch.uint8, device=self.geom.device)

    @property
    def data_shape(self):
        return (self.geom.n_sensors, self.nf, 2)

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Y as a real tensor [S][nf][2] (torch.view_as_complex gives the complex view)."""
        g = self.geom
        _check_tensor(x, g.n_pixels, "x")
        if x.dtype != self.dtype:
            raise TypeError("x must match the operator dtype")
        Y = torch.empty(self.data_shape, dtype=self.dtype, device=x.device) if out is None else out
        _check_tensor(Y, 2 * g.n_sensors * self.nf, "Y")
        _lib.check(_lib.load().pa_freq_forward(ctypes.byref(self._cg), self._code, self.f0, self.df, self.nf,
                                               x.data_ptr() or None, Y.data_ptr() or None, self.workspace.data_ptr(),
                                               self.workspace.numel(), _stream(x.device)))
        return Y

    def adjoint(self, Y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        g = self.geom
        _check_tensor(Y, 2 * g.n_sensors * self.nf, "Y")
        if Y.dtype != self.dtype:
            raise TypeError("Y must match the operator dtype")
        x = torch.empty(g.image_shape, dtype=self.dtype, device=Y.device) if out is None else out
        _check_tensor(x, g.n_pixels, "x")
        _lib.check(_lib.load().pa_freq_adjoint(ctypes.byref(self._cg), self._code, self.f0, self.df, self.nf,
                                               Y.data_ptr() or None, x.data_ptr() or None, self.workspace.data_ptr(),
                                               self.workspace.numel(), _stream(Y.device)))
        return x
