"""GPU parity of the operator kernels against the FP64 oracle.

Gates: PA_F32 within 1e-5 relative L2 per apply, PA_F64 within 1e-12; the
oracle always sees the exact FP64 value of the input the GPU used.
"""
import math

import numpy as np
import pytest

import oracle
from golden_cases import load_point_sources
from gpu_common import hemi_geom, rel_l2, ring_geom, rounded
from synth import Geometry, make_config, ring_sensors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F32_GATE = 1e-5
F64_GATE = 1e-12


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


def run_forward(pa, g, x, dtype):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    y = pa.forward(xt, g)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def run_adjoint(pa, g, y, dtype):
    yt = torch.from_numpy(np.ascontiguousarray(y)).to("cuda")
    x = pa.adjoint(yt, g)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64)


def check_pair(pa, g, seed, dtypes=(np.float32, np.float64), label=""):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=g.image_shape)
    y = rng.normal(size=g.data_shape)
    out = {}
    for dt in dtypes:
        gate = F32_GATE if dt == np.float32 else F64_GATE
        xg, x64 = rounded(x, dt)
        yg, y64 = rounded(y, dt)
        yf = run_forward(pa, g, xg, dt)
        xa = run_adjoint(pa, g, yg, dt)
        ef = rel_l2(yf, oracle.forward(g, x64))
        ea = rel_l2(xa, oracle.adjoint(g, y64))
        print(f"{label} {np.dtype(dt).name}: forward {ef:.3e} adjoint {ea:.3e}", flush=True)
        assert ef <= gate, f"forward rel-L2 {ef:.3e} > {gate}"
        assert ea <= gate, f"adjoint rel-L2 {ea:.3e} > {gate}"
        out[np.dtype(dt).name] = (ef, ea)
    return out


# ----------------------------------------------------------------- small cases

def test_ragged_2d(pa):
    check_pair(pa, ring_geom(), 1, label="ragged 2D 37x29 S70 K300")


def test_ragged_2d_sensor_count_not_multiple_of_64(pa):
    check_pair(pa, ring_geom(n=(50, 17), S=129, K=211), 2, label="2D 50x17 S129")


def test_ragged_3d(pa):
    check_pair(pa, hemi_geom(), 3, label="ragged 3D 19x13x11 S90")


@pytest.mark.parametrize("t0", [0.37e-7, -2.5e-7, 3 * 2.5e-8])
def test_time_origin(pa, t0):
    g = ring_geom(n=(40, 33), S=48, K=260, t0=t0)
    check_pair(pa, g, 4, label=f"t0={t0}")


def test_sensors_inside_grid_clamp(pa):
    # ring radius smaller than the half-width: some sensors sit among the pixels
    g = ring_geom(n=(64, 64), S=96, K=400, radius=2.5e-3)
    check_pair(pa, g, 5, label="inside")
    # a sensor exactly on a pixel centre (distance 0, clamped to h/2)
    sens = np.array([[0.5e-4, 0.5e-4], [1.2e-3, -0.3e-3]])
    g2 = ring_geom(n=(32, 32), S=2, K=300).replace(sensors=sens)
    check_pair(pa, g2, 6, label="on-pixel")


def test_large_distance_clamp(pa):
    # r_min of many pixels: every clamped pair must take the FP64 near path
    g = ring_geom(n=(64, 64), S=96, K=400, radius=2.5e-3, r_min=8e-4)
    check_pair(pa, g, 15, label="r_min 8 px")


def test_late_arrivals_dropped(pa):
    g = ring_geom(n=(48, 40), S=64, K=200)
    g = g.replace(dt=g.dt * 0.6)   # far edge arrives after the trace ends
    check_pair(pa, g, 7, label="truncated")


def test_coarse_and_fine_pitch(pa):
    # many samples per pixel (h / (c dt) ~ 13, near the largest pitch the
    # forward histogram window supports) and a fraction of a sample per pixel
    g = ring_geom(n=(30, 30), S=40, K=600)
    assert 12.0 < g.h / (g.c * g.dt) < 14.0
    check_pair(pa, g, 8, label="fine dt")
    g2 = ring_geom(n=(96, 80), S=32, K=64)
    check_pair(pa, g2, 9, label="coarse dt")


def test_coarse_pitch_matches_oracle(pa):
    # h / (c dt) ~ 60 samples per pixel: a base tile's window spans ~1280
    # samples, still within LDS for both operators
    g = ring_geom(n=(30, 30), S=40, K=2700)
    check_pair(pa, g, 15, label="60 samples per pixel")


def test_pitch_beyond_lds_window_is_unsupported(pa):
    import paper_2404_10928_amd._lib as L
    g = ring_geom(n=(30, 30), S=40, K=9000)   # h / (c dt) ~ 200 samples per pixel
    with pytest.raises(L.PaError) as e:
        pa.forward(torch.ones(g.image_shape, dtype=torch.float32, device="cuda"), g)
    assert e.value.status == L.PA_ERR_UNSUPPORTED


def test_point_sources_golden(pa):
    for case in load_point_sources():
        g = case["geom"]
        for dt, tol in ((np.float64, 1e-13), (np.float32, 2e-6)):
            x = np.zeros(g.n_pixels, dtype=dt)
            x[case["pixel"]] = 1
            y = run_forward(pa, g, x.reshape(g.image_shape), dt)[0]
            expect = np.zeros(g.n_samples)
            for k, v in case["taps"].items():
                expect[k] = v
            np.testing.assert_allclose(y, expect, rtol=tol, atol=tol * expect.max(), err_msg=case["name"])


def test_adjoint_identity_on_gpu(pa):
    for g in (ring_geom(n=(70, 45), S=100, K=350), hemi_geom(n=(12, 17, 9), S=70, K=200)):
        rng = np.random.default_rng(12)
        x = rng.normal(size=g.image_shape)
        y = rng.normal(size=g.data_shape)
        for dt, gate in ((np.float32, 1e-5), (np.float64, 1e-13)):
            xg, _ = rounded(x, dt)
            yg, _ = rounded(y, dt)
            lhs = float((run_forward(pa, g, xg, dt) * yg.astype(np.float64)).sum())
            rhs = float((xg.astype(np.float64) * run_adjoint(pa, g, yg, dt)).sum())
            err = abs(lhs - rhs) / (abs(lhs) + abs(rhs))
            print(f"adjointness {np.dtype(dt).name} {err:.2e}")
            assert err <= gate


def test_empty_and_degenerate(pa):
    g = ring_geom(n=(20, 20), S=10, K=50)
    dev = "cuda"
    for dt in (torch.float32, torch.float64):
        # no sensors
        g0 = g.replace(sensors=np.zeros((0, 2)))
        y = pa.forward(torch.ones(g.image_shape, dtype=dt, device=dev), g0)
        assert y.shape == (0, 50)
        x = pa.adjoint(torch.zeros((0, 50), dtype=dt, device=dev), g0)
        assert torch.count_nonzero(x).item() == 0
        # no samples
        gk = g.replace(n_samples=0)
        assert pa.forward(torch.ones(g.image_shape, dtype=dt, device=dev), gk).shape == (10, 0)
        assert torch.count_nonzero(pa.adjoint(torch.zeros((10, 0), dtype=dt, device=dev), gk)).item() == 0
        # no pixels
        gp = g.replace(nx=0)
        yp = pa.forward(torch.zeros((20, 0), dtype=dt, device=dev), gp)
        assert torch.count_nonzero(yp).item() == 0
        # one sample per trace, one pixel
        check_pair(pa, g.replace(n_samples=1, dt=1e-6), 13, label="K=1")
        check_pair(pa, ring_geom(n=(1, 1), S=5, K=40, radius=1e-3, dt=2e-8), 14, label="1 pixel")
    # every arrival beyond the trace
    far = g.replace(sensors=ring_sensors(10, 0.5))
    y = pa.forward(torch.ones(g.image_shape, dtype=torch.float32, device=dev), far)
    assert torch.count_nonzero(y).item() == 0


def test_invalid_arguments_raise(pa):
    import paper_2404_10928_amd._lib as L
    g = ring_geom(n=(8, 8), S=4, K=16)
    with pytest.raises(L.PaError):
        pa.forward(torch.ones((8, 8), dtype=torch.float32, device="cuda"), g.replace(dt=-1.0))
    with pytest.raises(TypeError):
        pa.forward(torch.ones((8, 8), dtype=torch.float16, device="cuda"), g)


# ------------------------------------------------------------ full workloads

def test_c1_full(pa):
    w = make_config("C1")
    check_pair(pa, w.geom, 101, label="C1")


def test_c2_full(pa):
    w = make_config("C2")
    g = w.geom
    x = w.x
    xg, x64 = rounded(x, np.float32)
    y_ref = oracle.forward(g, x64)
    yf = run_forward(pa, g, xg, np.float32)
    ef = rel_l2(yf, y_ref)
    r = np.random.default_rng(2002).normal(size=g.data_shape)
    rg, r64 = rounded(r, np.float32)
    ea = rel_l2(run_adjoint(pa, g, rg, np.float32), oracle.adjoint(g, r64))
    print(f"C2 full: forward(phantom) {ef:.3e} adjoint(noise) {ea:.3e}")
    assert ef <= F32_GATE and ea <= F32_GATE


def test_c5_sampled(pa):
    """128^3 voxels x 1024 sensors: compare outputs the oracle computes one by one."""
    w = make_config("C5")
    g = w.geom
    xg, x64 = rounded(w.x, np.float32)
    y = run_forward(pa, g, xg, np.float32)
    rng = np.random.default_rng(5005)
    # sample where the signal is: 24 random sensors, 4 samples each around its arrival peak
    picks = []
    for s in rng.choice(g.n_sensors, 24, replace=False):
        row = np.abs(y[s])
        top = np.argsort(row)[-40:]
        for k in rng.choice(top, 4, replace=False):
            picks.append((int(s), int(k)))
    got = np.array([y[s, k] for s, k in picks])
    ref = np.array([oracle.forward_at(g, x64, s, k) for s, k in picks])
    e_f = rel_l2(got, ref)
    yr = rng.normal(size=g.data_shape)
    yg, y64 = rounded(yr, np.float32)
    xa = run_adjoint(pa, g, yg, np.float32).reshape(-1)
    pix = rng.choice(g.n_pixels, 40, replace=False)
    e_a = rel_l2(xa[pix], np.array([oracle.adjoint_at(g, y64, int(p)) for p in pix]))
    print(f"C5 sampled: forward {e_f:.3e} adjoint {e_a:.3e}")
    assert e_f <= F32_GATE and e_a <= F32_GATE


@pytest.mark.parametrize("cut", ["late", "early"])
def test_adjoint_reads_only_inside_each_trace(pa, cut):
    """Aᵀ stages each sensor's trace window through a buffer resource whose
    range is that trace, so samples before 0 and from K on read as zero.  The
    traces sit inside a larger buffer whose other elements are NaN: a read
    before the first trace, past the last one or across into a neighbouring
    trace would change the image or make it NaN.  Arrivals run past the
    trace's end ("late") or start before sample 0 ("early")."""
    g = ring_geom(n=(48, 40), S=64, K=200)
    if cut == "late":
        g = g.replace(dt=g.dt * 0.6)
    else:
        half_diag = math.hypot(47, 39) * 1e-4 / 2
        g = g.replace(t0=half_diag / 1500.0)
    rng = np.random.default_rng(29)
    y = rng.normal(size=g.data_shape)
    pad = 4096
    n = g.data_shape[0] * g.data_shape[1]
    for dt, gate in ((np.float32, F32_GATE), (np.float64, F64_GATE)):
        yg, y64 = rounded(y, dt)
        big = torch.full((n + 2 * pad,), float("nan"), dtype=torch.float32 if dt == np.float32 else torch.float64,
                         device="cuda")
        big[pad:pad + n] = torch.from_numpy(np.ascontiguousarray(yg).reshape(-1)).to("cuda")
        yv = big[pad:pad + n].view(g.data_shape)
        xa = pa.adjoint(yv, g).cpu().numpy().astype(np.float64)
        e = rel_l2(xa, oracle.adjoint(g, y64))
        print(f"{cut} {np.dtype(dt).name}: adjoint {e:.3e}", flush=True)
        assert np.all(np.isfinite(xa)) and e <= gate
    # the forward operators on the same cut traces: sensor-major, and the
    # partial rows, whose pass 2 reads each row through a buffer resource
    xg, x64 = rounded(rng.uniform(size=g.image_shape), np.float32)
    y_ref = oracle.forward(g, x64)
    for method in ("sensor-major", "partial rows"):
        if method == "partial rows":
            pa.tuning_set(g, {"fwd_mode": 3, "fwd_tile": (2, 2, 1)}, torch.float32)
        try:
            yf = run_forward(pa, g, xg, np.float32)
        finally:
            pa.tuning_clear()
        e = rel_l2(yf, y_ref)
        print(f"{cut} forward ({method}): {e:.3e}", flush=True)
        assert e <= F32_GATE
