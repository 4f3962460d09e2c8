"""The C ABI's contract on the GPU: non-finite inputs surface, results repeat
bit for bit, pa_forward / pa_adjoint can be captured into a caller's graph
(the library allocates no device memory), a cached solve graph follows a
re-tuned plan, and the PA_MIXED operators match the oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, ring_geom, hemi_geom, rounded

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PRECISIONS = [(torch.float32, None), (torch.float64, None), (torch.float64, "mixed")]


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


PARTIAL_ROWS = {"fwd_mode": 3, "fwd_tile": (2, 2, 1)}


@pytest.mark.parametrize("dt,prec", PRECISIONS + [(torch.float32, "partial rows")])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_pixel_gives_non_finite_traces(pa, dt, prec, bad):
    g = ring_geom(n=(48, 40), S=64, K=300)
    if prec == "partial rows":   # the two-pass forward through a workspace
        pa.tuning_set(g, PARTIAL_ROWS, dt)
        prec = None
    try:
        x = torch.rand(g.image_shape, dtype=dt, device="cuda")
        x[17, 23] = bad
        y = pa.forward(x, g, precision=prec).cpu().numpy()
    finally:
        pa.tuning_clear()
    assert not np.all(np.isfinite(y))
    # the other sensors' arrivals from finite pixels stay finite somewhere
    assert np.any(np.isfinite(y))
    yb = torch.randn(g.data_shape, dtype=dt, device="cuda")
    yb[5, 100] = bad
    xa = pa.adjoint(yb, g, precision=prec).cpu().numpy()
    assert not np.all(np.isfinite(xa))


@pytest.mark.parametrize("dt,prec", PRECISIONS)
def test_nan_data_stops_cgls_at_iteration_zero(pa, dt, prec):
    import paper_2404_10928_amd._lib as L
    g = ring_geom(n=(32, 32), S=48, K=240)
    y = torch.randn(g.data_shape, dtype=dt, device="cuda")
    y[3, 50] = float("nan")
    x, hist, stop = pa.cgls(y, g, 6, 1e-3, precision=prec)
    assert stop == 0
    assert np.all(x.cpu().numpy() == 0)
    # the status call itself reports the breakdown
    solver = pa.CglsSolver(g, dt, 6, 1e-3, precision=prec)
    solver.solve(y)
    torch.cuda.synchronize()
    import ctypes
    out = ctypes.c_int32(-2)
    st = L.load().pa_cgls_stop_iteration(solver.workspace.data_ptr(), ctypes.byref(out))
    assert st == L.PA_ERR_BREAKDOWN and out.value == 0


@pytest.mark.parametrize("dt,prec", PRECISIONS + [(torch.float32, "partial rows")])
def test_operators_repeat_bit_for_bit(pa, dt, prec):
    from synth import make_config
    w = make_config("C2")
    g = pa.DeviceGeometry(w.geom, "cuda")
    if prec == "partial rows":
        pa.tuning_set(g, PARTIAL_ROWS, dt)
        prec = None
    try:
        x = torch.rand(g.image_shape, dtype=dt, device="cuda")
        y = torch.randn(g.data_shape, dtype=dt, device="cuda")
        op = pa.Operator(g, dt, precision=prec)
        ya, yb = torch.empty_like(y), torch.empty_like(y)
        xa, xb = torch.empty_like(x), torch.empty_like(x)
        op.forward_(x, ya)
        op.adjoint_(y, xa)
        op.forward_(x, yb)
        op.adjoint_(y, xb)
        torch.cuda.synchronize()
    finally:
        pa.tuning_clear()
    assert torch.equal(ya, yb) and torch.equal(xa, xb)


@pytest.mark.parametrize("dt,prec", PRECISIONS)
def test_mixed_and_plain_operators_match_oracle(pa, dt, prec):
    gate = 1e-12 if (dt == torch.float64 and prec is None) else 1e-5
    for g in (ring_geom(n=(70, 45), S=100, K=350), ring_geom(n=(50, 50), S=96, K=380, radius=2.0e-3),
              hemi_geom(n=(12, 17, 9), S=70, K=200)):
        rng = np.random.default_rng(41)
        npdt = np.float32 if dt == torch.float32 else np.float64
        xg, x64 = rounded(rng.uniform(size=g.image_shape), npdt)
        yg, y64 = rounded(rng.normal(size=g.data_shape), npdt)
        yo = pa.forward(torch.from_numpy(xg).to("cuda"), g, precision=prec).cpu().numpy()
        xo = pa.adjoint(torch.from_numpy(yg).to("cuda"), g, precision=prec).cpu().numpy()
        ef, ea = rel_l2(yo, oracle.forward(g, x64)), rel_l2(xo, oracle.adjoint(g, y64))
        print(f"{dt} {prec}: forward {ef:.2e} adjoint {ea:.2e}")
        assert ef <= gate and ea <= gate


@pytest.mark.parametrize("method", ["rule", "partial rows"])
def test_forward_and_adjoint_captured_in_a_torch_graph(pa, method):
    """pa_forward(_ws) and pa_adjoint allocate nothing, so a caller can
    capture them; each replay (with eager work in between) matches the
    oracle.  "partial rows": the two-pass forward through the Operator's
    torch-owned workspace."""
    g = ring_geom(n=(96, 80), S=120, K=480)
    dg = pa.DeviceGeometry(g, "cuda")
    pa.tuning_clear()
    if method == "partial rows":
        pa.tuning_set(dg, PARTIAL_ROWS, torch.float32)
    try:
        _captured_replays(pa, g, dg)
    finally:
        pa.tuning_clear()


def _captured_replays(pa, g, dg):
    op = pa.Operator(dg, torch.float32)
    x = torch.empty(g.image_shape, dtype=torch.float32, device="cuda")
    y = torch.empty(g.data_shape, dtype=torch.float32, device="cuda")
    x2 = torch.empty_like(x)
    x.uniform_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        op.forward_(x, y)
        op.adjoint_(y, x2)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        op.forward_(x, y)
        op.adjoint_(y, x2)
    for rep in range(3):
        rng = np.random.default_rng(300 + rep)
        xv = rng.uniform(size=g.image_shape).astype(np.float32)
        x.copy_(torch.from_numpy(xv))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        yv = y.cpu().numpy()
        ef = rel_l2(yv, oracle.forward(g, xv.astype(np.float64)))
        ea = rel_l2(x2.cpu().numpy(), oracle.adjoint(g, yv.astype(np.float64)))
        print(f"replay {rep}: forward {ef:.2e} adjoint {ea:.2e}")
        assert ef <= 1e-5 and ea <= 1e-5
        _ = (x * 2).sum().item()   # eager work between replays


def test_cached_solve_graph_follows_a_retuned_plan(pa):
    """cgls, autotune, cgls on the same tensors and workspace: the second
    solve must use the new plan (its graph is captured anew), i.e. equal a
    fresh solve under the new tuning bit for bit."""
    g = ring_geom(n=(96, 96), S=128, K=600)
    dg = pa.DeviceGeometry(g, "cuda")
    rng = np.random.default_rng(42)
    y = torch.from_numpy(rng.normal(size=g.data_shape).astype(np.float32)).to("cuda")
    pa.tuning_clear()
    try:
        solver = pa.CglsSolver(dg, torch.float32, 10, 1e-3, graph=True)
        x = torch.empty(g.image_shape, dtype=torch.float32, device="cuda")
        solver.solve(y, x)
        torch.cuda.synchronize()
        t = pa.autotune(dg, torch.float32)
        print("tuning:", t)
        solver.solve(y, x)
        torch.cuda.synchronize()
        fresh = pa.CglsSolver(dg, torch.float32, 10, 1e-3, graph=False)
        xf = fresh.solve(y)
        torch.cuda.synchronize()
        assert torch.equal(x, xf)
        # the same for a batch: solve, autotune (new plan and workspace), solve
        b = pa.Batch([dg, pa.DeviceGeometry(ring_geom(n=(40, 40), S=20, K=200), "cuda")], torch.float32)
        yp = torch.cat([y.reshape(-1), torch.zeros(20 * 200, device="cuda")])
        xb = b.cgls(yp, 10, 1e-3)
        print("batch kept tuned plans:", b.autotune())
        xb2 = b.cgls(yp, 10, 1e-3, x=xb).clone()
        xb3 = b.cgls(yp, 10, 1e-3, graph=False)   # eager: always the current plan
        torch.cuda.synchronize()
        assert torch.equal(xb2, xb3)
    finally:
        pa.tuning_clear()


@pytest.mark.parametrize("method", ["rule", "partial rows"])
@pytest.mark.parametrize("scale", [1e-33, 1e-20, 1e30])
def test_fixed_point_forward_keeps_tiny_and_huge_images(pa, method, scale):
    """The FP32 forward's fixed-point rows are scaled per group (or per
    forward tile) by the bound of their taps; images of any magnitude FP32
    holds come out at the same relative accuracy, tiny ones included (their
    groups are prescaled by an exact power of two)."""
    g = ring_geom(n=(70, 45), S=100, K=350)
    if method == "partial rows":
        pa.tuning_set(g, PARTIAL_ROWS, torch.float32)
    try:
        rng = np.random.default_rng(43)
        xg, x64 = rounded(rng.uniform(size=g.image_shape) * scale, np.float32)
        yo = pa.forward(torch.from_numpy(xg).to("cuda"), g).cpu().numpy()
    finally:
        pa.tuning_clear()
    e = rel_l2(yo, oracle.forward(g, x64))
    print(f"{method}, x ~ {scale:g}: forward {e:.2e}")
    assert np.all(np.isfinite(yo)) and e <= 1e-5
