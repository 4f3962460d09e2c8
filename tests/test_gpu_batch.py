"""Batched frames of uneven size (one launch per step for every frame) against
the single-frame calls and the FP64 oracle.

Both operators and the solver steps run the single-frame device code on each
frame's plan with every partial sum in the same order, so a batched result
equals the single-frame result bit for bit.
"""
import numpy as np
import pytest

import oracle
from gpu_common import hemi_geom, rel_l2, ring_geom, rounded
from synth import add_noise
from synth.configs import batched_frame

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


def mixed_frames():
    """Uneven 2D frames: sizes, sensor counts and trace lengths differ; one
    frame has a fractional time origin, one has sensors among its pixels, one
    has no sensors and one has no pixels."""
    return [
        ring_geom(n=(37, 29), S=70, K=300),
        ring_geom(n=(64, 48), S=129, K=411, t0=0.37e-7),
        ring_geom(n=(50, 50), S=96, K=380, radius=2.0e-3),
        ring_geom(n=(16, 16), S=8, K=100).replace(sensors=np.zeros((0, 2))),
        ring_geom(n=(20, 20), S=12, K=90).replace(nx=0),
        ring_geom(n=(96, 80), S=33, K=64),
    ]


def inputs(geoms, seed, dt):
    rng = np.random.default_rng(seed)
    xs = [rounded(rng.uniform(size=g.image_shape), dt) for g in geoms]
    ys = [rounded(rng.normal(size=g.data_shape), dt) for g in geoms]
    return xs, ys


def single(pa, fn, g, a, dt):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return fn(t, g).cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_batched_operators_match_single_frames(pa, dt):
    geoms = mixed_frames()
    tdt = torch.float32 if dt == np.float32 else torch.float64
    b = pa.Batch(geoms, tdt)
    assert b.x_offsets[-1] == sum(g.n_pixels for g in geoms)
    assert b.y_offsets[-1] == sum(g.n_sensors * g.n_samples for g in geoms)
    xs, ys = inputs(geoms, 31, dt)
    xp = b.pack_x([torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x, _ in xs])
    yp = b.pack_y([torch.from_numpy(np.ascontiguousarray(y)).to("cuda") for y, _ in ys])
    yb = [t.cpu().numpy().astype(np.float64) for t in b.unpack_y(b.forward(xp))]
    xb = [t.cpu().numpy().astype(np.float64) for t in b.unpack_x(b.adjoint(yp))]
    gate = 1e-5 if dt == np.float32 else 1e-12
    for i, g in enumerate(geoms):
        ys_single = single(pa, pa.forward, g, xs[i][0], dt)
        xs_single = single(pa, pa.adjoint, g, ys[i][0], dt)
        # adjoint: bit for bit
        assert np.array_equal(xb[i], xs_single), f"frame {i}: batched adjoint differs from the single-frame one"
        # forward: bit for bit as well (every sum in a fixed order)
        assert yb[i].shape == ys_single.shape and xb[i].shape == xs_single.shape
        assert np.array_equal(yb[i], ys_single), f"frame {i}: batched forward differs from the single-frame one"
        if g.n_pixels and g.n_sensors and g.n_samples:
            assert rel_l2(yb[i], oracle.forward(g, xs[i][1])) <= gate
            assert rel_l2(xb[i], oracle.adjoint(g, ys[i][1])) <= gate
        else:
            assert not np.any(yb[i]) and not np.any(xb[i])


def test_batched_3d_operators(pa):
    geoms = [hemi_geom(), hemi_geom(n=(12, 17, 9), S=70, K=200), hemi_geom(n=(8, 8, 8), S=33, K=150)]
    b = pa.Batch(geoms, torch.float32)
    xs, ys = inputs(geoms, 32, np.float32)
    xp = b.pack_x([torch.from_numpy(x).to("cuda") for x, _ in xs])
    yp = b.pack_y([torch.from_numpy(y).to("cuda") for y, _ in ys])
    yb = b.unpack_y(b.forward(xp))
    xb = b.unpack_x(b.adjoint(yp))
    for i, g in enumerate(geoms):
        assert np.array_equal(xb[i].cpu().numpy(), single(pa, pa.adjoint, g, ys[i][0], np.float32).astype(np.float32))
        assert rel_l2(yb[i].cpu().numpy(), oracle.forward(g, xs[i][1])) <= 1e-5
        assert rel_l2(xb[i].cpu().numpy(), oracle.adjoint(g, ys[i][1])) <= 1e-5


@pytest.mark.parametrize("graph", [True, False])
def test_batched_cgls_matches_single_frames_f64(pa, graph):
    geoms = mixed_frames()
    b = pa.Batch(geoms, torch.float64)
    rng = np.random.default_rng(33)
    ys = []
    for g in geoms:
        y = oracle.forward(g, rng.uniform(size=g.image_shape)) if g.n_pixels else np.zeros(g.data_shape)
        ys.append(y + 0.01 * rng.normal(size=g.data_shape))
    yp = b.pack_y([torch.from_numpy(y).to("cuda") for y in ys])
    iters, lam = 12, 1e-3
    x = b.cgls(yp, iters, lam, graph=graph)
    xb = [t.cpu().numpy() for t in b.unpack_x(x)]
    hb = b.history.cpu().numpy()
    stops = b.stop_iterations()
    for i, g in enumerate(geoms):
        xs_, hs_, stop = pa.cgls(torch.from_numpy(ys[i]).to("cuda"), g, iters, lam, graph=False)
        assert stops[i] == stop, f"frame {i}"
        np.testing.assert_allclose(hb[i], hs_.cpu().numpy(), rtol=1e-9, atol=1e-300, err_msg=f"frame {i}")
        xs_ = xs_.cpu().numpy()
        assert rel_l2(xb[i], xs_) <= 1e-9 or (not np.any(xs_) and not np.any(xb[i])), f"frame {i}"
    # frames without sensors (breakdown at k=0) and without pixels stop; the others run every iteration
    assert stops[0] == -1 and stops[1] == -1 and stops[2] == -1 and stops[5] == -1


def test_batched_cgls_uneven_workload_f32(pa):
    """Frames drawn from the uneven-batch workload (image 128-512, 64-512
    sensors, 512-2048 samples), the smaller ones so the oracle stays short.
    The batched FP32 solve equals, bit for bit, the solve of each frame
    batched on its own (the same per-frame plan: the other frames of the
    launch change nothing; batch plans may take shorter forward segments
    than single-frame plans, to keep the launch's LDS small), follows the oracle on its stable prefix, k <= 4 (a 1e-12 change of y
    moves the oracle's F by ~1e-13 up to k = 11 and by 1e2 more per step after
    that; FP32 rounding reaches that regime sooner: the first frame departs by
    4e-2 by k = 10), its reported final F is the objective of its final
    iterate, and F never rises."""
    frames = []
    f = 0
    while len(frames) < 4:
        g, x = batched_frame(f)
        f += 1
        if g.nx <= 256 and g.n_sensors <= 256:
            frames.append((g, x))
    geoms = [g for g, _ in frames]
    ys = [add_noise(oracle.forward(g, x), 0.01, [4004, i, 1]) for i, (g, x) in enumerate(frames)]
    b = pa.Batch(geoms, torch.float32)
    y32 = [rounded(y, np.float32) for y in ys]
    yp = b.pack_y([torch.from_numpy(y).to("cuda") for y, _ in y32])
    iters, lam, K = 15, 1e-3, 4
    xb = [t.cpu().numpy().astype(np.float64) for t in b.unpack_x(b.cgls(yp, iters, lam))]
    hb = b.history.cpu().numpy()
    for i, g in enumerate(geoms):
        b1 = pa.Batch([g], torch.float32)
        xs_ = b1.cgls(b1.pack_y([torch.from_numpy(y32[i][0]).to("cuda")]), iters, lam)
        assert np.array_equal(xb[i], xs_.cpu().numpy().astype(np.float64).reshape(g.image_shape)), f"frame {i}"
        assert np.array_equal(hb[i], b1.history.cpu().numpy()[0]), f"frame {i}"
        _, h_ref, _ = oracle.cgls(g, y32[i][1], iters, lam)
        e_all = np.abs(hb[i, :, 2] / h_ref[:, 2] - 1)
        print(f"frame {i} per-k F error:", np.array2string(e_all, precision=1))
        e_h = np.abs(hb[i, : K + 1] / h_ref[: K + 1] - 1).max()
        r = oracle.forward(g, xb[i]) - y32[i][1]
        F_true = float((r * r).sum()) + lam * float((xb[i] * xb[i]).sum())
        e_self = abs(hb[i, -1, 2] / F_true - 1)
        print(f"frame {i} ({g.nx}^2, S={g.n_sensors}, K={g.n_samples}): history k<={K} {e_h:.2e}; "
              f"F_15 vs objective of x_15 {e_self:.2e}; F_15 vs oracle {abs(hb[i, -1, 2] / h_ref[-1, 2] - 1):.2e}")
        assert e_h <= 1e-4 and e_self <= 1e-4
        assert np.all(hb[i, 1:, 2] <= hb[i, :-1, 2] * (1 + 1e-6))


def test_autotune_records_a_tiling_and_keeps_results(pa):
    g = ring_geom(n=(96, 80), S=100, K=500)
    xs, ys = inputs([g], 34, np.float32)
    x, x64 = xs[0]
    y, y64 = ys[0]
    pa.tuning_clear()
    before_f = single(pa, pa.forward, g, x, np.float32)
    before_a = single(pa, pa.adjoint, g, y, np.float32)
    t = pa.autotune(g, torch.float32)
    print("tuning:", t)
    assert t["fwd_seg"] >= 1 and t["adj_lds_bytes"] > 0 and t["fwd_us"] > 0 and t["adj_us"] > 0
    after_f = single(pa, pa.forward, g, x, np.float32)
    after_a = single(pa, pa.adjoint, g, y, np.float32)
    # another tiling changes only the order of sums
    assert rel_l2(after_f, before_f) <= 1e-6 and rel_l2(after_a, before_a) <= 1e-6
    assert rel_l2(after_f, oracle.forward(g, x64)) <= 1e-5 and rel_l2(after_a, oracle.adjoint(g, y64)) <= 1e-5
    # a batch times its rule plans against the frames' tuned plans and keeps the faster
    b = pa.Batch([g, ring_geom(n=(40, 40), S=20, K=200)], torch.float32)
    kept_tuned = b.autotune()
    print("batch kept tuned plans:", kept_tuned)
    yb = b.unpack_y(b.forward(b.pack_x([torch.from_numpy(x).to("cuda"), torch.zeros((40, 40), device="cuda")])))
    assert rel_l2(yb[0].cpu().numpy(), oracle.forward(g, x64)) <= 1e-5
    xb = b.unpack_x(b.adjoint(b.pack_y([torch.from_numpy(y).to("cuda"), torch.zeros((20, 200), device="cuda")])))
    assert rel_l2(xb[0].cpu().numpy(), oracle.adjoint(g, y64)) <= 1e-5
    pa.tuning_clear()
