"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-derives the oracle's own loops: they check hand-worked
arrivals (tests/golden), exact invariants of linear interpolation, the
adjoint identity, geometric symmetry, and the textbook solutions that CGLS
and Landweber must reach on tiny dense problems.
"""
import math

import numpy as np
import pytest

import oracle
from synth import Geometry, ring_sensors, fibonacci_hemisphere, segment_phantom
from golden_cases import load_point_sources


def small_geom(ndim=2, n=12, S=8, K=96, h=2e-4, radius=4e-3, dt=None, t0=0.0, nz=None):
    if ndim == 2:
        sens = ring_sensors(S, radius)
        nzz = 1
    else:
        sens = fibonacci_hemisphere(S, radius)
        nzz = n if nz is None else nz
    if dt is None:
        # all arrivals inside the trace: max distance / (c * (K - 3))
        half = math.sqrt(ndim) * (n - 1) * h / 2
        dt = (radius + half) / (1500.0 * (K - 3))
    return Geometry(ndim, n, n, nzz, h, (0.0, 0.0, 0.0), sens, K, dt, t0)


def pixel_positions(g):
    ix = np.arange(g.nx) - (g.nx - 1) / 2
    iy = np.arange(g.ny) - (g.ny - 1) / 2
    iz = np.arange(g.nz) - (g.nz - 1) / 2
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    pos = np.stack([X.ravel() * g.h + g.center[0], Y.ravel() * g.h + g.center[1],
                    Z.ravel() * g.h + g.center[2]], 1)
    return pos[:, : g.ndim]


def distances(g):
    P = pixel_positions(g)
    d = np.sqrt(((P[:, None, :] - g.sensors[None, :, :]) ** 2).sum(-1))
    rmin = g.r_min if g.r_min > 0 else g.h / 2
    return np.maximum(d, rmin)           # [P][S]


# --------------------------------------------------------------------------
# hand-worked arrivals (closed form)

@pytest.mark.parametrize("case", load_point_sources(), ids=lambda c: c["name"])
def test_point_source_golden(case):
    g = case["geom"]
    x = np.zeros(g.n_pixels)
    x[case["pixel"]] = 1.0
    y = oracle.forward(g, x.reshape(g.image_shape))
    expect = np.zeros(g.n_samples)
    for k, v in case["taps"].items():
        expect[k] = v
    np.testing.assert_allclose(y[0], expect, rtol=1e-13, atol=1e-13 * max(expect.max(), 1))
    # the adjoint of a unit sample returns the same weight at that pixel
    for k, v in case["taps"].items():
        e = np.zeros(g.data_shape)
        e[0, k] = 1.0
        xa = oracle.adjoint(g, e).reshape(-1)
        assert xa[case["pixel"]] == pytest.approx(v, rel=1e-13)
        if g.n_pixels == 1:
            assert np.count_nonzero(xa) == 1


# --------------------------------------------------------------------------
# invariants

@pytest.mark.parametrize("ndim", [2, 3])
def test_zeroth_and_first_moment(ndim):
    """With both taps inside the trace, sum_k y = sum_p x/R and sum_k k y = sum_p x tau/R."""
    g = small_geom(ndim, n=10 if ndim == 2 else 6, S=6, K=80)
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, size=g.image_shape)
    y = oracle.forward(g, x)
    R = distances(g)
    tau = (R / g.c - g.t0) / g.dt
    assert tau.min() > 0 and tau.max() < g.n_samples - 1
    xf = x.reshape(-1)
    m0 = (xf[:, None] / R).sum(0)
    m1 = (xf[:, None] * tau / R).sum(0)
    k = np.arange(g.n_samples)
    np.testing.assert_allclose(y.sum(1), m0, rtol=1e-12)
    np.testing.assert_allclose((y * k).sum(1), m1, rtol=1e-12)


def test_adjoint_of_unit_trace_is_inverse_distance():
    g = small_geom(2, n=9, S=5, K=64)
    R = distances(g)
    for s in range(g.n_sensors):
        y = np.zeros(g.data_shape)
        y[s, :] = 1.0
        x = oracle.adjoint(g, y).reshape(-1)
        np.testing.assert_allclose(x, 1.0 / R[:, s], rtol=1e-13)


@pytest.mark.parametrize("ndim,t0", [(2, 0.0), (2, 3.7e-7), (3, -2e-7)])
def test_adjoint_identity(ndim, t0):
    g = small_geom(ndim, n=14 if ndim == 2 else 7, S=9, K=70, t0=t0)
    rng = np.random.default_rng(11)
    x = rng.normal(size=g.image_shape)
    y = rng.normal(size=g.data_shape)
    lhs = float((oracle.forward(g, x) * y).sum())
    rhs = float((x * oracle.adjoint(g, y)).sum())
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_dense_brute_force_transpose_and_hat_definition():
    """A built column by column equals (A^T built row by row)^T, and every entry
    equals the direct hat-function evaluation (taps leaving the trace included)."""
    g = small_geom(2, n=6, S=4, K=40)
    g = g.replace(dt=g.dt * 0.8)         # push some late arrivals past the trace end
    P, M = g.n_pixels, g.n_sensors * g.n_samples
    A = np.zeros((M, P))
    for p in range(P):
        e = np.zeros(P)
        e[p] = 1.0
        A[:, p] = oracle.forward(g, e.reshape(g.image_shape)).reshape(-1)
    At = np.zeros((P, M))
    for m in range(M):
        e = np.zeros(M)
        e[m] = 1.0
        At[:, m] = oracle.adjoint(g, e.reshape(g.data_shape)).reshape(-1)
    assert np.array_equal(A, At.T)
    rng = np.random.default_rng(3)
    x = rng.normal(size=P)
    y = A @ x
    for m in range(0, M, 7):
        s, k = divmod(m, g.n_samples)
        assert oracle.forward_at(g, x, s, k) == pytest.approx(y[m], rel=1e-12, abs=1e-9)
    r = rng.normal(size=M)
    xa = At @ r
    for p in range(P):
        assert oracle.adjoint_at(g, r, p) == pytest.approx(xa[p], rel=1e-12, abs=1e-9)
    # some energy really was dropped past the end of the trace
    R = distances(g)
    assert ((R / g.c - g.t0) / g.dt).max() > g.n_samples - 1


def test_rotation_by_quarter_turn_shifts_sensors():
    """Ring of S = 0 mod 4 sensors around a square centred grid: rotating the
    image by +90 degrees rotates every arrival to the sensor S/4 further on."""
    g = small_geom(2, n=16, S=12, K=90)
    rng = np.random.default_rng(5)
    x = rng.uniform(size=g.image_shape)
    xr = x[::-1, :].T                       # x'(X, Y) = x(Y, -X): +90 degrees about the centre
    y = oracle.forward(g, x)
    yr = oracle.forward(g, xr)
    np.testing.assert_allclose(yr, np.roll(y, g.n_sensors // 4, axis=0), rtol=1e-9, atol=1e-9 * np.abs(y).max())


def test_time_origin_shift():
    g = small_geom(2, n=10, S=5, K=100)
    m = 7
    g = g.replace(dt=g.dt * 1.3)          # leave the last m+1 samples of every trace empty
    rng = np.random.default_rng(9)
    x = rng.uniform(size=g.image_shape)
    y = oracle.forward(g, x)
    assert np.all(y[:, -m - 1:] == 0)
    ys = oracle.forward(g.replace(t0=g.t0 - m * g.dt), x)
    np.testing.assert_allclose(ys[:, m:], y[:, :-m], rtol=1e-9, atol=1e-10 * np.abs(y).max())
    assert np.all(ys[:, :m] == 0)


def test_empty_and_degenerate_shapes():
    g = small_geom(2, n=4, S=3, K=16)
    g0 = g.replace(sensors=np.zeros((0, 2)))
    assert oracle.forward(g0, np.ones(g.image_shape)).shape == (0, 16)
    np.testing.assert_array_equal(oracle.adjoint(g0, np.zeros((0, 16))), 0)
    gk = g.replace(n_samples=0)
    assert oracle.forward(gk, np.ones(g.image_shape)).shape == (3, 0)
    np.testing.assert_array_equal(oracle.adjoint(gk, np.zeros((3, 0))), 0)
    gp = g.replace(nx=0)
    assert oracle.adjoint(gp, np.ones((3, 16))).size == 0
    np.testing.assert_array_equal(oracle.forward(gp, np.zeros((4, 0))), 0)


# --------------------------------------------------------------------------
# solvers against textbook solutions on tiny dense problems

def dense(g):
    P = g.n_pixels
    A = np.zeros((g.n_sensors * g.n_samples, P))
    for p in range(P):
        e = np.zeros(P)
        e[p] = 1.0
        A[:, p] = oracle.forward(g, e.reshape(g.image_shape)).reshape(-1)
    return A


def tiny_problem(seed=0):
    g = small_geom(2, n=6, S=5, K=40)
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(size=g.image_shape)
    y = oracle.forward(g, x_true) + 0.01 * rng.normal(size=g.data_shape)
    return g, y


@pytest.mark.parametrize("lam_rel", [1e-2, 1e-1])
def test_cgls_reaches_regularised_normal_equations(lam_rel):
    g, y = tiny_problem(1)
    A = dense(g)
    lam = lam_rel * np.linalg.norm(A, 2) ** 2
    x_ref = np.linalg.solve(A.T @ A + lam * np.eye(A.shape[1]), A.T @ y.reshape(-1))
    x, hist, stop = oracle.cgls(g, y, 3 * A.shape[1], lam)
    assert stop == 3 * A.shape[1] or hist[stop, 1] < 1e-10 * hist[0, 1]
    np.testing.assert_allclose(x.reshape(-1), x_ref, rtol=1e-8, atol=1e-8 * np.abs(x_ref).max())


def krylov_minimiser(M, b, k):
    """argmin over span{b, Mb, ..., M^(k-1) b} of x'Mx - 2 b'x (Arnoldi basis, twice re-orthogonalised)."""
    n = b.size
    V = np.zeros((n, k))
    v = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):
            v = v - V[:, :j] @ (V[:, :j].T @ v)
        v = v / np.linalg.norm(v)
        V[:, j] = v
        v = M @ v
    c = np.linalg.solve(V.T @ M @ V, V.T @ b)
    return V @ c


def test_cgls_iterates_minimise_over_krylov_spaces():
    g, y = tiny_problem(2)
    A = dense(g)
    lam = 1e-2 * np.linalg.norm(A, 2) ** 2
    M = A.T @ A + lam * np.eye(A.shape[1])
    b = A.T @ y.reshape(-1)
    prevF = np.inf
    for k in range(1, 7):
        x, hist, _ = oracle.cgls(g, y, k, lam)
        xk = krylov_minimiser(M, b, k)
        np.testing.assert_allclose(x.reshape(-1), xk, rtol=1e-7, atol=1e-7 * np.abs(xk).max())
        F = np.sum((A @ x.reshape(-1) - y.reshape(-1)) ** 2) + lam * np.sum(x ** 2)
        assert hist[k, 2] == pytest.approx(F, rel=1e-10)
        assert hist[k, 0] == pytest.approx(np.linalg.norm(y.reshape(-1) - A @ x.reshape(-1)), rel=1e-9)
        assert hist[k, 1] == pytest.approx(np.linalg.norm(A.T @ (y.reshape(-1) - A @ x.reshape(-1)) - lam * x.reshape(-1)), rel=1e-7)
        assert F <= prevF * (1 + 1e-12)
        prevF = F


def test_cgls_reorder_floor():
    """How far a correct CGLS may sit from the oracle's when it sums in another
    order.  On a 64x48 image with a 96-sensor ring and 320 samples (the GPU
    graph-versus-eager problem), CGLS written with numpy on the dense matrix
    built from the oracle's own operator columns follows the oracle to 1e-10
    for 8 iterations, then departs at ~20x per two iterations (3e-8 at 12):
    the rounding of CG's inner products, not the operator, sets that floor.
    Both solves are the textbook recursion, so their agreement at k <= 8 also
    pins the oracle's CGLS on a problem far larger than the tiny ones above."""
    import math as _m
    from synth import Geometry as _G
    nx, ny, S, K, h = 64, 48, 96, 320, 1e-4
    hd = _m.hypot(nx - 1, ny - 1) * h / 2
    rad = 1.2 * hd
    g = _G(2, nx, ny, 1, h, (0.0, 0.0, 0.0), ring_sensors(S, rad), K, (rad + hd) / (1500.0 * (K - 4)))
    rng = np.random.default_rng(21)
    y = oracle.forward(g, rng.uniform(size=g.image_shape)) + 0.01 * rng.normal(size=g.data_shape)
    P = g.n_pixels
    A = np.empty((g.n_sensors * g.n_samples, P))
    e = np.zeros(P)
    for p in range(P):
        e[p] = 1.0
        A[:, p] = oracle.forward(g, e.reshape(g.image_shape)).reshape(-1)
        e[p] = 0.0

    def cgls(n, lam=1e-3):
        x = np.zeros(P)
        r = y.reshape(-1).copy()
        s = A.T @ r
        p_ = s.copy()
        gam = s @ s
        for _ in range(n):
            q = A @ p_
            a = gam / (q @ q + lam * (p_ @ p_))
            x += a * p_
            r -= a * q
            s = A.T @ r - lam * x
            g2 = s @ s
            p_ = s + (g2 / gam) * p_
            gam = g2
        return x

    def rel(n):
        xo, _, _ = oracle.cgls(g, y, n, 1e-3)
        xd = cgls(n)
        return np.linalg.norm(xd - xo.reshape(-1)) / np.linalg.norm(xo)

    e8, e12 = rel(8), rel(12)
    print(f"dense CGLS vs oracle: {e8:.2e} at k = 8, {e12:.2e} at k = 12")
    assert e8 <= 1e-9
    assert 1e-9 <= e12 <= 1e-7


def test_cgls_warm_start_and_breakdown():
    g, y = tiny_problem(3)
    # y = 0 with x0 = 0: gamma_0 = 0, stops at iteration 0 with x = 0
    x, hist, stop = oracle.cgls(g, np.zeros(g.data_shape), 5, 1e-3)
    assert stop == 0 and np.all(x == 0) and np.all(hist == 0)
    # warm start from the exact solution of a well-posed problem stays there
    A = dense(g)
    lam = 1e-1 * np.linalg.norm(A, 2) ** 2
    x_ref = np.linalg.solve(A.T @ A + lam * np.eye(A.shape[1]), A.T @ y.reshape(-1))
    x, hist, stop = oracle.cgls(g, y, 3, lam, x0=x_ref.reshape(g.image_shape))
    np.testing.assert_allclose(x.reshape(-1), x_ref, rtol=1e-8, atol=1e-10 * np.abs(x_ref).max())
    assert hist[0, 1] < 1e-8 * np.linalg.norm(A.T @ y.reshape(-1))


def test_landweber_closed_form():
    g, y = tiny_problem(4)
    A = dense(g)
    lam = 1e-2 * np.linalg.norm(A, 2) ** 2
    M = A.T @ A + lam * np.eye(A.shape[1])
    b = A.T @ y.reshape(-1)
    omega = 1.0 / (np.linalg.norm(A, 2) ** 2 + lam)
    k = 9
    x, hist = oracle.landweber(g, y, k, lam, omega)
    T = np.eye(M.shape[0]) - omega * M
    x_ref = sum(np.linalg.matrix_power(T, j) @ (omega * b) for j in range(k))
    np.testing.assert_allclose(x.reshape(-1), x_ref, rtol=1e-10, atol=1e-12 * np.abs(x_ref).max())
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_power_iteration_reaches_the_largest_singular_value():
    """sigma2 from power iteration on A^T A equals ||A||_2^2 of the dense
    matrix (numpy SVD) once converged, and never exceeds it."""
    g, _ = tiny_problem(4)
    A = dense(g)
    smax2 = np.linalg.norm(A, 2) ** 2
    s200 = oracle.power_sigma2(g, 200)
    s3 = oracle.power_sigma2(g, 3)
    assert abs(s200 / smax2 - 1) <= 1e-8
    assert s3 <= smax2 * (1 + 1e-12) and s3 >= 0.5 * smax2
    # one step from the all-ones vector: ||A^T A 1|| / sqrt(P)
    one = np.ones(A.shape[1]) / np.sqrt(A.shape[1])
    assert abs(oracle.power_sigma2(g, 1) / np.linalg.norm(A.T @ (A @ one)) - 1) <= 1e-12


# --------------------------------------------------------------------------
# total variation term (Eq. 8) and the loss gradient

def test_tv_closed_forms():
    eps = 1e-3
    ny, nx = 6, 9
    assert oracle.tv2d(np.full((ny, nx), 3.7), eps)[0] == pytest.approx(nx * ny * eps, rel=1e-14)
    a, b = 0.7, -0.4
    iy, ix = np.mgrid[0:ny, 0:nx].astype(np.float64)
    v, g = oracle.tv2d(a * ix + b * iy, eps)
    expect = ((nx - 1) * (ny - 1) * math.sqrt(a * a + b * b + eps * eps) + (ny - 1) * math.sqrt(b * b + eps * eps)
              + (nx - 1) * math.sqrt(a * a + eps * eps) + eps)
    assert v == pytest.approx(expect, rel=1e-13)
    # a plane has zero TV gradient away from the borders
    np.testing.assert_allclose(g[1:-1, 1:-1], 0.0, atol=1e-12)


def test_tv_gradient_matches_finite_differences_and_shift_invariance():
    rng = np.random.default_rng(17)
    x = rng.uniform(size=(7, 8))
    eps = 1e-2
    v, g = oracle.tv2d(x, eps)
    h = 1e-6
    for p in rng.choice(x.size, 20, replace=False):
        e = np.zeros(x.size)
        e[p] = h
        e = e.reshape(x.shape)
        fd = (oracle.tv2d(x + e, eps)[0] - oracle.tv2d(x - e, eps)[0]) / (2 * h)
        assert g.reshape(-1)[p] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    assert oracle.tv2d(x + 5.0, eps)[0] == pytest.approx(v, rel=1e-12)
    assert abs(g.sum()) < 1e-10


def test_loss_gradient_is_exact_for_the_quadratic_term():
    g, y = tiny_problem(6)
    rng = np.random.default_rng(8)
    x = rng.uniform(size=g.image_shape)
    val, grad = oracle.loss_gradient(g, x, y, tv_weight=0.0)
    A = dense(g)
    np.testing.assert_allclose(grad.reshape(-1), 2 * A.T @ (A @ x.reshape(-1) - y.reshape(-1)), rtol=1e-10,
                               atol=1e-10 * np.abs(grad).max())
    # central differences are exact for a quadratic (up to rounding)
    val_t, grad_t = oracle.loss_gradient(g, x, y, tv_weight=1e-3, eps=1e-2)
    h = 1e-3
    for p in rng.choice(x.size, 10, replace=False):
        e = np.zeros(x.size)
        e[p] = h
        e = e.reshape(x.shape)
        fp = oracle.loss_gradient(g, x + e, y, 1e-3, 1e-2)[0]
        fm = oracle.loss_gradient(g, x - e, y, 1e-3, 1e-2)[0]
        assert grad_t.reshape(-1)[p] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-6 * np.abs(grad_t).max())


# --------------------------------------------------------------------------
# FISTA on the l1 + TV objective of Eq. 8 (identity sparsifying transforms)

def fista_objective_dense(A, y, x, lam, alpha, beta, eps, shape):
    r = A @ x - y
    F = r @ r + lam * x @ x + alpha * np.abs(x).sum()
    if beta:
        F += beta * oracle.tv2d(x.reshape(shape), eps)[0]
    return F


def tv_gradient_fd(x, eps, shape, h=1e-7):
    """dTV/dx by central differences of the TV value alone."""
    g = np.zeros(x.size)
    for p in range(x.size):
        e = np.zeros(x.size)
        e[p] = h
        g[p] = (oracle.tv2d((x + e).reshape(shape), eps)[0] - oracle.tv2d((x - e).reshape(shape), eps)[0]) / (2 * h)
    return g


def fista_setup(seed, lam_rel=1e-3):
    g, y = tiny_problem(seed)
    A = dense(g)
    L2 = np.linalg.norm(A, 2) ** 2
    return g, y, A, L2, lam_rel * L2


@pytest.mark.parametrize("nonneg", [False, True])
def test_fista_without_penalties_reaches_normal_equations(nonneg):
    """alpha = beta = 0: the minimiser is (A^T A + lam I)^-1 A^T y (numpy solve);
    with the x >= 0 constraint it must satisfy the bound-constrained KKT conditions."""
    g, y, A, L2, lam = fista_setup(11, 1e-1)
    omega = 1.0 / (L2 + lam)
    x, hz, _ = oracle.fista(g, y, 400, lam, 0.0, 0.0, 1.0, omega, nonneg=nonneg)
    x = x.reshape(-1)
    b = A.T @ y.reshape(-1)
    if not nonneg:
        x_ref = np.linalg.solve(A.T @ A + lam * np.eye(A.shape[1]), b)
        np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-9 * np.abs(x_ref).max())
    else:
        grad = 2 * (A.T @ (A @ x) - b + lam * x)
        scale = np.abs(2 * b).max()
        assert np.all(x >= 0)
        assert np.all(np.abs(grad[x > 0]) <= 1e-8 * scale)
        assert np.all(grad[x == 0] >= -1e-8 * scale)
    assert hz[-1] == pytest.approx(fista_objective_dense(A, y.reshape(-1), x, lam, 0, 0, 1, g.image_shape), rel=1e-12)


@pytest.mark.parametrize("nonneg", [False, True])
def test_fista_l1_satisfies_kkt(nonneg):
    """beta = 0, alpha > 0 (lasso with a ridge term): at the minimiser,
    2(A^T(Ax - y) + lam x)_i = -alpha sign(x_i) where x_i != 0 and
    |2(A^T(Ax - y) + lam x)_i| <= alpha where x_i = 0 (>= -alpha with x >= 0)."""
    g, y, A, L2, lam = fista_setup(12, 1e-2)
    b = A.T @ y.reshape(-1)
    alpha = 0.3 * np.abs(2 * b).max()
    omega = 1.0 / (L2 + lam)
    x, hz, hx = oracle.fista(g, y, 1500, lam, alpha, 0.0, 1.0, omega, nonneg=nonneg, x_history=True)
    x = x.reshape(-1)
    grad = 2 * (A.T @ (A @ x) - b + lam * x)
    nz = x != 0
    assert 0 < nz.sum() < x.size        # the threshold is active on some pixels and not on others
    np.testing.assert_allclose(grad[nz], -alpha * np.sign(x[nz]), rtol=0, atol=1e-7 * alpha)
    if nonneg:
        assert np.all(x >= 0) and np.all(grad[~nz] >= -alpha * (1 + 1e-7))
    else:
        assert np.all(np.abs(grad[~nz]) <= alpha * (1 + 1e-7))
    assert hx[-1] == pytest.approx(fista_objective_dense(A, y.reshape(-1), x, lam, alpha, 0, 1, g.image_shape),
                                   rel=1e-12)


def test_fista_tv_satisfies_kkt():
    """beta > 0 with alpha > 0 and x >= 0: stationarity with the TV gradient
    taken by central differences of the TV value (not the oracle's analytic
    gradient)."""
    g, y, A, L2, lam = fista_setup(13, 1e-3)
    b = A.T @ y.reshape(-1)
    eps = 0.05
    beta = 0.05 * np.abs(2 * b).max()
    alpha = 0.6 * np.abs(2 * b).max()
    omega = 1.0 / (L2 + lam + 4 * beta / eps)
    x, hz, hx = oracle.fista(g, y, 3000, lam, alpha, beta, eps, omega, nonneg=True, x_history=True)
    x = x.reshape(-1)
    grad = 2 * (A.T @ (A @ x) - b + lam * x) + beta * tv_gradient_fd(x, eps, g.image_shape)
    nz = x > 0
    assert 0 < nz.sum() < x.size
    np.testing.assert_allclose(grad[nz], -alpha, rtol=0, atol=1e-6 * alpha)
    assert np.all(grad[~nz] >= -alpha * (1 + 1e-6))
    assert hx[-1] == pytest.approx(fista_objective_dense(A, y.reshape(-1), x, lam, alpha, beta, eps, g.image_shape),
                                   rel=1e-12)


def test_fista_meets_the_accelerated_rate_bound():
    """Beck and Teboulle's bound F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k + 1)^2,
    with L = 2 / omega the Lipschitz constant of the smooth part's gradient.  The
    data are A v for the eigenvector v of A^T A whose eigenvalue is about
    L / (4 N): an unaccelerated proximal gradient leaves an error near
    (1 - 1/(2N))^(2k) there, an order of magnitude above the bound at k = N."""
    g, _, A, L2, lam = fista_setup(14, 1e-9)
    w, V = np.linalg.eigh(A.T @ A)
    N = 300
    omega = 1.0 / (L2 + lam)
    j = int(np.argmin(np.abs(w * omega - 1.0 / (2 * N))))
    y = (A @ V[:, j]).reshape(g.data_shape)
    alpha = 1e-4 * np.abs(2 * A.T @ y.reshape(-1)).max()
    xs, _, _ = oracle.fista(g, y, 40000, lam, alpha, 0.0, 1.0, omega)
    Fs = fista_objective_dense(A, y.reshape(-1), xs.reshape(-1), lam, alpha, 0, 1, g.image_shape)
    _, _, hx = oracle.fista(g, y, N, lam, alpha, 0.0, 1.0, omega, x_history=True)
    k = np.arange(1, N + 1)
    bound = 2 * (2 / omega) * np.sum(xs ** 2) / (k + 1) ** 2
    assert np.all(hx[1:] - Fs <= bound)
    assert np.all(hx >= Fs * (1 - 1e-12))


# --------------------------------------------------------------------------
# frequency-domain matrix (Eq. 7)

def test_freq_point_source_quarter_cycles():
    """One pixel at the origin and a sensor at (3 mm, 4 mm): R = 5 mm.  With
    c = 1500 m/s, f_n = 75 kHz * (n + 1) puts (n + 1) quarter cycles on the path,
    so exp(-i k_n R) = (-i)^(n+1) and K = i * 2 pi f_n * (-i)^(n+1) / R:
    2 pi f / R, -i 4 pi f_0 / R... worked out by hand below."""
    g = Geometry(2, 1, 1, 1, 1e-4, (0.0, 0.0, 0.0), np.array([[3e-3, 4e-3]]), 8, 1e-7, 0.0)
    Y = oracle.freq_forward(g, np.ones((1, 1)), 75e3, 75e3, 4)[0]
    u = 2 * math.pi * 75e3 / 5e-3
    expect = [1 * u, -2j * u, -3 * u, 4j * u]     # i (-i)^m m u for m = 1..4
    np.testing.assert_allclose(Y.real, np.real(expect), rtol=0, atol=1e-9 * u)
    np.testing.assert_allclose(Y.imag, np.imag(expect), rtol=0, atol=1e-9 * u)


@pytest.mark.parametrize("ndim", [2, 3])
def test_freq_adjoint_identity(ndim):
    g = small_geom(ndim, n=7 if ndim == 3 else 11, S=6)
    rng = np.random.default_rng(71)
    x = rng.normal(size=g.image_shape)
    Y = rng.normal(size=(g.n_sensors, 9)) + 1j * rng.normal(size=(g.n_sensors, 9))
    KX = oracle.freq_forward(g, x, 2e5, 3.1e5, 9)
    KtY = oracle.freq_adjoint(g, Y, 2e5, 3.1e5, 9)
    lhs = np.sum(KX.real * Y.real + KX.imag * Y.imag)
    rhs = np.sum(x * KtY)
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(np.abs(KX) ** 2) * np.sum(np.abs(Y) ** 2))


def test_freq_rotation_by_quarter_turn_shifts_sensors():
    g = small_geom(2, n=10, S=8)
    rng = np.random.default_rng(72)
    x = rng.uniform(size=g.image_shape)
    Y = oracle.freq_forward(g, x, 1e5, 2e5, 5)
    Yr = oracle.freq_forward(g, np.rot90(x, 1), 1e5, 2e5, 5)
    sh = g.n_sensors // 4
    a = np.allclose(Yr, np.roll(Y, sh, axis=0), rtol=1e-12, atol=1e-12 * np.abs(Y).max())
    b = np.allclose(Yr, np.roll(Y, -sh, axis=0), rtol=1e-12, atol=1e-12 * np.abs(Y).max())
    assert a or b


def test_freq_is_the_spectrum_of_the_time_domain_derivative():
    """K(omega) = i omega exp(-i omega R / c) / R is the Fourier transform of
    d/dt [delta(t - R/c) / R].  The time-domain operator (pinned above) spreads
    the delta over a unit-peak hat on the sample grid (dt times a unit-area
    pulse), whose transform is dt exp(-i omega tau dt) up to O((omega dt)^2);
    the sample sum's own dt cancels it, so at omega dt = 0.02
    i omega sum_k y[s,k] exp(-i omega k dt) matches K x to ~1e-4."""
    g = small_geom(2, n=9, S=5, K=400)
    rng = np.random.default_rng(73)
    x = rng.uniform(size=g.image_shape)
    y = oracle.forward(g, x)
    omega = 0.02 / g.dt
    f = omega / (2 * math.pi)
    k = np.arange(g.n_samples)
    spec = 1j * omega * (y * np.exp(-1j * omega * k * g.dt)[None, :]).sum(1)
    Y = oracle.freq_forward(g, x, f, 0.0, 1)[:, 0]
    err = np.abs(Y - spec).max() / np.abs(Y).max()
    assert err <= 2e-4
    # a sign error in the phase or a lost i turns the match into a mismatch of order one
    assert np.abs(np.conj(Y) - spec).max() / np.abs(Y).max() > 0.1
