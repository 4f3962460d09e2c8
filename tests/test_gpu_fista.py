"""GPU FISTA on the l1 + TV objective of Eq. 8 against the FP64 oracle (or_fista).

Weights follow one recipe, scaled by the data: alpha = 1e-2 max|2 A^T y|,
beta = 1e-4 max|2 A^T y|, eps = 1e-2, x >= 0.  The step is the oracle's
(power iteration) where the test fixes it, so both sides take the same steps.
Proximal steps are non-expansive, so FP32 rounding is not amplified the way
CG amplifies it: the iterate and the whole history are gated (PA_F64 1e-9,
PA_F32 1e-4).
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, ring_geom, hemi_geom, rounded
from synth import add_noise, make_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


def weights(g, y64):
    b = np.abs(2 * oracle.adjoint(g, y64)).max()
    return 1e-2 * b, 1e-4 * b, 1e-2


def problem(name):
    w = make_config(name)
    g = w.geom
    y = add_noise(oracle.forward(g, w.x), w.noise_rel, w.noise_seeds[0])
    return w, g, y


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-9), (np.float32, 1e-4)])
@pytest.mark.parametrize("nonneg", [True, False])
def test_fista_128(pa, dt, tol, nonneg):
    w, g, y = problem("C1")
    yg, y64 = rounded(y, dt)
    alpha, beta, eps = weights(g, y64)
    omega = 1.0 / (oracle.power_sigma2(g, 30) + w.lam + 4 * beta / eps)
    x_ref, h_ref, _ = oracle.fista(g, y64, 20, w.lam, alpha, beta, eps, omega, nonneg=nonneg)
    x, h, om, s2 = pa.fista(torch.from_numpy(yg).to("cuda"), g, 20, w.lam, alpha, beta, eps, omega=omega,
                            nonneg=nonneg)
    xn = x.cpu().numpy()
    e_x = rel_l2(xn, x_ref)
    e_h = np.abs(h.cpu().numpy() / h_ref - 1).max()
    print(f"FISTA 128^2 {np.dtype(dt).name} nonneg={nonneg}: iterate {e_x:.2e} history {e_h:.2e}")
    assert om == omega and s2 == 0.0
    assert e_x <= tol and e_h <= tol
    if nonneg:
        assert (xn >= 0).all()
    # the threshold is active: a good share of exact zeros, on the same pixels up to the ones at the threshold
    z_ref, z = x_ref == 0, xn == 0
    assert 0.2 < z_ref.mean() < 0.95 and np.mean(z_ref != z) <= (1e-9 if dt == np.float64 else 1e-2)


def test_fista_512_fp32_power_step(pa):
    w, g, y = problem("C2")
    yg, y64 = rounded(y, np.float32)
    alpha, beta, eps = weights(g, y64)
    s2_ref = oracle.power_sigma2(g, 30)
    x, h, om, s2 = pa.fista(torch.from_numpy(yg).to("cuda"), g, 12, w.lam, alpha, beta, eps, omega=0.0,
                            power_iters=30, nonneg=True)
    assert abs(s2 / s2_ref - 1) <= 1e-5
    x_ref, h_ref, _ = oracle.fista(g, y64, 12, w.lam, alpha, beta, eps, om, nonneg=True)
    e_x = rel_l2(x.cpu().numpy(), x_ref)
    e_h = np.abs(h.cpu().numpy() / h_ref - 1).max()
    print(f"FISTA 512^2 FP32: sigma2 {abs(s2 / s2_ref - 1):.2e}, iterate {e_x:.2e}, history {e_h:.2e}")
    assert abs(om * (s2_ref + w.lam + 4 * beta / eps) - 1) <= 1e-5
    assert e_x <= 1e-4 and e_h <= 1e-4


def test_fista_volume_l1_only(pa):
    """3D with the l1 term only (the TV term is defined for 2D images)."""
    g = hemi_geom()
    rng = np.random.default_rng(51)
    xt = rng.uniform(size=g.image_shape) * (rng.uniform(size=g.image_shape) < 0.2)
    y = oracle.forward(g, xt)
    b = np.abs(2 * oracle.adjoint(g, y)).max()
    omega = 1.0 / (oracle.power_sigma2(g, 30) + 1e-3)
    for dt, tol in [(np.float64, 1e-9), (np.float32, 1e-4)]:
        yg, y64 = rounded(y, dt)
        x_ref, h_ref, _ = oracle.fista(g, y64, 15, 1e-3, 0.05 * b, 0.0, 1.0, omega)
        x, h, _, _ = pa.fista(torch.from_numpy(yg).to("cuda"), g, 15, 1e-3, 0.05 * b, 0.0, omega=omega)
        assert rel_l2(x.cpu().numpy(), x_ref) <= tol
        assert np.abs(h.cpu().numpy() / h_ref - 1).max() <= tol


def test_fista_graph_eager_and_edges(pa):
    g = ring_geom(n=(30, 26), S=40, K=200)
    rng = np.random.default_rng(52)
    y = torch.from_numpy(rng.normal(size=g.data_shape).astype(np.float32)).to("cuda")
    # FP32: integer forward bins and fixed-order sums make the solve reproducible bit for bit
    xa, ha, oa, _ = pa.fista(y, g, 6, 1e-2, 5.0, 1e-1, 1e-2, omega=0.0, power_iters=10, graph=True)
    xb, hb, ob, _ = pa.fista(y, g, 6, 1e-2, 5.0, 1e-1, 1e-2, omega=0.0, power_iters=10, graph=False)
    xc, hc, oc, _ = pa.fista(y, g, 6, 1e-2, 5.0, 1e-1, 1e-2, omega=0.0, power_iters=10, graph=True)
    assert oa == ob == oc
    assert torch.equal(xa, xb) and torch.equal(xa, xc)
    assert torch.equal(ha, hb) and torch.equal(ha, hc)
    # zero iterations: x = 0 and the history holds F(0) = ||y||^2 + beta TV(0) = ||y||^2 + beta P eps
    x, h, _, _ = pa.fista(y, g, 0, 1e-2, 5.0, 1e-1, 1e-2, omega=1e-3)
    F0 = float((y.double() ** 2).sum()) + 1e-1 * g.n_pixels * 1e-2
    assert torch.count_nonzero(x) == 0 and abs(h[0].item() / F0 - 1) <= 1e-12
    # no sensors: the gradient is lambda z + TV only; from 0 every step stays at 0
    g0 = g.replace(sensors=np.zeros((0, 2)))
    y0 = torch.zeros((0, 200), dtype=torch.float32, device="cuda")
    x, h, om, s2 = pa.fista(y0, g0, 3, 0.5, 1.0, 1e-1, 1e-2, omega=0.0)
    assert s2 == 0.0 and om == pytest.approx(1.0 / (0.5 + 4 * 1e-1 / 1e-2), rel=1e-15)
    assert torch.count_nonzero(x) == 0
    np.testing.assert_allclose(h.cpu().numpy(), 1e-1 * g.n_pixels * 1e-2, rtol=1e-12)
    import paper_2404_10928_amd._lib as L
    with pytest.raises(L.PaError):
        pa.fista(y, g, 3, 1e-2, 1.0, 1e-1, 0.0)          # eps must be > 0 with a TV term
    with pytest.raises(L.PaError):
        pa.fista(y, g, 3, 1e-2, -1.0, 0.0)
