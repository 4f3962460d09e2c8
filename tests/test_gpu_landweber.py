"""GPU Landweber iteration and its power-iteration step size against the
FP64 oracle (or_landweber, or_power_sigma2).

The gradient iteration is a contraction (the step keeps the spectral radius
of I - omega (A^T A + lambda I) below 1), so per-apply rounding is not
amplified and the whole history is gated: PA_F64 to 1e-10, PA_F32 to 1e-5.
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, ring_geom, rounded
from synth import add_noise, make_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


def problem(name):
    w = make_config(name)
    g = w.geom
    y = add_noise(oracle.forward(g, w.x), w.noise_rel, w.noise_seeds[0])
    return w, g, y


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-10), (np.float32, 1e-5)])
def test_landweber_fixed_step_128(pa, dt, tol):
    w, g, y = problem("C1")
    yg, y64 = rounded(y, dt)
    omega = 1.0 / (oracle.power_sigma2(g, 30) + w.lam)
    x_ref, h_ref = oracle.landweber(g, y64, 20, w.lam, omega)
    x, h, om, s2 = pa.landweber(torch.from_numpy(yg).to("cuda"), g, 20, w.lam, omega=omega)
    e_x = rel_l2(x.cpu().numpy(), x_ref)
    e_h = np.abs(h.cpu().numpy() / h_ref - 1).max()
    print(f"Landweber 128^2 {np.dtype(dt).name}: iterate {e_x:.2e} history {e_h:.2e}")
    assert om == omega and s2 == 0.0
    assert e_x <= tol and e_h <= tol


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-10), (np.float32, 1e-5)])
def test_power_iteration_step(pa, dt, tol):
    g = ring_geom(n=(48, 40), S=64, K=300)
    rng = np.random.default_rng(41)
    y = rng.normal(size=g.data_shape)
    yg, y64 = rounded(y, dt)
    lam = 1e-3
    s2_ref = oracle.power_sigma2(g, 30)
    x, h, om, s2 = pa.landweber(torch.from_numpy(yg).to("cuda"), g, 5, lam, omega=0.0, power_iters=30)
    print(f"power iteration {np.dtype(dt).name}: sigma2 {s2:.6e} vs oracle {s2_ref:.6e}")
    assert abs(s2 / s2_ref - 1) <= tol
    assert abs(om * (s2_ref + lam) - 1) <= tol
    x_ref, h_ref = oracle.landweber(g, y64, 5, lam, 1.0 / (s2_ref + lam))
    assert rel_l2(x.cpu().numpy(), x_ref) <= 10 * tol
    assert np.abs(h.cpu().numpy() / h_ref - 1).max() <= 10 * tol


def test_landweber_512_fp32(pa):
    w, g, y = problem("C2")
    yg, y64 = rounded(y, np.float32)
    s2_ref = oracle.power_sigma2(g, 30)
    x, h, om, s2 = pa.landweber(torch.from_numpy(yg).to("cuda"), g, 10, w.lam, omega=0.0, power_iters=30)
    x_ref, h_ref = oracle.landweber(g, y64, 10, w.lam, 1.0 / (s2_ref + w.lam))
    e_x = rel_l2(x.cpu().numpy(), x_ref)
    e_h = np.abs(h.cpu().numpy() / h_ref - 1).max()
    print(f"Landweber 512^2 FP32: sigma2 {abs(s2 / s2_ref - 1):.2e}, iterate {e_x:.2e}, history {e_h:.2e}")
    assert abs(s2 / s2_ref - 1) <= 1e-5 and e_x <= 1e-4 and e_h <= 1e-5


def test_landweber_graph_eager_and_edges(pa):
    g = ring_geom(n=(30, 26), S=40, K=200)
    rng = np.random.default_rng(42)
    y = torch.from_numpy(rng.normal(size=g.data_shape)).to("cuda")
    xa, ha, oa, _ = pa.landweber(y, g, 6, 1e-2, omega=0.0, power_iters=10, graph=True)
    xb, hb, ob, _ = pa.landweber(y, g, 6, 1e-2, omega=0.0, power_iters=10, graph=False)
    # the FP64 forward operator adds its histogram terms in hardware order, so
    # two runs agree to FP64 rounding, not bit for bit
    assert abs(oa / ob - 1) <= 1e-13
    assert rel_l2(xa.cpu().numpy(), xb.cpu().numpy()) <= 1e-12
    np.testing.assert_allclose(ha.cpu().numpy(), hb.cpu().numpy(), rtol=1e-12)
    # zero iterations: history holds F(x0) only
    x0 = torch.from_numpy(rng.uniform(size=g.image_shape)).to("cuda")
    x, h, _, _ = pa.landweber(y, g, 0, 1e-2, omega=1e-3, x0=x0)
    r = oracle.forward(g, x0.cpu().numpy()) - y.cpu().numpy()
    F = float((r * r).sum()) + 1e-2 * float((x0.cpu().numpy() ** 2).sum())
    assert torch.equal(x, x0) and abs(h[0].item() / F - 1) <= 1e-12
    # no sensors: pure shrinkage x <- (1 - omega lambda) x
    g0 = g.replace(sensors=np.zeros((0, 2)))
    x, h, om, s2 = pa.landweber(torch.zeros((0, 200), dtype=torch.float64, device="cuda"), g0, 3, 0.5, omega=0.0,
                                x0=x0)
    assert s2 == 0.0 and om == 2.0
    np.testing.assert_allclose(x.cpu().numpy(), 0.0 * x0.cpu().numpy(), atol=1e-15)
    import paper_2404_10928_amd._lib as L
    with pytest.raises(L.PaError):
        pa.landweber(y, g, 3, 1e-2, omega=0.0, power_iters=0)
    with pytest.raises(L.PaError):
        pa.landweber(y, g, 3, 1e-2, omega=-1.0)
