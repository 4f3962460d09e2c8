"""Frequency-domain operator of Eq. 7 on the GPU against the FP64 oracle
(or_freq_forward / or_freq_adjoint).

The 128x128 workload uses the DFT bins of its own trace length as the
frequency grid: f_n = (n + 1) / (K dt), n = 0 .. K/2 - 1 (78 kHz to 20 MHz,
up to ~270 cycles along a path).  Gates: PA_F64 1e-10, PA_F32 1e-5 rel-L2.
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, ring_geom, hemi_geom, rounded
from synth import make_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


def run(pa, g, f0, df, nf, dt, seed):
    rng = np.random.default_rng(seed)
    tdt = torch.float64 if dt == np.float64 else torch.float32
    op = pa.FreqOperator(g, f0, df, nf, tdt, "cuda")
    x = rng.uniform(size=g.image_shape)
    Y = rng.normal(size=(g.n_sensors, nf, 2))
    xg, x64 = rounded(x, dt)
    Yg, Y64 = rounded(Y, dt)
    Yo = op.forward(torch.from_numpy(xg).to("cuda")).cpu().numpy()
    xo = op.adjoint(torch.from_numpy(Yg).to("cuda")).cpu().numpy()
    Yr = oracle.freq_forward(g, x64, f0, df, nf)
    xr = oracle.freq_adjoint(g, Y64[..., 0] + 1j * Y64[..., 1], f0, df, nf)
    e_f = rel_l2(np.stack([Yo[..., 0], Yo[..., 1]]), np.stack([Yr.real, Yr.imag]))
    e_a = rel_l2(xo, xr)
    return op, e_f, e_a, (xg, Yg, Yo, xo)


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-10), (np.float32, 1e-5)])
def test_freq_128_dft_bins(pa, dt, tol):
    w = make_config("C1")
    g = w.geom
    df = 1.0 / (g.n_samples * g.dt)
    op, e_f, e_a, (xg, Yg, Yo, xo) = run(pa, g, df, df, g.n_samples // 2, dt, 81)
    print(f"freq 128^2 {np.dtype(dt).name}: K {e_f:.2e} K^H {e_a:.2e}")
    assert e_f <= tol and e_a <= tol
    # fixed-order sums: repeat calls agree bit for bit
    assert np.array_equal(Yo, op.forward(torch.from_numpy(xg).to("cuda")).cpu().numpy())
    assert np.array_equal(xo, op.adjoint(torch.from_numpy(Yg).to("cuda")).cpu().numpy())


@pytest.mark.parametrize("kind", ["ring", "hemi"])
def test_freq_ragged(pa, kind):
    """Image sizes that are not multiples of 256, more than one block of 256
    frequencies, a sensor count that leaves a short sensor chunk."""
    g = ring_geom(n=(37, 29), S=23, K=150) if kind == "ring" else hemi_geom(n=(9, 7, 5), S=17, K=120)
    for dt, tol in [(np.float64, 1e-10), (np.float32, 1e-5)]:
        _, e_f, e_a, _ = run(pa, g, 1.3e5, 7.1e4, 300, dt, 82)
        print(f"freq {kind} {np.dtype(dt).name}: K {e_f:.2e} K^H {e_a:.2e}")
        assert e_f <= tol and e_a <= tol


def test_freq_edges(pa):
    import paper_2404_10928_amd._lib as L
    g = ring_geom(n=(11, 9), S=6, K=80)
    # no frequencies: Y is empty and K^H Y = 0
    op = pa.FreqOperator(g, 1e5, 1e5, 0, torch.float32, "cuda")
    x = torch.rand(g.image_shape, dtype=torch.float32, device="cuda")
    assert op.forward(x).numel() == 0
    assert torch.count_nonzero(op.adjoint(torch.zeros((6, 0, 2), dtype=torch.float32, device="cuda"))) == 0
    # no sensors
    g0 = g.replace(sensors=np.zeros((0, 2)))
    op0 = pa.FreqOperator(g0, 1e5, 1e5, 4, torch.float64, "cuda")
    assert op0.forward(x.double()).numel() == 0
    assert torch.count_nonzero(op0.adjoint(torch.zeros((0, 4, 2), dtype=torch.float64, device="cuda"))) == 0
    # f = 0: K = 0
    opz = pa.FreqOperator(g, 0.0, 0.0, 3, torch.float64, "cuda")
    assert torch.count_nonzero(opz.forward(x.double())) == 0
    with pytest.raises(L.PaError):
        pa.FreqOperator(g, -1.0, 1e5, 4).forward(x)
    with pytest.raises(L.PaError):
        pa.FreqOperator(g, 1e5, 1e5, 70000)
