"""Gradients through the autograd wrappers (16 frames of 256x256, 128-sensor
ring, 1024 samples): loss = sum_b ||A x_b - y_b||^2 + 1e-3 TV(x_b).

* FP32 operator with FP64 loss reductions vs the FP64 oracle gradient
  2 A^T (A x - y) + 1e-3 dTV/dx, relative L2 over all frames.
* FP64 operator: central finite differences (h = 1e-3) at 64 seeded pixels
  against the autograd gradient (exact up to rounding for the quadratic term).
"""
import numpy as np
import pytest

import oracle
from gpu_common import rel_l2
from synth import add_noise, make_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TV_W = 1e-3


@pytest.fixture(scope="module")
def c3():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.autograd as ag
    import paper_2404_10928_amd.ops as ops
    w = make_config("C3")
    g = w.geom
    ys = np.stack([add_noise(oracle.forward(g, x), w.noise_rel, sd) for x, sd in zip(w.x_true, w.noise_seeds)])
    rng = np.random.default_rng([3003, 500])
    xe = rng.uniform(0.0, 1.0, size=(len(w.x_true),) + g.image_shape)   # evaluation point, far from the data
    return ag, ops, w, g, ys, xe


def loss(ag, geom, X, Y):
    return ag.data_term(X, Y, geom) + TV_W * ag.tv(X)


def test_gradient_fp32_vs_fp64_oracle(c3):
    ag, ops, w, g, ys, xe = c3
    geom = ops.DeviceGeometry(g)
    X = torch.from_numpy(xe.astype(np.float32)).cuda().requires_grad_(True)
    Y = torch.from_numpy(ys.astype(np.float32)).cuda()
    L = loss(ag, geom, X, Y)
    L.backward()
    got = X.grad.double().cpu().numpy()
    ref = np.stack([oracle.loss_gradient(g, xe.astype(np.float32)[b].astype(np.float64),
                                         ys.astype(np.float32)[b].astype(np.float64), TV_W)[1]
                    for b in range(xe.shape[0])])
    e = rel_l2(got, ref)
    print(f"C3 FP32 gradient vs FP64 oracle: rel-L2 {e:.3e}")
    assert e <= 1e-5


def test_gradient_fp64_finite_differences(c3):
    ag, ops, w, g, ys, xe = c3
    geom = ops.DeviceGeometry(g)
    X = torch.from_numpy(xe).cuda().requires_grad_(True)
    Y = torch.from_numpy(ys).cuda()
    loss(ag, geom, X, Y).backward()
    grad = X.grad.cpu().numpy()
    rng = np.random.default_rng([3003, 999])
    flat = rng.choice(xe.size, 64, replace=False)
    h = 1e-3
    errs = []
    for f in flat:
        b, p = divmod(int(f), g.n_pixels)
        xb = torch.from_numpy(xe[b]).cuda()
        yb = torch.from_numpy(ys[b]).cuda()
        e = torch.zeros(g.n_pixels, dtype=torch.float64, device="cuda")
        e[p] = h
        e = e.reshape(g.image_shape)
        with torch.no_grad():
            lp = loss(ag, geom, xb + e, yb).item()
            lm = loss(ag, geom, xb - e, yb).item()
        fd = (lp - lm) / (2 * h)
        errs.append(abs(fd - grad.reshape(-1)[f]) / max(abs(grad.reshape(-1)[f]), 1e-12))
    errs = np.array(errs)
    print(f"C3 FP64 central differences at 64 pixels: max rel err {errs.max():.2e}, median {np.median(errs):.2e}")
    assert errs.max() <= 1e-5


def test_adjoint_wrapper_backward_is_forward(c3):
    ag, ops, w, g, ys, xe = c3
    geom = ops.DeviceGeometry(g)
    Y = torch.from_numpy(ys[:2]).cuda().requires_grad_(True)
    V = torch.from_numpy(xe[:2]).cuda()
    (ag.PAAdjoint.apply(Y, geom) * V).sum().backward()
    ref = ops.forward(V, geom)
    assert rel_l2(Y.grad.cpu().numpy(), ref.cpu().numpy()) <= 1e-14
