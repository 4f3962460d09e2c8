"""3D and precision modes: the 128^3-voxel, 1024-sensor hemisphere solve in
PA_F32 (FP32 bulk, FP64 reductions) and PA_F64, 30 CGLS iterations each,
against the FP64 oracle's solve stored in tests/golden/c5_cgls_reference.json
(written by tests/golden/make_c5_reference.py, which calls only the oracle).

Gates after the solve: the iterate at 4096 stored voxels and F(x_30) within
1e-4 of the oracle for both precisions (PA_F64 is expected far closer); the
history follows the oracle's descent curve (see test_gpu_cgls).
"""
import json
import os
import sys

import numpy as np
import pytest

from gpu_common import rel_l2
from test_gpu_cgls import off_curve

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_c5_reference import c5_data, sample_indices  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    return ops


@pytest.fixture(scope="module")
def reference():
    with open(os.path.join(HERE, "golden", "c5_cgls_reference.json")) as f:
        ref = json.load(f)
    w, g, y = c5_data(threads=min(16, os.cpu_count() or 1))
    return ref, w, g, y


@pytest.fixture(scope="module")
def solves(pa, reference):
    ref, w, g, y = reference
    out = {}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        yt = torch.from_numpy(y).to("cuda", dtype=dt)
        x, hist, stop = pa.cgls(yt, g, w.iters, w.lam)
        out[name] = (x.double().cpu().numpy().reshape(-1), hist.cpu().numpy(), stop)
    return out


@pytest.mark.parametrize("name", ["f64", "f32"])
def test_volume_solve_matches_oracle(reference, solves, name):
    ref, w, g, y = reference
    x, hist, stop = solves[name]
    idx = np.array(ref["sample_index"])
    h_ref = np.array(ref["history"])
    e_x = rel_l2(x[idx], np.array(ref["x_sample"]))
    e_norm = abs(np.linalg.norm(x) / ref["x_norm"] - 1)
    e_F = abs(hist[-1, 2] / h_ref[-1, 2] - 1)
    err = np.abs(hist / h_ref - 1)
    print(f"3D {name}: sampled iterate {e_x:.2e}, ||x|| {e_norm:.2e}, final F {e_F:.2e}; "
          f"max over k: F {err[:, 2].max():.2e} ||r|| {err[:, 0].max():.2e}")
    assert stop == -1
    assert e_x <= 1e-4 and e_norm <= 1e-4 and e_F <= 1e-4
    if name == "f64":
        assert e_x <= 1e-8 and err[:, 2].max() <= 1e-8
    assert off_curve(hist[:, 2], h_ref[:, 2]) == [] and off_curve(hist[:, 0], h_ref[:, 0]) == []


def test_f32_against_f64_on_the_gpu(solves):
    x32, h32, _ = solves["f32"]
    x64, h64, _ = solves["f64"]
    e = rel_l2(x32, x64)
    print(f"3D FP32 vs FP64 iterate {e:.2e}, final F {abs(h32[-1, 2] / h64[-1, 2] - 1):.2e}")
    assert e <= 1e-4
