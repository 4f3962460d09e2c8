"""pa_forward_noalloc (the forward operator with the library's static device
scratch, for callers that cannot allocate) against pa_forward_ws with a
caller workspace, through the C ABI: the same plan gives the same bits.

The partial-row method is recorded for each shape with pa_tuning_set, so the
scratch is what both calls run through.  Two calls in a row, the second on a
smaller geometry; then the 512x512 workload; then a capture of the call into a
torch graph, replayed with eager work in between; and a shape whose rows do
not fit the scratch is refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_common import rel_l2, ring_geom

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TILE = {"fwd_mode": 3, "fwd_tile": (2, 2, 1)}


@pytest.fixture(scope="module")
def pa():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2404_10928_amd.ops as ops
    yield ops
    ops.tuning_clear()


def run_pair(pa, dg, x):
    import paper_2404_10928_amd._lib as L
    lib = L.load()
    cg = dg.c_struct()
    n = int(lib.pa_forward_workspace_bytes(ctypes.byref(cg), L.PA_F32))
    assert 0 < n <= (64 << 20), n      # the partial-row method is planned and fits the scratch
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    y_ws = torch.full(dg.data_shape, float("nan"), dtype=torch.float32, device="cuda")
    y_na = torch.full(dg.data_shape, float("nan"), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    L.check(lib.pa_forward_noalloc(ctypes.byref(cg), L.PA_F32, x.data_ptr(), y_na.data_ptr(), s))
    L.check(lib.pa_forward_ws(ctypes.byref(cg), L.PA_F32, x.data_ptr(), y_ws.data_ptr(), ws.data_ptr(), n, s))
    torch.cuda.synchronize()
    return y_na, y_ws


@pytest.mark.parametrize("shape", [((200, 176), 150, 900), ((64, 48), 40, 300)])
def test_noalloc_matches_workspace_call(pa, shape):
    """Runs in the listed order: the second call is on a smaller geometry and
    reuses the scratch the first left behind."""
    n, S, K = shape
    g = ring_geom(n=n, S=S, K=K)
    dg = pa.DeviceGeometry(g, "cuda")
    pa.tuning_set(dg, TILE, torch.float32)
    rng = np.random.default_rng([7007, n[0]])
    xv = rng.uniform(size=g.image_shape).astype(np.float32)
    x = torch.from_numpy(xv).to("cuda")
    y_na, y_ws = run_pair(pa, dg, x)
    assert torch.equal(y_na, y_ws)
    e = rel_l2(y_na.cpu().numpy(), oracle.forward(g, xv.astype(np.float64)))
    print(f"noalloc {n} S={S} K={K}: equal to pa_forward_ws, rel-L2 vs oracle {e:.2e}")
    assert e <= 1e-5


def test_noalloc_at_full_size(pa):
    from synth import make_config
    w = make_config("C2")
    dg = pa.DeviceGeometry(w.geom, "cuda")
    pa.tuning_set(dg, TILE, torch.float32)
    x = torch.from_numpy(w.x.astype(np.float32)).to("cuda")
    y_na, y_ws = run_pair(pa, dg, x)
    assert torch.equal(y_na, y_ws)
    # sampled entries against the oracle, one output at a time
    rng = np.random.default_rng([7007, 512])
    flat = y_na.cpu().numpy().reshape(-1)
    idx = np.unique(np.concatenate([rng.choice(flat.size, 96, replace=False), np.argsort(np.abs(flat))[-96:]]))
    x64 = w.x.astype(np.float32).astype(np.float64)
    ref = np.array([oracle.forward_at(w.geom, x64, j // w.geom.n_samples, j % w.geom.n_samples) for j in idx])
    e = rel_l2(flat[idx], ref)
    print(f"noalloc 512x512: sampled rel-L2 vs oracle {e:.2e}")
    assert e <= 1e-5


def test_noalloc_captured_in_a_graph(pa):
    import paper_2404_10928_amd._lib as L
    lib = L.load()
    g = ring_geom(n=(160, 144), S=120, K=700)
    dg = pa.DeviceGeometry(g, "cuda")
    pa.tuning_set(dg, TILE, torch.float32)
    cg = dg.c_struct()
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda")
    y = torch.zeros(g.data_shape, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # first call on the device outside the capture
        L.check(lib.pa_forward_noalloc(ctypes.byref(cg), L.PA_F32, x.data_ptr(), y.data_ptr(), side.cuda_stream))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        L.check(lib.pa_forward_noalloc(ctypes.byref(cg), L.PA_F32, x.data_ptr(), y.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream))
    for rep in range(3):
        xv = np.random.default_rng([7008, rep]).uniform(size=g.image_shape).astype(np.float32)
        x.copy_(torch.from_numpy(xv))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        y_na, y_ws = run_pair(pa, dg, x)   # eager calls between replays
        assert torch.equal(y, y_ws) and torch.equal(y_na, y_ws)
    print("noalloc graph replays equal the eager workspace call")


def test_noalloc_refuses_rows_beyond_the_scratch(pa):
    import paper_2404_10928_amd._lib as L
    lib = L.load()
    g = ring_geom(n=(1024, 1024), S=256, K=2048)
    dg = pa.DeviceGeometry(g, "cuda")
    pa.tuning_set(dg, {"fwd_mode": 3, "fwd_tile": (1, 1, 1)}, torch.float32)
    cg = dg.c_struct()
    assert int(lib.pa_forward_workspace_bytes(ctypes.byref(cg), L.PA_F32)) > (64 << 20)
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda")
    y = torch.zeros(g.data_shape, dtype=torch.float32, device="cuda")
    st = lib.pa_forward_noalloc(ctypes.byref(cg), L.PA_F32, x.data_ptr(), y.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    assert st == L.PA_ERR_UNSUPPORTED and "PA_NOALLOC_SCRATCH_BYTES" in L.last_error()
    pa.tuning_clear()
