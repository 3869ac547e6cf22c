"""The allocation-free cost-model forward pass (shp_mlp_forward_noalloc, a
static per-device work array) against shp_mlp_forward with a caller work
buffer, through the C ABI: two calls in a row, the second with fewer samples,
each equal bit for bit (the same kernels in the same order), and the size
limit rejected before any launch."""
import ctypes

import numpy as np
import pytest

from oracle import mlp_oracle as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2604_04644_amd import shp
    L = shp.lib()
    vp = ctypes.c_void_p
    L.shp_mlp_num_params.argtypes = [ctypes.POINTER(ctypes.c_int)]
    L.shp_mlp_work_floats.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    L.shp_mlp_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp]
    L.shp_mlp_forward_noalloc.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    for f in (L.shp_mlp_num_params, L.shp_mlp_work_floats, L.shp_mlp_forward, L.shp_mlp_forward_noalloc):
        f.restype = ctypes.c_int
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_forward_matches_buffered_forward(L):
    print("[no-alloc] MLP forward with the static work array vs a caller work buffer", flush=True)
    from paper_2604_04644_amd import shp
    n = ctypes.c_int()
    assert L.shp_mlp_num_params(ctypes.byref(n)) == 0
    rng = np.random.default_rng(12)
    params = torch.from_numpy(rng.normal(0, 0.3, n.value).astype(np.float32)).cuda()
    stream = shp._stream(torch)
    for ns in (3000, 700):
        X = torch.from_numpy(rng.normal(0, 1, (ns, 11)).astype(np.float32)).cuda()
        m = ctypes.c_longlong()
        assert L.shp_mlp_work_floats(ns, ctypes.byref(m)) == 0
        work = torch.empty(m.value, dtype=torch.float32, device="cuda")
        y_ref = torch.full((ns,), float("nan"), dtype=torch.float32, device="cuda")
        y = torch.full((ns,), float("nan"), dtype=torch.float32, device="cuda")
        assert L.shp_mlp_forward(_p(params), _p(X), ns, _p(y_ref), _p(work), stream) == 0
        assert L.shp_mlp_forward_noalloc(_p(params), _p(X), ns, _p(y), stream) == 0, L.shp_last_error()
        torch.cuda.synchronize()
        a, b = y.cpu().numpy(), y_ref.cpu().numpy()
        yo, _ = M.forward(params.cpu().numpy().astype(np.float64), X.cpu().numpy().astype(np.float64))
        print(f"    n={ns}: bitwise equal {np.array_equal(a, b)}, vs FP64 oracle "
              f"{np.abs(a - yo).max() / max(1.0, np.abs(yo).max()):.2e}", flush=True)
        assert np.array_equal(a, b)
        assert np.abs(a - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())
    X = torch.zeros(4097, 11, dtype=torch.float32, device="cuda")
    y = torch.zeros(4097, dtype=torch.float32, device="cuda")
    assert L.shp_mlp_forward_noalloc(_p(params), _p(X), 4097, _p(y), stream) == -1
    assert b"4096" in L.shp_last_error()
    assert L.shp_mlp_forward_noalloc(_p(params), _p(X), 0, _p(y), stream) == -1
    assert L.shp_mlp_forward_noalloc(None, _p(X), 10, _p(y), stream) == -1
