"""The allocation-free whole-window Gram (dmd_window_gram_noalloc) against the
allocating call (dmd_window_gram) on the same inputs: the same kernels and
row splits, so every entry is bitwise equal.  Two calls in a row on one
device, the second with a smaller window, so the second call runs over the
scratch the first one left behind.  The largest first call fills every
partial tile the scratch holds (257 columns)."""

import ctypes

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def _frames(n, k, dtype):
    """k snapshots of length n as a (k, n) CUDA view with 16-byte aligned rows
    (the leading dimension rounded up; ragged n stays ragged)."""
    v = gen.BlobVideo(height=(n + 127) // 128, width=128, n=n, blob_sigma=5.0)
    F = v.frames(0, k).astype(np.float32 if dtype == "f32" else np.float64)
    per = 16 // F.dtype.itemsize
    ld = (n + per - 1) // per * per
    Xp = torch.zeros((k, ld), dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")
    Xp[:, :n] = torch.from_numpy(F.T.copy()).cuda()
    return F, Xp[:, :n]


def _gram_err(G, ref):
    d = np.sqrt(np.outer(np.abs(np.diag(ref)), np.abs(np.diag(ref))))
    return np.max(np.abs(G - ref) / d)


@pytest.mark.parametrize("dtype,prec,tol", [
    ("f32", "default", 2e-5), ("f32", "bf16x3", 2e-4), ("f64", "default", 1e-12),
])
@pytest.mark.parametrize("first,second", [((70001, 257), (5003, 66)), ((9000, 130), (333, 3))])
def test_noalloc_matches_allocating_call(dtype, prec, tol, first, second):
    dmd = _dmd()
    for n, k in (first, second):
        print(f"noalloc dtype={dtype} prec={prec} n={n} k={k}", flush=True)
        F, X = _frames(n, k, dtype)
        out = torch.full((k, k), np.nan, dtype=torch.float64, device="cuda")
        G = dmd.window_gram(X, precision=prec, out=out, noalloc=True).cpu().numpy()
        ref = dmd.window_gram(X, precision=prec).cpu().numpy()
        assert np.array_equal(G, ref)
        assert _gram_err(G, oracle.gram(F)) < tol


def test_noalloc_on_a_side_stream_and_errors():
    dmd = _dmd()
    n, k = 12345, 40
    F, X = _frames(n, k, "f64")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = torch.empty((k, k), dtype=torch.float64, device="cuda")
        dmd.window_gram(X, out=out, noalloc=True, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), dmd.window_gram(X).cpu().numpy())
    lib = dmd.load()
    G = torch.empty((300, 300), dtype=torch.float64, device="cuda")
    Xb = torch.zeros((258, 256), dtype=torch.float32, device="cuda")
    assert lib.dmd_window_gram_noalloc(ctypes.c_void_p(Xb.data_ptr()), 256, 256, 258, 0, 0,
                                       ctypes.c_void_p(G.data_ptr()), 300, None) == dmd.E_INVAL
    assert "ncols" in dmd.last_error()
