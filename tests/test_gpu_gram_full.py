"""Whole-window Gram on the matrix cores (Algorithm 1 first step) and the
precision study: FP64, FP32 and BF16x3 (hi*hi + hi*lo + lo*hi) products.

Tolerances per precision (per Gram entry, relative to sqrt(G_ii G_jj)):
* FP64 MFMA: 1e-12 (exact FP32 products, FP64 sums in another order);
* FP32 MFMA: products rounded to 2^-24 and FP32 sums over a row split
  (<= 2^14 rows here), then FP64 across splits: 2e-5;
* BF16x3: products carry ~2^-16 relative error (the dropped lo*lo term and
  the bf16 rounding of lo), FP32 sums: 2e-4.
Singular values: the method of snapshots squares the condition number.  By
Weyl's inequality a Gram error dG moves sigma_k by at most ||dG||_2 / sigma_k,
a relative error of ||dG||_2 / sigma_k^2; every sigma_k must respect that bound
(dG measured from the GPU's own Gram) and the leading ones must meet the stated
tolerance (1e-5 for FP32, 1e-4 for BF16x3).
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def padded_columns(F):
    """The columns of F (n x k) as a (k, n) CUDA view whose rows start 16-byte
    aligned (leading dimension n rounded up to 16 bytes), as the stateless
    Gram requires; ragged n is then the caller's padding, not a copy."""
    n, k = F.shape
    per = 16 // F.dtype.itemsize
    ld = (n + per - 1) // per * per
    Xp = torch.zeros((k, ld), dtype=torch.float32 if F.dtype == np.float32 else torch.float64, device="cuda")
    Xp[:, :n] = torch.from_numpy(F.T.copy()).cuda()
    return Xp[:, :n]


def gram_err(G, ref):
    d = np.sqrt(np.outer(np.abs(np.diag(ref)), np.abs(np.diag(ref))))
    return np.max(np.abs(G - ref) / d)


def test_load_window_fp64_then_stream():
    dmd = _dmd()
    g = gen.ModalStream(n=5000, noise=1e-3)
    m, r = 32, 10
    F = g.frames(0, m + 6)
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(5000, m, r, dtype="f64") as s:
        s.load_window(X[: m + 1])
        assert gram_err(s.gram(), oracle.gram(F[:, : m + 1])) < 1e-12
        ref = oracle.exact_dmd(F[:, :m], F[:, 1:m + 1], r)
        lam, sig, _ = s.eigs()
        assert metrics.sigma_relerr(sig, ref.sigma[:r]).max() < 1e-10
        assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-8
        for t in range(m + 1, m + 6):   # streaming continues from the bulk window
            s.push(X[t])
            W = F[:, t - m:t + 1]
            assert gram_err(s.gram(), oracle.gram(W)) < 1e-12
            ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
            lam, sig, _ = s.eigs()
            assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-8


def test_partial_window_load_reports_not_ready():
    dmd = _dmd()
    g = gen.ModalStream(n=3000, noise=1e-3)
    m, r = 16, 6
    F = g.frames(0, m + 1)
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(3000, m, r, dtype="f64") as s:
        s.load_window(X[:10])
        assert s.info().count == 10
        assert gram_err(s.gram(), oracle.gram(F[:, :10])) < 1e-12
        with pytest.raises(dmd.DMDError) as ei:
            s.eigs()
        assert ei.value.code == dmd.E_NOT_READY
        for t in range(10, m + 1):
            s.push(X[t])
        assert gram_err(s.gram(), oracle.gram(F)) < 1e-12
        lam, sig, _ = s.eigs()
        ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r)
        assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-8


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5), ("bf16x3", 2e-4)])
@pytest.mark.parametrize("H,W,m", [(128, 128, 64), (100, 130, 37)])
def test_resync_gram_precision(prec, tol, H, W, m):
    dmd = _dmd()
    v = gen.BlobVideo(height=H, width=W, blob_sigma=4.0)
    F = v.frames(0, m + 1)
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(H * W, m, min(m, 12), precision=prec) as s:
        for t in range(m + 1):
            s.push(X[t])
        G_stream = s.gram()
        s.resync()
        G = s.gram()
    ref = oracle.gram(F)
    assert gram_err(G_stream, ref) < 1e-12        # the streamed Gram is always FP64
    e = gram_err(G, ref)
    assert e < tol, e
    if prec != "fp64":
        assert e > 1e-12  # the reduced precision is really in effect


@pytest.mark.parametrize("prec,tol,need", [("fp32", 1e-5, 4), ("bf16x3", 1e-4, 3)])
def test_precision_study_travelling_waves(prec, tol, need):
    """Sigma and lambda with a Gram in reduced precision vs the FP64 oracle on
    data with condition ~10^3.5 (8 waves, amplitudes 10^(-k/2)).

    Weyl's inequality bounds the effect of the Gram error dG on each singular
    value: |sigma'_k - sigma_k| <= ||dG||_2 / sigma_k, i.e. a relative error of
    at most ||dG||_2 / sigma_k^2 (dG measured from the GPU's own Gram).  Every
    sigma_k must respect that bound, and at least `need` of them must meet the
    stated tolerance."""
    dmd = _dmd()
    w = gen.TravelingWaves(n=1 << 16, n_waves=8)
    m, r = 48, 16
    F = w.frames(0, m + 1)
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(1 << 16, m, r, precision=prec, rcond=0.0) as s:
        for t in range(m + 1):
            s.push(X[t])
        lam64, sig64, _ = s.eigs()
        s.resync()
        lam, sig, _ = s.eigs()
        G = s.gram()
    ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r, r_eff=r)
    err64 = metrics.sigma_relerr(sig64, ref.sigma[:r])
    assert err64.max() < 1e-9                      # streamed FP64 Gram
    dG = np.linalg.norm(G[:m, :m] - oracle.gram(F[:, :m]), 2)
    k = sig.size
    err = metrics.sigma_relerr(sig, ref.sigma[:k])
    bound = dG / ref.sigma[:k] ** 2 + 1e-12
    assert np.all(err <= bound), (err, bound)
    meets = err <= tol
    assert meets[:need].all(), (err, bound)
    # the generating eigenvalues e^{+-i w} are recovered where sigma is resolved
    lam_err, perm = metrics.eig_relerr(lam, w.true_eigs())
    assert np.median(lam_err) < 1e-2


@pytest.mark.parametrize("dtype,prec,tol", [
    ("f64", "default", 1e-12), ("f32", "fp64", 1e-12), ("f32", "default", 2e-5), ("f32", "bf16x3", 2e-4),
])
@pytest.mark.parametrize("n,k", [(9000, 33), (70001, 65), (5000, 257), (333, 1)])
def test_stateless_window_gram(dtype, prec, tol, n, k):
    """dmd_window_gram: G = X^* X of a caller's matrix (no stream handle),
    every entry within the precision's bound of the oracle; it equals the
    Gram a stream computes when it loads the same window (same kernel, same
    row splits), bit for bit."""
    dmd = _dmd()
    v = gen.BlobVideo(height=(n + 127) // 128, width=128, n=n, blob_sigma=5.0)
    F = v.frames(0, k).astype(np.float32 if dtype == "f32" else np.float64)
    X = padded_columns(F)
    G = dmd.window_gram(X, precision=prec).cpu().numpy()
    ref = oracle.gram(F)
    assert np.array_equal(G, G.T)
    assert gram_err(G, ref) < tol, gram_err(G, ref)
    if k >= 3:
        with dmd.Stream(n, k - 1, 1, dtype=dtype, precision=prec, auto_solve=False) as s:
            s.load_window(X)
            assert np.array_equal(s.gram(), G)


def test_stateless_window_gram_padding_and_errors():
    dmd = _dmd()
    from paper_1612_07875_amd import binding
    n, k = 4096, 20
    X = torch.rand((k, n), dtype=torch.float64, device="cuda")
    out = torch.full((k + 3, k + 5), -7.0, dtype=torch.float64, device="cuda")
    dmd.window_gram(X, out=out)
    o = out.cpu().numpy()
    np.testing.assert_array_equal(o[k:, :], -7.0)           # padding untouched
    np.testing.assert_array_equal(o[:k, k:], -7.0)
    assert gram_err(o[:k, :k], oracle.gram(X.cpu().numpy().T)) < 1e-12
    lib = dmd.load()
    G = torch.empty((k, k), dtype=torch.float64, device="cuda")
    Xs = X[:, 1:]                                            # columns not 16-byte aligned
    assert lib.dmd_window_gram(Xs.data_ptr(), n, n - 1, k, 1, 0, G.data_ptr(), k, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(X.data_ptr(), n, n, 258, 1, 0, G.data_ptr(), 258, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(X.data_ptr(), n, n, k, 1, 2, G.data_ptr(), k, None) == dmd.E_UNSUPPORTED
    assert lib.dmd_window_gram(X.data_ptr(), n, n, k, 1, 0, G.data_ptr(), k - 1, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(None, n, n, k, 1, 0, G.data_ptr(), k, None) == dmd.E_INVAL
    assert binding.DTYPES["f64"] == 1
