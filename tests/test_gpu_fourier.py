"""Spatial -> Fourier ingest (Sec. 3.5) on the GPU against the oracle.

The device evaluates the unitary 2-D DFT at the kept support points with
FP64 sums and stores complex64 values, then pushes them into the sparse
path.  The oracle takes the same support and transform in FP64 and rounds
the coefficients to complex64 as the device stores them, so both sides run
the DMD on the same data.  Tolerances: Gram 1e-6 sqrt(G_ii G_jj) (the
device's coefficients differ from the rounded oracle ones at most by one
complex64 rounding); sigma as the dense tests; lambda 1e-6 (a coefficient
that rounds differently moves lambda by ~1e-7 kappa); modes 1e-4.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import fourier as fo
from oracle import metrics
from test_gpu_dense import sigma_tol

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def run_fourier(frames, H, W, m, r, nkeep, T):
    dmd = _dmd()
    n = H * W
    X = torch.from_numpy(frames.T.reshape(-1, H, W).copy()).cuda()
    s = dmd.Stream(n, m, r, dtype="c64_csr", max_nnz=nkeep)
    s.fourier_setup(H, W, nkeep)
    for t in range(T):
        s.push_fourier(X[t])
    return s


def oracle_coeffs(frames, H, W, idx):
    return fo.fourier_frames(frames, H, W, idx).astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("H,W,nkeep", [(60, 80, 300), (45, 64, 211)])
def test_fourier_ingest_matches_oracle(H, W, nkeep):
    m, r = 20, 8
    T = m + 3
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, T)
    s = run_fourier(frames, H, W, m, r, nkeep, T)
    idx = fo.lowest_k_support(H, W, nkeep)
    assert np.array_equal(s.fourier_support(), idx)
    C = oracle_coeffs(frames[:, -(m + 1):], H, W, idx)
    G = s.gram()
    Gr = C.conj().T @ C
    d = np.sqrt(np.outer(np.diag(Gr).real, np.diag(Gr).real))
    assert np.max(np.abs(G - Gr) / d) < 1e-6
    ref = oracle.exact_dmd(C[:, :m], C[:, 1:], r)
    lam, sig, _ = s.eigs()
    k = lam.size
    assert k == ref.r_eff
    assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= np.maximum(sigma_tol(ref.sigma[:k]), 1e-6))
    err, perm = metrics.eig_relerr(lam, ref.lam)
    assert err.max() < 1e-6, err.max()
    phi = s.modes().cpu().numpy()
    outside = np.setdiff1d(np.arange(H * W), idx)
    assert np.all(phi[outside, :k] == 0)
    for i in range(k):
        assert metrics.phase_aligned_relerr(phi[idx, i], ref.Phi[:, perm[i]]) < 1e-4
    s.close()


def test_full_support_is_the_spatial_dmd():
    """Keeping every coefficient: sigma and lambda of the spatial frames (Sec. 3.5)."""
    H, W, m, r = 24, 20, 12, 6
    T = m + 1
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=2.0).frames(0, T)
    s = run_fourier(frames, H, W, m, r, H * W, T)
    F = oracle.as_fp64(frames)
    ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r)
    lam, sig, _ = s.eigs()
    k = lam.size
    assert k == ref.r_eff
    assert np.max(np.abs(sig - ref.sigma[:k]) / ref.sigma[:k]) < 1e-5
    assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-4
    s.close()


def test_fourier_full_size_512():
    """The sparse configuration's size: 512 x 512 frames, 2,621 kept coefficients, m = 128, r = 24."""
    H = W = 512
    m, r, nkeep = 128, 24, 2621
    T = m + 2
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=12.0).frames(0, T)
    s = run_fourier(frames, H, W, m, r, nkeep, T)
    idx = fo.lowest_k_support(H, W, nkeep)
    assert np.array_equal(s.fourier_support(), idx)
    C = oracle_coeffs(frames[:, -(m + 1):], H, W, idx)
    ref = oracle.exact_dmd(C[:, :m], C[:, 1:], r)
    lam, sig, _ = s.eigs()
    k = lam.size
    assert k == ref.r_eff
    assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= np.maximum(sigma_tol(ref.sigma[:k]), 1e-6))
    assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-6
    s.close()


def test_fourier_argument_errors():
    dmd = _dmd()
    with dmd.Stream(4800, 8, 4, dtype="c64_csr", max_nnz=100) as s:
        with pytest.raises(dmd.DMDError) as ei:
            s.push_fourier(torch.zeros((60, 80), device="cuda"))
        assert ei.value.code == dmd.E_NOT_READY
        for args in [(60, 81, 50), (60, 80, 0), (60, 80, 101)]:
            with pytest.raises(dmd.DMDError) as ei:
                s.fourier_setup(*args)
            assert ei.value.code == dmd.E_INVAL
    with dmd.Stream(4800, 8, 4) as s:
        with pytest.raises(dmd.DMDError) as ei:
            s.fourier_setup(60, 80, 50)
        assert ei.value.code == dmd.E_UNSUPPORTED
