"""Pins of the Fourier-ingest oracle (Sec. 3.5) by facts other than itself:
closed forms of single waves (sign and normalization of the transform), an
explicit double sum on a tiny grid, Parseval's identity, a support listed by
hand, and the unitary invariance of the DMD that the sparse path relies on."""

import numpy as np

import gen
import oracle
from oracle import fourier as fo
from oracle import metrics


def test_single_cosine_and_sine_closed_forms():
    H, W = 12, 10
    ky0, kx0 = 2, 3
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    ph = 2 * np.pi * (ky0 * y / H + kx0 * x / W)
    full = np.arange(H * W)
    c = fo.fourier_coefficients(np.cos(ph).ravel(), H, W, full).reshape(H, W)
    s = fo.fourier_coefficients(np.sin(ph).ravel(), H, W, full).reshape(H, W)
    half = np.sqrt(H * W) / 2
    expect_c = np.zeros((H, W), complex)
    expect_c[ky0, kx0] = half
    expect_c[-ky0, -kx0] = half
    # exp(-i k.x) transform: sin -> -i/2 at +k and +i/2 at -k
    expect_s = np.zeros((H, W), complex)
    expect_s[ky0, kx0] = -1j * half
    expect_s[-ky0, -kx0] = 1j * half
    assert np.max(np.abs(c - expect_c)) < 1e-12
    assert np.max(np.abs(s - expect_s)) < 1e-12


def test_explicit_double_sum_on_a_tiny_grid():
    rng = np.random.default_rng(5)
    H, W = 4, 6
    x = rng.standard_normal(H * W)
    X = x.reshape(H, W)
    ref = np.zeros((H, W), complex)
    for ky in range(H):
        for kx in range(W):
            acc = 0j
            for yy in range(H):
                for xx in range(W):
                    acc += X[yy, xx] * np.exp(-2j * np.pi * (ky * yy / H + kx * xx / W))
            ref[ky, kx] = acc / np.sqrt(H * W)
    got = fo.fourier_coefficients(x, H, W, np.arange(H * W)).reshape(H, W)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_parseval():
    rng = np.random.default_rng(6)
    H, W = 16, 24
    x = rng.standard_normal(H * W)
    xh = fo.fourier_coefficients(x, H, W, np.arange(H * W))
    assert abs(np.linalg.norm(xh) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def test_support_listed_by_hand():
    # 4 x 4 grid: signed bins 0, 1, -2, -1.  |k|^2 = 0 at index 0; |k|^2 = 1 at
    # (0, 1) -> 1, (0, -1) -> 3, (1, 0) -> 4, (-1, 0) -> 12; |k|^2 = 2 at
    # (1, 1) -> 5, (1, -1) -> 7, (-1, 1) -> 13, (-1, -1) -> 15.
    assert list(fo.signed_bins(4)) == [0, 1, -2, -1]
    assert list(fo.signed_bins(5)) == [0, 1, 2, -2, -1]
    assert list(fo.lowest_k_support(4, 4, 1)) == [0]
    assert list(fo.lowest_k_support(4, 4, 3)) == [0, 1, 3]          # ties by index
    assert list(fo.lowest_k_support(4, 4, 5)) == [0, 1, 3, 4, 12]
    assert list(fo.lowest_k_support(4, 4, 7)) == [0, 1, 3, 4, 5, 7, 12]
    assert len(fo.lowest_k_support(30, 20, 600)) == 600


def test_dmd_is_invariant_under_the_unitary_transform():
    """Full support: the Fourier stream has the spatial stream's sigma and
    lambda, and its modes are the transformed spatial modes (Sec. 3.5)."""
    H, W, m, r = 24, 20, 10, 6
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=2.0).frames(0, m + 1).astype(np.float64)
    full = np.arange(H * W)
    Fh = fo.fourier_frames(frames, H, W, full)
    a = oracle.exact_dmd(frames[:, :m], frames[:, 1:], r)
    b = oracle.exact_dmd(Fh[:, :m], Fh[:, 1:], r)
    assert a.r_eff == b.r_eff
    k = a.r_eff
    assert np.max(np.abs(a.sigma[:k] - b.sigma[:k]) / a.sigma[:k]) < 1e-10
    err, perm = metrics.eig_relerr(b.lam, a.lam)
    assert err.max() < 1e-8
    for i in range(k):
        phat = fo.fourier_coefficients(a.Phi[:, perm[i]].real, H, W, full) + \
            1j * fo.fourier_coefficients(a.Phi[:, perm[i]].imag, H, W, full)
        assert metrics.phase_aligned_relerr(b.Phi[:, i], phat) < 1e-8
