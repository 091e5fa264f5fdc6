"""Spatial -> Fourier ingest (Sec. 3.5): test infrastructure only.

The SVD and the DMD of a snapshot matrix are unchanged by a unitary change
of basis applied to every snapshot (Sec. 3.5), so a stream of spatial frames
may be handed to the sparse path as their 2-D discrete Fourier coefficients,
of which only the lowest wavenumbers are kept.  This module states, in FP64,
what that ingest computes:

* the unitary 2-D DFT of an H x W frame (row-major),
  xhat[ky, kx] = (H W)^-1/2 sum_{y, x} x[y, x] exp(-2 pi i (ky y / H + kx x / W)),
  flattened row-major (index ky W + kx) -- NumPy's fft2 with norm="ortho" is
  the library step;
* signed wavenumbers: bin k of N stands for k when k < (N + 1) // 2, else for
  k - N (NumPy's fftfreq order);
* the support: the nkeep bins with the smallest ky^2 + kx^2 (signed), ties
  broken by the flattened index, listed in increasing index order.
"""

import numpy as np

from .dmd import as_fp64


def signed_bins(N: int) -> np.ndarray:
    k = np.arange(N)
    return np.where(k < (N + 1) // 2, k, k - N)


def lowest_k_support(H: int, W: int, nkeep: int) -> np.ndarray:
    """Flattened indices of the nkeep lowest-|k| bins, increasing."""
    ky = signed_bins(H)[:, None]
    kx = signed_bins(W)[None, :]
    k2 = (ky * ky + kx * kx).ravel()
    order = np.lexsort((np.arange(H * W), k2))  # by k2, then by index
    return np.sort(order[:nkeep]).astype(np.int32)


def fourier_coefficients(frame, H: int, W: int, idx) -> np.ndarray:
    """The unitary 2-D DFT of one frame at the flattened indices idx."""
    x = as_fp64(frame).reshape(H, W)
    return np.fft.fft2(x, norm="ortho").ravel()[np.asarray(idx)]


def fourier_frames(frames, H: int, W: int, idx) -> np.ndarray:
    """Columns of `frames` (n x T, n = H W) mapped to their kept coefficients."""
    F = as_fp64(frames)
    return np.stack([fourier_coefficients(F[:, t], H, W, idx) for t in range(F.shape[1])], axis=1)
