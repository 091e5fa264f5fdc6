"""Degenerate windows, checked against their closed forms.

* All-zero snapshots: every singular value is zero, so no mode is kept:
  DMD_W_RANK with r_eff = 0, and the modes output is left untouched.
* Constant snapshots x_t = x: X = x 1^T has rank one and X' = X, so the one
  kept eigenvalue is exactly 1 and its mode is parallel to x (Eq. Atilde,
  Eq. Phi with a single singular triplet).
* Geometric snapshots x_t = rho^t v (the smallest sizes the boundary allows:
  n = 1, m = 2, and a ragged n = 3): X' = rho X, so the eigenvalue is rho.
"""

import numpy as np
import pytest
import torch

from oracle import metrics

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def push_all(s, frames):
    X = torch.from_numpy(np.ascontiguousarray(frames.T)).cuda()
    for t in range(X.shape[0]):
        s.push(X[t])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_zero_window(dtype):
    dmd = _dmd()
    n, m, r = 1000, 8, 4
    frames = np.zeros((n, m + 1), dtype=np.float32 if dtype == "f32" else np.float64)
    with dmd.Stream(n, m, r, dtype=dtype) as s:
        push_all(s, frames)
        lam, sig, rc = s.eigs()
        assert rc == dmd.W_RANK and lam.size == 0 and sig.size == 0
        sentinel = 7.0 + 7.0j
        out = torch.full((r, n), sentinel, dtype=s.mode_dtype, device="cuda").T
        s.modes(out)
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == sentinel)


@pytest.mark.parametrize("dtype,tol_phi", [("f32", 1e-6), ("f64", 1e-12)])
def test_constant_window_has_eigenvalue_one(dtype, tol_phi):
    dmd = _dmd()
    n, m, r = 5000, 12, 5
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n)
    if dtype == "f32":
        x = x.astype(np.float32)
    frames = np.repeat(x[:, None], m + 1, axis=1)
    with dmd.Stream(n, m, r, dtype=dtype) as s:
        push_all(s, frames)
        lam, sig, rc = s.eigs()
        assert rc == dmd.W_RANK and lam.size == 1
        # the Gram is exact (FP32 products in FP64) up to its FP64 sums
        assert abs(lam[0] - 1.0) < 1e-12, lam
        xs = np.asarray(x, dtype=np.float64)
        assert abs(sig[0] - np.linalg.norm(xs) * np.sqrt(m)) < 1e-10 * sig[0]
        phi = s.modes().cpu().numpy()[:, 0]
        assert metrics.phase_aligned_relerr(phi / np.linalg.norm(phi), xs / np.linalg.norm(xs)) < tol_phi


@pytest.mark.parametrize("n,dtype", [(1, "f64"), (3, "f32"), (3, "f64")])
def test_geometric_window_smallest_sizes(n, dtype):
    dmd = _dmd()
    m, r, rho = 2, 1, 0.9
    v = np.arange(1, n + 1, dtype=np.float64)
    frames = np.stack([rho ** t * v for t in range(m + 1)], axis=1)
    if dtype == "f32":
        frames = frames.astype(np.float32)
    with dmd.Stream(n, m, r, dtype=dtype) as s:
        push_all(s, frames)
        lam, sig, rc = s.eigs()
        assert rc in (0, 1) and lam.size == 1
        # FP32 data: rho^t v is rounded, so X' = rho X holds to ~1e-7
        tol = 1e-12 if dtype == "f64" else 1e-6
        assert abs(lam[0] - rho) < tol, lam
        phi = s.modes().cpu().numpy()[:, 0]
        assert metrics.phase_aligned_relerr(phi / np.linalg.norm(phi), v / np.linalg.norm(v)) < tol


def test_sparse_windows_with_empty_snapshots():
    """Sparse frames with no coefficients (zero snapshots) inside the window:
    the window's DMD equals the oracle's on the densified frames; a window of
    empty frames keeps no mode."""
    import gen
    import oracle
    from test_gpu_sparse import check_sparse_window
    dmd = _dmd()
    fs = gen.FourierSparse(side=40, nnz=50, redraw=0.1)
    m, r = 10, 4
    empty_i = torch.zeros(0, dtype=torch.int32, device="cuda")
    empty_v = torch.zeros(0, dtype=torch.complex64, device="cuda")
    dense = []
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=60) as s:
        for t in range(m + 6):
            if t % 5 == 3:
                s.push_csr(empty_i, empty_v)
                dense.append(np.zeros(fs.n, dtype=np.complex128))
            else:
                idx, val = fs.frame(t)
                s.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
                dense.append(oracle.densify(idx, val, fs.n))
            if t >= m:
                check_sparse_window(s, np.stack(dense[t - m:t + 1], axis=1), m, r)
        for _ in range(m + 1):
            s.push_csr(empty_i, empty_v)
        lam, sig, rc = s.eigs()
        assert rc == dmd.W_RANK and lam.size == 0
