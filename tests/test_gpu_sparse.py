"""GPU parity of the sparse complex (Fourier-domain) path against the oracle.

The oracle densifies every CSR snapshot (exactly) and runs the same dense
complex exact DMD; by the unitary invariance of Sec. 3.5 this is also the DMD
of the spatial fields (pinned on the CPU in test_oracle_pins.py).

Tolerances: Hermitian Gram |dG_ij| <= 1e-12 sqrt(G_ii G_jj) (complex64
products are exact in FP64); sigma as the dense path; lambda 1e-13 + 32 u kappa_i (as the dense path); modes
(FP32 projection of complex64 data) 2e-4.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_dense import check_lambda

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def push_frame(s, fs, t):
    idx, val = fs.frame(t)
    s.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
    return oracle.densify(idx, val, fs.n)


def check_sparse_window(s, W, m, r, phi_tol=2e-4):
    ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
    lam, sig, rc = s.eigs()
    k = lam.size
    assert k == ref.r_eff
    err_s = metrics.sigma_relerr(sig, ref.sigma[:k])
    assert np.all(err_s <= 1e-11 + 1e-13 * (ref.sigma[0] / ref.sigma[:k]) ** 2), err_s
    err_l, perm = check_lambda(lam, ref)
    sg, V, _ = s.svd()
    for i in range(k):
        assert metrics.phase_aligned_relerr(V[:, i], ref.V[:, i]) < 1e-7
    phi = s.modes().cpu().numpy()
    for i in range(k):
        assert metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]]) < phi_tol
    return ref


@pytest.mark.parametrize("side,nnz,m,r", [(64, 80, 16, 6), (48, 61, 9, 5)])
def test_sparse_every_window(side, nnz, m, r):
    dmd = _dmd()
    fs = gen.FourierSparse(side=side, nnz=nnz, redraw=0.05)
    T = m + 8
    dense = []
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=nnz + 5) as s:
        for t in range(T):
            dense.append(push_frame(s, fs, t))
            lo = max(0, t - m)
            Wn = np.stack(dense[lo:t + 1], axis=1)
            G = s.gram()
            ref = Wn.conj().T @ Wn
            d = np.sqrt(np.outer(np.diag(ref).real, np.diag(ref).real))
            assert np.all(np.abs(G - ref) <= 1e-12 * d + 1e-300)
            if t >= m:
                check_sparse_window(s, Wn, m, r)


def test_sparse_rejects_bad_indices_and_keeps_window():
    dmd = _dmd()
    fs = gen.FourierSparse(side=32, nnz=40)
    m, r = 8, 4
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=64) as s:
        dense = [push_frame(s, fs, t) for t in range(m + 1)]
        G0 = s.gram()
        idx, val = fs.frame(m + 1)
        bad = idx.copy()
        bad[3], bad[4] = bad[4], bad[3]          # not increasing
        s.push_csr(torch.from_numpy(bad).cuda(), torch.from_numpy(val).cuda())
        with pytest.raises(dmd.DMDError) as ei:
            s.sync()
        assert ei.value.code == dmd.E_INVAL
        assert np.array_equal(s.gram(), G0)
        # out of range past n, negative, and the largest int32: the pushed
        # snapshot's own product never reads the scatter vector at its
        # indices, so none of these addresses memory outside it
        for pos, value in ((-1, fs.n + 5), (0, -1), (-1, 2**31 - 1), (5, -2**31)):
            oob = idx.copy()
            oob[pos] = value
            s.push_csr(torch.from_numpy(oob).cuda(), torch.from_numpy(val).cuda())
            with pytest.raises(dmd.DMDError) as ei:
                s.sync()
            assert ei.value.code == dmd.E_INVAL
            assert np.array_equal(s.gram(), G0)
        dense.append(push_frame(s, fs, m + 1))   # a good push still works afterwards
        check_sparse_window(s, np.stack(dense[1:], axis=1), m, r)


def test_sparse_full_size_last_window():
    """512^2 Fourier coefficients, 1 % density, m = 128, r = 24: the last window."""
    dmd = _dmd()
    fs = gen.FourierSparse(side=512, nnz=2621, redraw=0.05)
    m, r = 128, 24
    T = m + 3
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=2621) as s:
        frames = []
        for t in range(T):
            idx, val = fs.frame(t)
            frames.append((idx, val))
            s.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
        W = np.stack([oracle.densify(i, v, fs.n) for i, v in frames[T - m - 1:]], axis=1)
        check_sparse_window(s, W, m, r)
