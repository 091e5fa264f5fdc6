"""The two symmetric eigensolvers (Jacobi; Householder tridiagonalization +
multisection + twisted factorizations) against the FP64 oracle and each other,
including windows too large for LDS (m = 128, 256) and Hermitian windows.

Tolerances as in the dense tests: sigma_k 1e-11 + 1e-13 (sigma_1/sigma_k)^2,
lambda 1e-8, V columns 1e-7 (canonical phases on both sides), Phi 2e-4 (FP32
projections) or 1e-8 (FP64).
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_dense import check_window, sigma_tol

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


@pytest.mark.parametrize("solver", ["jacobi", "tridiag"])
@pytest.mark.parametrize("n,m,r", [(4133, 16, 6), (4096, 33, 10), (3000, 64, 20)])
def test_modal_fp64_both_solvers(solver, n, m, r):
    dmd = _dmd()
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, m + 3)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype="f64", eig_solver=solver) as s:
        for t in range(m + 3):
            s.push(X[t])
            if t >= m:
                check_window(s, frames[:, t - m:t + 1], m, r, phi_tol=1e-8, pod=(t == m + 2))


@pytest.mark.parametrize("m,r", [(128, 32), (256, 32), (100, 24)])
def test_large_windows_tridiag(m, r):
    """Windows beyond the LDS path (m > 64): the matrix lives in the workspace."""
    dmd = _dmd()
    n = 200 * 200
    frames = gen.BlobVideo(height=200, width=200, blob_sigma=6.0).frames(0, m + 2)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, eig_solver="tridiag") as s:
        for t in range(m + 2):
            s.push(X[t])
        check_window(s, frames[:, 1:], m, r, phi_tol=2e-4)


def test_solvers_agree_on_video():
    dmd = _dmd()
    H, W, m, r = 90, 160, 64, 20
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, m + 1)
    X = torch.from_numpy(frames.T.copy()).cuda()
    out = {}
    for solver in ("jacobi", "tridiag"):
        with dmd.Stream(H * W, m, r, eig_solver=solver) as s:
            for t in range(m + 1):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            sg, V, _ = s.svd()
            out[solver] = (lam, sig, V)
    (lj, sj, Vj), (lt, st, Vt) = out["jacobi"], out["tridiag"]
    assert lj.size == lt.size
    assert np.all(np.abs(sj - st) <= sigma_tol(sj) * sj)
    assert metrics.eig_relerr(lt, lj)[0].max() < 1e-8
    assert np.max(np.abs(Vj - Vt)) < 1e-7


@pytest.mark.parametrize("solver", ["jacobi", "tridiag"])
def test_sparse_hermitian_both_solvers(solver):
    dmd = _dmd()
    fs = gen.FourierSparse(side=64, nnz=120, redraw=0.05)
    m, r = 40, 10
    dense = []
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=130, eig_solver=solver) as s:
        for t in range(m + 1):
            idx, val = fs.frame(t)
            s.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
            dense.append(oracle.densify(idx, val, fs.n))
        W = np.stack(dense, axis=1)
        ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
        lam, sig, _ = s.eigs()
        assert lam.size == ref.r_eff
        assert np.all(metrics.sigma_relerr(sig, ref.sigma[:lam.size]) <= sigma_tol(ref.sigma[:lam.size]))
        assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-8
        sg, V, _ = s.svd()
        for i in range(lam.size):
            assert metrics.phase_aligned_relerr(V[:, i], ref.V[:, i]) < 1e-7


def test_solver_option_checks():
    dmd = _dmd()
    with pytest.raises(dmd.DMDError) as ei:
        dmd.Stream(1000, 8, 4, eig_solver="tridiag", warm_start=True)
    assert ei.value.code == dmd.E_INVAL
