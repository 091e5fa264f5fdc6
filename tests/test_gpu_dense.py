"""GPU parity of the dense streaming path against the FP64 oracle.

Every case pushes seeded synthetic frames through the C ABI and compares, per
window, the streamed Gram, sigma, V, A~, lambda, W, Phi and U with the oracle
computed from the same frames (widened exactly to FP64).

Tolerances:
* Gram: products of FP32/FP64 data summed in FP64 in a different order than
  the oracle: |dG_ij| <= 1e-12 sqrt(G_ii G_jj).
* sigma_k: the method of snapshots squares the condition number, so FP64
  rounding of the Gram moves sigma_k by ~ u (sigma_1/sigma_k)^2:
  tol_k = 1e-11 + 1e-13 (sigma_1/sigma_k)^2.
* lambda (matched), per eigenvalue: 1e-13 + 32 u kappa_i, kappa_i the
  eigenvalue's first-order sensitivity to a Gram perturbation of size
  sigma_1^2 (metrics.eig_sensitivity): the method of snapshots solves from
  the FP64 Gram, whose rounding (u sigma_1^2 per entry) moves lambda_i by up
  to u kappa_i; the oracle's own Gram and SVD routes differ by at most
  0.46 u kappa_i on these workloads.  W, V, A~: 1e-7 (FP64 solves,
  well-separated data).
* Phi, U with FP64 projections: 1e-8; with FP32 projections (FP32
  coefficients, FP32 accumulation over m terms): 2e-4 relative per column.
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


def sigma_tol(sig):
    return 1e-11 + 1e-13 * (sig[0] / sig) ** 2


def eig_bound(ref):
    """Bound on the relative error of each eigenvalue, in ref's order (see the
    module docstring): 1e-13 + 32 u kappa_i."""
    return 1e-13 + 32 * 2.0 ** -52 * metrics.eig_sensitivity(ref)


def check_lambda(lam, ref):
    """Matched eigenvalue errors against eig_bound; returns the matching."""
    err_l, perm = metrics.eig_relerr(lam, ref.lam)
    bound = eig_bound(ref)[perm]
    assert np.all(err_l <= bound), (err_l, bound)
    return err_l, perm


def check_window(s, frames_window, m, r, phi_tol, pod=False, check_matrices=True):
    """Compare the GPU's latest solve with the oracle on the given (n, m+1) window."""
    F = oracle.as_fp64(frames_window)
    ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r, pod=pod)
    lam, sig, rc = s.eigs()
    assert rc in (0, 1)
    k = lam.size
    assert k == ref.r_eff, (k, ref.r_eff)
    err_s = metrics.sigma_relerr(sig, ref.sigma[:k])
    assert np.all(err_s <= sigma_tol(ref.sigma[:k])), err_s
    err_l, perm = check_lambda(lam, ref)
    if check_matrices:
        sg_all, V, _ = s.svd()
        np.testing.assert_allclose(sg_all[:k], sig, rtol=0, atol=0)
        # V columns equal up to the canonical sign (same convention on both sides)
        assert np.max(np.abs(V - ref.V)) < 1e-7 * max(1.0, (ref.sigma[0] / ref.sigma[k - 1]) ** 2 * 1e-6)
        At, W, _ = s.atilde()
        assert np.max(np.abs(At - ref.Atilde)) < 1e-7 * np.max(np.abs(ref.Atilde))
        for i in range(k):
            assert metrics.phase_aligned_relerr(W[:, i], ref.W[:, perm[i]]) < 1e-7
    phi = s.modes().cpu().numpy()
    for i in range(k):
        e = metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]])
        assert e < phi_tol, (i, e)
    if pod:
        U = s.pod().cpu().numpy()[:, :k]
        for i in range(k):
            e = np.linalg.norm(U[:, i] - ref.U[:, i]) / np.linalg.norm(ref.U[:, i])
            assert e < phi_tol, (i, e)
    return ref


def check_gram(s, window):
    G = s.gram()
    F = oracle.as_fp64(window)
    ref = oracle.gram(F)
    assert G.shape == ref.shape
    d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert np.all(np.abs(G - ref) <= 1e-12 * d + 1e-300), np.max(np.abs(G - ref) / d)


@pytest.mark.parametrize("n", [4096, 4096 + 37, 1000])
def test_modal_fp64_every_window(n):
    """Plain streaming DMD, FP64 data (n=4096, m=32, r=10, 64 frames) plus ragged n."""
    dmd = _dmd()
    m, r, T = 32, 10, 64
    g = gen.ModalStream(n=n, noise=1e-3)
    frames = g.frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype="f64") as s:
        for t in range(T):
            s.push(X[t])
            lo = max(0, t - m)
            check_gram(s, frames[:, lo:t + 1])
            if t < m:
                with pytest.raises(dmd.DMDError) as ei:
                    s.eigs()
                assert ei.value.code == dmd.E_NOT_READY
                continue
            check_window(s, frames[:, t - m:t + 1], m, r, phi_tol=1e-8, pod=(t % 8 == 0))


def test_modal_closed_form_on_gpu():
    """Noiseless modal data: the GPU recovers the generating eigenvalues."""
    dmd = _dmd()
    m, r = 32, 10
    g = gen.ModalStream(n=4096, noise=0.0)
    X = torch.from_numpy(g.frames(0, m + 1).T.copy()).cuda()
    with dmd.Stream(4096, m, r, dtype="f64", rcond=0.0) as s:
        for t in range(m + 1):
            s.push(X[t])
        lam, sig, _ = s.eigs()
    err, _ = metrics.eig_relerr(lam, g.true_eigs())
    assert err.max() < 1e-10


@pytest.mark.parametrize("H,W,m,r", [(90, 160, 64, 20), (61, 67, 16, 8), (128, 255, 33, 12)])
def test_video_fp32(H, W, m, r):
    """FP32 video frames (reduced size), FP32 projections; odd m and ragged n included."""
    dmd = _dmd()
    v = gen.BlobVideo(height=H, width=W, blob_sigma=max(3.0, H / 36))
    T = m + 6
    frames = v.frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    n = H * W
    with dmd.Stream(n, m, r, dtype="f32") as s:
        for t in range(T):
            s.push(X[t])
            if t >= m:
                check_gram(s, frames[:, t - m:t + 1])
                check_window(s, frames[:, t - m:t + 1], m, r, phi_tol=2e-4, pod=(t == T - 1))


def test_video_fp32_with_fp64_projection():
    dmd = _dmd()
    v = gen.BlobVideo(height=72, width=128, blob_sigma=4.0)
    m, r = 24, 10
    frames = v.frames(0, m + 3)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(72 * 128, m, r, dtype="f32", precision="fp64") as s:
        for t in range(m + 3):
            s.push(X[t])
        check_window(s, frames[:, 2:], m, r, phi_tol=1e-9, pod=True)


def test_bitwise_replay():
    """Fixed reduction order: two identical streams give bitwise identical results."""
    dmd = _dmd()
    v = gen.BlobVideo(height=100, width=150, blob_sigma=4.0)
    m, r = 20, 8
    X = torch.from_numpy(v.frames(0, 30).T.copy()).cuda()
    outs = []
    for _ in range(2):
        with dmd.Stream(15000, m, r) as s:
            for t in range(30):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            outs.append((s.gram(), lam, sig, s.modes().cpu().numpy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_nonfinite_snapshot_rejected_window_unchanged():
    dmd = _dmd()
    g = gen.ModalStream(n=2048, noise=1e-3)
    m, r = 8, 4
    X = torch.from_numpy(g.frames(0, 12).T.copy()).cuda()
    with dmd.Stream(2048, m, r, dtype="f64") as s:
        for t in range(10):
            s.push(X[t])
        G0 = s.gram()
        lam0, _, _ = s.eigs()
        bad = X[10].clone()
        bad[77] = float("nan")
        s.push(bad)
        with pytest.raises(dmd.DMDError) as ei:
            s.sync()
        assert ei.value.code == dmd.E_NONFINITE
        assert np.array_equal(s.gram(), G0)
        lam1, _, _ = s.eigs()
        assert np.array_equal(lam0, lam1)
        s.push(X[10])
        check_window(s, g.frames(2, m + 1), m, r, phi_tol=1e-8)


def test_reset_and_manual_solve():
    dmd = _dmd()
    g = gen.ModalStream(n=3000, noise=1e-3)
    m, r = 10, 6
    X = torch.from_numpy(g.frames(0, 30).T.copy()).cuda()
    with dmd.Stream(3000, m, r, dtype="f64", auto_solve=False) as s:
        for t in range(m + 1):
            s.push(X[t])
        with pytest.raises(dmd.DMDError):
            s.eigs()
        s.solve()
        check_window(s, g.frames(0, m + 1), m, r, phi_tol=1e-8)
        s.reset()
        assert s.info().count == 0
        for t in range(15, 15 + m + 1):
            s.push(X[t])
        s.solve()
        check_window(s, g.frames(15, m + 1), m, r, phi_tol=1e-8)


def test_rank_deficient_window_reports_w_rank():
    """Noiseless modal data has real rank 10; asking for r=14 uses r_eff=10."""
    dmd = _dmd()
    g = gen.ModalStream(n=2048, noise=0.0)
    m = 20
    X = torch.from_numpy(g.frames(0, m + 1).T.copy()).cuda()
    with dmd.Stream(2048, m, 14, dtype="f64") as s:
        for t in range(m + 1):
            s.push(X[t])
        lam, sig, rc = s.eigs()
    assert rc == dmd.W_RANK and lam.size == 10
    err, _ = metrics.eig_relerr(lam, g.true_eigs())
    assert err.max() < 1e-9


def test_warm_start_option_matches_oracle():
    """Jacobi started from the previous solve's eigenvectors (rows shifted by one
    window position) reaches the same decomposition as a cold start."""
    dmd = _dmd()
    v = gen.BlobVideo(height=90, width=160, blob_sigma=3.0)
    m, r = 32, 12
    T = m + 8
    frames = v.frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(90 * 160, m, r, warm_start=True) as s:
        for t in range(T):
            s.push(X[t])
            if t >= m:
                check_window(s, frames[:, t - m:t + 1], m, r, phi_tol=2e-4)
