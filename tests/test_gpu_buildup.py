"""Build-up start (Sec. 5: results while the window fills).

With the option on, after c >= 3 pushes into a stream of window m the GPU
solves the partial window of c snapshots as exact DMD with m' = c - 1 columns
(X = the first c - 1 snapshots, X' = the last c - 1), truncated to
min(r, m'); the oracle is the same exact DMD on those columns.  Once the
window is full everything is as without the option.  sigma past m' and the
rows of V past m' read zero.

Tolerances as in the dense tests (sigma_k 1e-11 + 1e-13 (sigma_1/sigma_k)^2,
lambda 1e-13 + 32 u kappa_i (as the dense tests), V 1e-7, Phi 1e-8 FP64 / 2e-4 FP32 projections; background 1e-9
FP64 / 2e-4 FP32 of max |x|).
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import background as bgo
from oracle import metrics
from test_gpu_dense import sigma_tol, check_lambda

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def check_partial(s, frames_window, m, r, phi_tol, bg_tol=None):
    """The GPU's latest solve vs exact DMD of the given (n, c) window."""
    c = frames_window.shape[1]
    mp = c - 1
    F = oracle.as_fp64(frames_window)
    ref = oracle.exact_dmd(F[:, :mp], F[:, 1:], r)
    lam, sig, rc = s.eigs()
    assert rc in (0, 1)
    k = lam.size
    assert k == ref.r_eff, (c, k, ref.r_eff)
    assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= sigma_tol(ref.sigma[:k]))
    err_l, perm = check_lambda(lam, ref)
    sg, V, _ = s.svd()
    assert np.all(sg[mp:] == 0.0)                       # sigma past m' reads zero
    assert np.all(metrics.sigma_relerr(sg[:mp], ref.sigma[:mp]) <= sigma_tol(ref.sigma[:mp]))
    assert np.all(V[mp:, :k] == 0.0)                    # so do the rows of V past m'
    assert np.max(np.abs(V[:mp, :k] - ref.V)) < 1e-7 * max(1.0, (ref.sigma[0] / ref.sigma[k - 1]) ** 2 * 1e-6)
    phi = s.modes().cpu().numpy()
    for i in range(k):
        assert metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]]) < phi_tol, (c, i)
    if bg_tol is not None:
        b, idx, _ = s.amplitudes()
        b_ref = bgo.amplitudes(ref)
        assert np.max(np.abs(b - b_ref[perm])) < 1e-7 * np.max(np.abs(b_ref))
        assert perm[idx] == bgo.background_index(ref.lam)
        s_ref, bg_ref, _ = bgo.background_split(F, ref, b_ref)
        fg, bg = s.background()
        scale = np.max(np.abs(F))
        assert np.max(np.abs(fg.cpu().numpy() - s_ref)) < bg_tol * scale
        assert np.max(np.abs(bg.cpu().numpy() - bg_ref)) < bg_tol * scale
    return ref


@pytest.mark.parametrize("solver", ["tridiag", "jacobi"])
def test_buildup_fp64_every_push(solver):
    dmd = _dmd()
    n, m, r = 4133, 16, 6
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, m + 4)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype="f64", buildup=True, eig_solver=solver) as s:
        for t in range(m + 4):
            s.push(X[t])
            c = min(t + 1, m + 1)
            if c < 3:
                with pytest.raises(dmd.DMDError) as ei:
                    s.eigs()
                assert ei.value.code == dmd.E_NOT_READY
                continue
            check_partial(s, frames[:, t + 1 - c:t + 1], m, r, 1e-8, bg_tol=1e-9)


def test_buildup_fp32_video_and_off_by_default():
    dmd = _dmd()
    H, W, m, r = 72, 96, 33, 12
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, m + 3)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(H * W, m, r, buildup=True) as s, dmd.Stream(H * W, m, r) as plain:
        for t in range(m + 3):
            s.push(X[t])
            plain.push(X[t])
            c = min(t + 1, m + 1)
            if c >= 3 and (c < 8 or c % 7 == 0 or c == m + 1):
                check_partial(s, frames[:, t + 1 - c:t + 1], m, r, 2e-4, bg_tol=2e-4)
            if c < m + 1:
                with pytest.raises(dmd.DMDError) as ei:
                    plain.eigs()
                assert ei.value.code == dmd.E_NOT_READY
            else:
                # full windows: identical with and without the option
                l1, s1, _ = s.eigs()
                l2, s2, _ = plain.eigs()
                assert np.array_equal(l1, l2) and np.array_equal(s1, s2)
                assert torch.equal(s.modes(), plain.modes())


def test_buildup_in_a_batch_equals_alone():
    dmd = _dmd()
    specs = [(20000, 16, 8), (9000, 24, 12), (33333, 12, 6)]
    gens = [gen.MixStream(stream=400 + i, n=n, m=0, r=0, kind="video") for i, (n, m, r) in enumerate(specs)]
    T = 10
    dev = [torch.from_numpy(np.stack([g.frame(t) for t in range(T)], axis=0)).cuda() for g in gens]
    alone = []
    for (n, m, r), X in zip(specs, dev):
        with dmd.Stream(n, m, r, buildup=True) as s:
            res = []
            for t in range(T):
                s.push(X[t])
                if t >= 2:
                    lam, sig, _ = s.eigs()
                    res.append((lam, sig, s.modes().cpu().numpy()))
            alone.append(res)
    streams = [dmd.Stream(n, m, r, buildup=True) for (n, m, r) in specs]
    batch = dmd.Batch(max_streams=4)
    for s in streams:
        batch.attach(s)
    outs = [torch.zeros((s.r, s.n), dtype=torch.complex64, device="cuda").T for s in streams]
    for t in range(T):
        batch.tick(streams, [X[t] for X in dev], modes=outs)
        torch.cuda.synchronize()
        if t >= 2:
            for i, s in enumerate(streams):
                lam, sig, _ = s.eigs()
                a = alone[i][t - 2]
                assert np.array_equal(lam, a[0]) and np.array_equal(sig, a[1]), (i, t)
                k = lam.size
                assert np.array_equal(outs[i].cpu().numpy()[:, :k], a[2][:, :k]), (i, t)
    batch.close()
    for s in streams:
        s.close()
