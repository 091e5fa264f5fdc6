"""Split-BF16 projections (DMD_PREC_BF16X3): the modes of single pushes, of
every window of a block push and of grouped batch ticks against the FP64
oracle, next to the same streams in FP32.

The eigen-data do not depend on the projection precision (the per-frame and
block Gram accumulate in FP64 and the small solves run in FP64), so sigma and
lambda meet the FP64-Gram bounds of the dense tests.  A mode Phi_i = X' c_i
formed from products with relative error eps obeys
||dPhi_i|| <= eps || |X'| |c_i| || + ||X'|| ||dc_i||.  Splitting x = hi + lo + d
with hi = bf16(x), lo = bf16(x - hi) leaves |d| <= 2^-18 |x|, so the three
products hi*hi + hi*lo + lo*hi miss at most about 3 * 2^-18 |a||b|; FP32
accumulation of m <= 64 terms and the FP32 rounding of c add below 2^-18.  The
tests allow eps = 2^-14 (BF16x3) and 2^-17 (FP32), plus 1e-6 for the FP64
coefficients' own error, each times the cancellation factor
kappa_i = || |X'| |c_i| || / ||Phi_i||, computed from the oracle.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_dense import sigma_tol, check_lambda

pytestmark = pytest.mark.gpu

EPS = {"bf16x3": 2.0 ** -14, "fp32": 2.0 ** -17}


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def mode_bounds(W, ref, k, eps):
    """Per-mode relative error allowed for Phi_i = X' c_i (c = V Sigma^-1 W)."""
    Xp = np.abs(oracle.as_fp64(W[:, 1:]))
    C = (ref.V[:, :k] / ref.sigma[:k]) @ ref.W
    kappa = np.linalg.norm(Xp @ np.abs(C), axis=0) / np.linalg.norm(ref.Phi, axis=0)
    return (eps + 1e-6) * kappa


def check_modes(lam, sig, phi, W, m, r, eps, want_err=False):
    ref = oracle.exact_dmd(oracle.as_fp64(W[:, :m]), oracle.as_fp64(W[:, 1:]), r)
    k = lam.size
    assert k == ref.r_eff, (k, ref.r_eff)
    assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= sigma_tol(ref.sigma[:k]))
    err_l, perm = check_lambda(lam, ref)
    bound = mode_bounds(W, ref, k, eps)
    errs = np.array([metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]]) for i in range(k)])
    assert np.all(errs <= bound[perm[:k]]), (errs, bound[perm[:k]])
    return errs


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_single_push_modes_video(prec):
    dmd = _dmd()
    H, Wd, m, r = 100, 130, 37, 12
    frames = gen.BlobVideo(height=H, width=Wd, blob_sigma=4.0).frames(0, m + 3)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(H * Wd, m, r, precision=prec) as s:
        for t in range(m + 3):
            s.push(X[t])
            if t >= m:
                lam, sig, _ = s.eigs()
                check_modes(lam, sig, s.modes().cpu().numpy(), frames[:, t - m:t + 1], m, r, EPS[prec])
        # POD modes U = X V Sigma^-1 (unit columns): same product bound with X
        U = s.pod().cpu().numpy()
        F = oracle.as_fp64(frames[:, -(m + 1):])
        ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r, pod=True)
        k = ref.r_eff
        kap = np.linalg.norm(np.abs(F[:, :m]) @ np.abs(ref.V[:, :k] / ref.sigma[:k]), axis=0)
        for i in range(k):
            e = np.linalg.norm(U[:, i] - ref.U[:, i]) / np.linalg.norm(ref.U[:, i])
            assert e <= (EPS[prec] + 1e-6) * kap[i], (i, e, kap[i])


def test_bf16x3_modes_travelling_waves():
    """Data with condition ~10^3.5: the weak waves' modes cancel strongly, the
    bound grows with kappa_i and BF16x3 stays within it; the strong waves'
    modes are accurate to ~1e-4."""
    dmd = _dmd()
    n, m, r = 1 << 16, 48, 16
    w = gen.TravelingWaves(n=n, n_waves=8)
    F = w.frames(0, m + 1)
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(n, m, r, precision="bf16x3") as s:
        for t in range(m + 1):
            s.push(X[t])
        lam, sig, _ = s.eigs()
        errs = check_modes(lam, sig, s.modes().cpu().numpy(), F, m, r, EPS["bf16x3"])
    assert np.sort(errs)[:4].max() < 1e-4, errs


def test_bf16x3_block_modes_every_window():
    dmd = _dmd()
    H, Wd, m, r, kb = 90, 160, 24, 10, 5
    blocks = [3, 5, 5, 4, 1, 5, 2, 5]
    T = sum(blocks)
    frames = gen.BlobVideo(height=H, width=Wd, blob_sigma=3.0).frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(H * Wd, m, r, max_block=kb, precision="bf16x3") as s:
        t = 0
        for k in blocks:
            s.push_block(X[t:t + k])
            t += k
            if t < m + 1:
                continue
            wins, rc = s.block_eigs()
            phis = s.block_modes().cpu().numpy()
            for w, (stat, lam, sig) in enumerate(wins):
                te = t - k + w
                if te < m:
                    continue
                assert stat in (0, 1)
                check_modes(lam, sig, phis[w].T, frames[:, te - m:te + 1], m, r, EPS["bf16x3"])
            # the last window is the current one: the block kernel and the
            # single-window kernel give the same modes to the bound
            lam_c, sig_c, _ = s.eigs()
            check_modes(lam_c, sig_c, s.modes().cpu().numpy(), frames[:, t - 1 - m:t], m, r, EPS["bf16x3"])


MIX = [  # (n, m, r, kind, precision)
    (20000, 16, 8, "video", "bf16x3"),
    (33333, 32, 16, "flow", "fp32"),
    (70001, 64, 20, "video", "bf16x3"),
    (50000, 33, 10, "flow", "bf16x3"),
    (9000, 24, 12, "video", "fp32"),
]


def test_batch_mixed_precision_equals_alone():
    """A grouped tick holding FP32 and BF16x3 streams gives each stream the
    modes it gets alone, bit for bit."""
    dmd = _dmd()
    gens = [gen.MixStream(stream=300 + i, n=n, m=0, r=0, kind=kind) for i, (n, m, r, kind, p) in enumerate(MIX)]
    dev = []
    for g, (n, m, r, kind, p) in zip(gens, MIX):
        F = np.stack([g.frame(t) for t in range(m + 3)], axis=1)
        dev.append((F, torch.from_numpy(F.T.copy()).cuda()))
    alone = []
    for (n, m, r, kind, p), (F, X) in zip(MIX, dev):
        with dmd.Stream(n, m, r, precision=p) as s:
            for t in range(X.shape[0]):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            alone.append((lam, sig, s.modes().cpu().numpy()))
    streams = [dmd.Stream(n, m, r, precision=p) for (n, m, r, kind, p) in MIX]
    batch = dmd.Batch(max_streams=8)
    for s in streams:
        batch.attach(s)
    T = max(X.shape[0] for _, X in dev)
    outs = [torch.zeros((s.r, s.n), dtype=torch.complex64, device="cuda").T for s in streams]
    for t in range(T):
        act = [i for i, (_, X) in enumerate(dev) if t >= T - X.shape[0]]
        batch.tick([streams[i] for i in act], [dev[i][1][t - (T - dev[i][1].shape[0])] for i in act],
                   modes=[outs[i] for i in act])
    torch.cuda.synchronize()
    for i, s in enumerate(streams):
        lam, sig, _ = s.eigs()
        k = lam.size
        assert np.array_equal(lam, alone[i][0]) and np.array_equal(sig, alone[i][1]), i
        phi = outs[i].cpu().numpy()
        assert np.array_equal(phi[:, :k], alone[i][2][:, :k]), i
        n, m, r, kind, p = MIX[i]
        F = dev[i][0]
        W = F[:, -(m + 1):]
        ref = oracle.exact_dmd(oracle.as_fp64(W[:, :m]), oracle.as_fp64(W[:, 1:]), r)
        _, perm = metrics.eig_relerr(lam, ref.lam)
        bound = mode_bounds(W, ref, k, EPS[p])
        for j in range(k):
            assert metrics.phase_aligned_relerr(phi[:, j], ref.Phi[:, perm[j]]) <= bound[perm[j]], (i, j)
    batch.close()
    for s in streams:
        s.close()
