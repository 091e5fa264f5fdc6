"""Multi-column updates (Sec. 5: more than one new column per update).

A block push of k snapshots must leave the stream as k single pushes would,
and every window the block passes through is solved.  Each is compared with
the FP64 oracle on the same frames.

Tolerances: the block's inner products are exact products summed in FP64 in
another order than the one-column update, so the Gram bound of the dense path
applies (|dG_ij| <= 1e-12 sqrt(G_ii G_jj)); sigma, lambda and Phi as in the
dense tests (sigma_k: 1e-11 + 1e-13 (sigma_1/sigma_k)^2, lambda 1e-13 + 32 u kappa_i, Phi 1e-8
with FP64 projections, 2e-4 with FP32 projections).
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_dense import check_gram, check_window, sigma_tol, check_lambda

pytestmark = pytest.mark.gpu

BLOCKS = [3, 5, 5, 4, 1, 5, 2, 5]


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def check_eigs(stat, lam, sig, W, m, r):
    ref = oracle.exact_dmd(oracle.as_fp64(W[:, :m]), oracle.as_fp64(W[:, 1:]), r)
    assert stat in (0, 1), stat
    k = lam.size
    assert k == ref.r_eff, (k, ref.r_eff)
    err_s = metrics.sigma_relerr(sig, ref.sigma[:k])
    assert np.all(err_s <= sigma_tol(ref.sigma[:k])), err_s
    err_l, perm = check_lambda(lam, ref)
    return ref, perm


def check_phi(phi, ref, perm, k, tol):
    for i in range(k):
        e = metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]])
        assert e < tol, (i, e)


def run_blocks(s, X, frames, blocks, m, r, phi_tol, every_window=True):
    """Push X (T, n) in blocks; check the Gram after each block, every solved
    window of each block and the current window's matrices and modes."""
    dmd = _dmd()
    t = 0
    for k in blocks:
        s.push_block(X[t:t + k])
        t += k
        check_gram(s, frames[:, max(0, t - 1 - m):t])
        if t < m + 1:
            with pytest.raises(dmd.DMDError) as ei:
                s.block_eigs()
            assert ei.value.code == dmd.E_NOT_READY
            continue
        wins, rc = s.block_eigs()
        assert len(wins) == k and rc in (0, 1)
        sentinel = 7.0 + 7.0j
        phis = s.block_modes(torch.full((s.max_block, r, s.n), sentinel, dtype=s.mode_dtype, device="cuda"))
        phis = phis.cpu().numpy()
        for w, (stat, lam, sig) in enumerate(wins):
            te = t - k + w  # newest frame of window w
            if te < m:
                assert stat == dmd.E_NOT_READY
                assert np.all(phis[w] == sentinel)       # unsolved windows are left untouched
            elif every_window or w == 0:
                ref, perm = check_eigs(stat, lam, sig, frames[:, te - m:te + 1], m, r)
                check_phi(phis[w].T, ref, perm, lam.size, phi_tol)
                assert np.all(phis[w][lam.size:] == sentinel)
        # the last window is the current one: identical to eigs() and modes()
        lam_c, sig_c, _ = s.eigs()
        assert np.array_equal(lam_c, wins[-1][1]) and np.array_equal(sig_c, wins[-1][2])
        phi_c = s.modes().cpu().numpy()
        kc = lam_c.size
        np.testing.assert_allclose(phis[k - 1].T[:, :kc], phi_c[:, :kc], rtol=0,
                                   atol=1e-6 * np.abs(phi_c[:, :kc]).max())
        check_window(s, frames[:, t - 1 - m:t], m, r, phi_tol=phi_tol)


@pytest.mark.parametrize("n", [4133, 1000])
def test_block_fp64_every_window(n):
    dmd = _dmd()
    m, r = 16, 6
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, sum(BLOCKS))
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype="f64", max_block=5) as s:
        run_blocks(s, X, frames, BLOCKS, m, r, phi_tol=1e-8)


@pytest.mark.parametrize("aligned", [True, False])
def test_block_fp32_video_every_window(aligned):
    """Odd m, ragged n, k up to 16; unaligned columns (odd leading dimension) too."""
    dmd = _dmd()
    H, W, m, r = 100, 130, 37, 12
    n = H * W
    blocks = [16, 16, 7, 16, 1, 11]
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, sum(blocks))
    if aligned:
        X = torch.from_numpy(frames.T.copy()).cuda()
    else:
        buf = torch.zeros((frames.shape[1], n + 1), dtype=torch.float32, device="cuda")
        buf[:, :n] = torch.from_numpy(frames.T.copy()).cuda()
        X = buf[:, :n]
        assert X.stride(0) == n + 1
    with dmd.Stream(n, m, r, max_block=16) as s:
        run_blocks(s, X, frames, blocks, m, r, phi_tol=2e-4)


def test_block_matches_single_pushes():
    """Blocks and single pushes of the same frames: same windows, same results
    up to the summation order of the inner products."""
    dmd = _dmd()
    n, m, r, kb = 20000, 64, 20, 16
    frames = gen.BlobVideo(height=100, width=200, blob_sigma=5.0).frames(0, 8 * kb + 1)
    X = torch.from_numpy(frames.T.copy()).cuda()
    T = X.shape[0]
    with dmd.Stream(n, m, r) as a, dmd.Stream(n, m, r, max_block=kb) as b:
        singles = {}
        for t in range(T):
            a.push(X[t])
            if t >= m:
                singles[t] = a.eigs()
        t = 0
        while t < T:
            k = min(kb, T - t)
            b.push_block(X[t:t + k])
            t += k
            if t >= m + 1:
                wins, _ = b.block_eigs()
                for w, (stat, lam, sig) in enumerate(wins):
                    te = t - k + w
                    if te < m:
                        continue
                    lam_a, sig_a, _ = singles[te]
                    assert lam.size == lam_a.size
                    assert np.all(np.abs(sig - sig_a) <= sigma_tol(sig_a) * sig_a)
                    err, _ = metrics.eig_relerr(lam, lam_a)
                    assert err.max() < 1e-8
        Ga, Gb = a.gram(), b.gram()
        d = np.sqrt(np.outer(np.diag(Ga), np.diag(Ga)))
        assert np.all(np.abs(Ga - Gb) <= 1e-13 * d)
        # a single push after blocks continues the same window
        x = torch.from_numpy(gen.BlobVideo(height=100, width=200, blob_sigma=5.0).frame(T)).cuda()
        a.push(x)
        b.push(x)
        with pytest.raises(dmd.DMDError) as ei:
            b.block_eigs()
        assert ei.value.code == dmd.E_NOT_READY
        la, sa, _ = a.eigs()
        lb, sb, _ = b.eigs()
        assert metrics.eig_relerr(lb, la)[0].max() < 1e-8


def test_block_with_nonfinite_rejected_whole():
    dmd = _dmd()
    g = gen.ModalStream(n=2048, noise=1e-3)
    m, r = 8, 4
    frames = g.frames(0, 16)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(2048, m, r, dtype="f64", max_block=4) as s:
        for t in range(10):
            s.push(X[t])
        G0 = s.gram()
        lam0, sig0, _ = s.eigs()
        bad = X[10:13].clone()
        bad[1, 77] = float("inf")
        s.push_block(bad)
        with pytest.raises(dmd.DMDError) as ei:
            s.sync()
        assert ei.value.code == dmd.E_NONFINITE
        assert np.array_equal(s.gram(), G0)
        wins, _ = s.block_eigs()
        assert [w[0] for w in wins] == [dmd.E_NONFINITE] * 3
        out = s.block_modes(torch.full((4, r, 2048), 3.0, dtype=s.mode_dtype, device="cuda"))
        assert torch.all(out == 3.0).item()
        lam1, sig1, _ = s.eigs()
        assert np.array_equal(lam0, lam1) and np.array_equal(sig0, sig1)
        s.push_block(X[10:13])           # the same frames without the bad value
        wins, _ = s.block_eigs()
        for w, (stat, lam, sig) in enumerate(wins):
            te = 10 + w
            check_eigs(stat, lam, sig, frames[:, te - m:te + 1], m, r)
        check_window(s, frames[:, 13 - 1 - m:13], m, r, phi_tol=1e-8)


def test_block_argument_errors():
    dmd = _dmd()
    with dmd.Stream(1000, 8, 4, max_block=3) as s:
        X = torch.zeros((4, 1000), device="cuda")
        with pytest.raises(dmd.DMDError) as ei:
            s.push_block(X)
        assert ei.value.code == dmd.E_INVAL
        with pytest.raises(dmd.DMDError) as ei:
            s.block_eigs()
        assert ei.value.code == dmd.E_NOT_READY
        with pytest.raises(dmd.DMDError) as ei:
            s.block_modes()
        assert ei.value.code == dmd.E_NOT_READY
    with dmd.Stream(1000, 8, 4, dtype="c64_csr", max_nnz=16) as s:
        Xc = torch.zeros((1, 1000), dtype=torch.complex64, device="cuda")
        with pytest.raises(dmd.DMDError) as ei:
            s.push_block(Xc)
        assert ei.value.code == dmd.E_UNSUPPORTED


def test_block_full_hd_video():
    """1920 x 1080 FP32 frames, m = 64, r = 20, blocks of 16: the Gram of the
    window and the first, a middle and the last window of the last block."""
    dmd = _dmd()
    H, W, m, r, kb = 1080, 1920, 64, 20, 16
    n = H * W
    v = gen.BlobVideo(height=H, width=W)
    T = 5 * kb
    frames = v.frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=kb) as s:
        for t in range(0, T, kb):
            s.push_block(X[t:t + kb])
        wins, _ = s.block_eigs()
        check_gram(s, frames[:, T - 1 - m:T])
        phis = s.block_modes()
        for w in (0, kb // 2, kb - 1):
            te = T - kb + w
            stat, lam, sig = wins[w]
            ref, perm = check_eigs(stat, lam, sig, frames[:, te - m:te + 1], m, r)
            check_phi(phis[w].cpu().numpy().T, ref, perm, lam.size, 2e-4)


@pytest.mark.parametrize("m,r,kb", [(160, 24, 32), (200, 32, 48), (64, 20, 64), (64, 32, 64)])
def test_block_modes_large_windows(m, r, kb):
    """Windows beyond the default shapes (m > 64, k up to the largest block
    of 64 frames): the first, a middle and the last window's modes from the
    one-pass block projection must match the oracle."""
    dmd = _dmd()
    H, W = 100, 130
    n = H * W
    T = m + 1 + kb
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=kb) as s:
        t = 0
        while t < m + 1:
            k = min(kb, m + 1 - t)
            s.push_block(X[t:t + k])
            t += k
        s.push_block(X[t:t + kb])
        t += kb
        wins, _ = s.block_eigs()
        phis = s.block_modes().cpu().numpy()
        for w in (0, kb // 2, kb - 1):
            te = t - kb + w
            stat, lam, sig = wins[w]
            ref, perm = check_eigs(stat, lam, sig, frames[:, te - m:te + 1], m, r)
            check_phi(phis[w].T, ref, perm, lam.size, 2e-4)


@pytest.fixture
def projection_form(request, tmp_path):
    """Streams created in the test use block projection form `param` (0: the
    built-in rule, else named by a tuning-table entry for the test's shape)."""
    dmd = _dmd()
    dmd.tune_clear()

    def use(n, m, r, kb):
        form = request.param
        if form:
            f = tmp_path / "form.txt"
            f.write_text(f"0 0 {round(8 * np.log2(n))} {m} {r} {kb} 1 {form} 0 0\n")
            dmd.tune_load(str(f))
        return form
    yield use
    dmd.tune_clear()


@pytest.mark.parametrize("projection_form", [0, 2, 3], indirect=True)
@pytest.mark.parametrize("H,W,m,r", [(97, 134, 32, 12), (100, 200, 64, 12), (50, 100, 31, 4)])
def test_block_fp32_window_pairs(H, W, m, r, projection_form):
    """FP32 ranks r = 4, 12 (2r = 8 mod 16): two windows per product (form 2),
    or one banded product in which a 32-column tile spans up to five windows
    (form 3, and the rule).  Odd blocks end with a window of its own, and the
    block in which the window fills pairs unsolved windows with solved ones:
    every window against the oracle, unsolved windows and columns past r_eff
    left untouched."""
    dmd = _dmd()
    n = H * W
    form = projection_form(n, m, r, 16)
    blocks = [16, 16, 7, 16, 1, 11, 16, 5]
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, sum(blocks))
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=16) as s:
        assert s.info().proj_form == form
        run_blocks(s, X, frames, blocks, m, r, phi_tol=2e-4)


@pytest.mark.parametrize("projection_form", [0, 2], indirect=True)
def test_block_fp32_pairs_rank_deficient(projection_form):
    """Noiseless modal data has rank 10; with r = 12 every window uses
    r_eff = 10 (both windows of a pair, or every window of a banded tile):
    modes 0..9 against the oracle of the same rank, modes 10, 11 left
    untouched."""
    dmd = _dmd()
    n, m, r, kb = 6000, 32, 12, 7
    projection_form(n, m, r, kb)
    g = gen.ModalStream(n=n, noise=0.0)
    T = m + 1 + 3 * kb
    frames = g.frames(0, T).astype(np.float32)
    X = torch.from_numpy(frames.T.copy()).cuda()
    sentinel = 7.0 + 7.0j
    with dmd.Stream(n, m, r, max_block=kb) as s:
        t = 0
        while t < m + 1:
            k = min(kb, m + 1 - t)
            s.push_block(X[t:t + k])
            t += k
        checked = 0
        while t + kb <= T:
            s.push_block(X[t:t + kb])
            t += kb
            wins, rc = s.block_eigs()
            assert rc == dmd.W_RANK
            phis = s.block_modes(torch.full((kb, r, n), sentinel, dtype=torch.complex64, device="cuda"))
            phis = phis.cpu().numpy()
            for w, (stat, lam, sig) in enumerate(wins):
                te = t - kb + w
                assert stat == dmd.W_RANK and lam.size == 10, (w, stat, lam.size)
                Wf = oracle.as_fp64(frames[:, te - m:te + 1])
                ref = oracle.exact_dmd(Wf[:, :m], Wf[:, 1:], r, r_eff=10)
                err, perm = metrics.eig_relerr(lam, ref.lam)
                assert err.max() < 1e-6, (w, err.max())
                check_phi(phis[w].T, ref, perm, 10, 2e-4)
                assert np.all(phis[w][10:] == sentinel)
                checked += 1
        assert checked == 3 * kb


@pytest.mark.parametrize("H,W,m,r,kb", [(61, 83, 16, 8, 12), (90, 70, 48, 16, 16), (40, 50, 16, 4, 9)])
def test_block_fp32_banded_16x16_instances(H, W, m, r, kb):
    """The FP32 block projection's 16 x 16 x 4 banded kernel at the step
    counts the full-HD test does not take (4-column steps per tile: 5 at
    m = 16, 13 at m = 48; r = 4 puts up to five windows in a 32-column tile):
    every window of every block against the oracle, ragged row count."""
    dmd = _dmd()
    n = H * W
    blocks = [kb, kb, 5, kb, 1, kb]
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, sum(blocks))
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=kb) as s:
        run_blocks(s, X, frames, blocks, m, r, phi_tol=2e-4)
