"""Parity of the one-frame Gram pass (Sec. 3.1, Algorithms 1-2) in every slab
form and at the full sizes of the benchmark workloads.

The pass reads each window column in slabs of 1, 2 or 4 16-byte loads per
thread and column (chosen by n; DMD_GRAM_ITER forces one), with column
groups of 2 or 4 and a scalar path for a partial last slab and for a
snapshot that is not 16-byte aligned.  These tests drive every form:
* each slab form, forced, at a ragged n (partial last slab), FP32 and FP64
  data, aligned and misaligned snapshots, single streams and batch ticks;
* single pushes of 1920 x 1080 blob video (n = 2,073,600, m = 64, r = 20,
  the large-slab form chosen by n), Gram and DMD of the last windows;
* streamed travelling waves at n = 2^20, m = 256, r = 32 with FP32 and FP64
  data, 500 frames: the Gram of every 50th window and of the last, and the
  DMD of the last window;
* pushes from host memory (pageable and pinned) against device pushes.

Tolerances are those of the dense tests (Gram 1e-12 sqrt(G_ii G_jj); sigma
1e-11 + 1e-13 (sigma_1/sigma_k)^2), with each eigenvalue held to its own
first-order sensitivity (32 u kappa_i, see test_gpu_batch.eig_bound) and each
mode to its product bound (see test_gpu_precision.mode_bounds).
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_batch import eig_bound
from test_gpu_dense import check_gram, check_window, sigma_tol
from test_gpu_precision import mode_bounds

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def pooled_frames(g, t0, count, dtype=np.float32):
    with ThreadPoolExecutor(max_workers=16) as ex:
        cols = list(ex.map(g.frame, range(t0, t0 + count)))
    return np.stack(cols, axis=1).astype(dtype, copy=False)


def misaligned_copy(x):
    """x in device memory at an address 4 (FP32) or 8 (FP64) bytes past a
    16-byte boundary: the pass takes its scalar path for the snapshot."""
    buf = torch.empty(x.numel() + 1, dtype=x.dtype, device="cuda")
    buf[1:].copy_(x)
    y = buf[1:]
    assert y.data_ptr() % 16 != 0
    return y, buf


def check_dmd(s, window, m, r, proj_eps, ref=None):
    """sigma, per-eigenvalue lambda and per-mode Phi of the latest solve."""
    if ref is None:
        F = oracle.as_fp64(window)
        ref = oracle.exact_dmd(F[:, :m], F[:, 1:], r)
    lam, sig, rc = s.eigs()
    assert rc in (0, 1)
    k = lam.size
    assert k == ref.r_eff, (k, ref.r_eff)
    err_s = metrics.sigma_relerr(sig, ref.sigma[:k])
    assert np.all(err_s <= sigma_tol(ref.sigma[:k])), err_s
    err_l, perm = metrics.eig_relerr(lam, ref.lam)
    bound = eig_bound(ref)[perm]
    assert np.all(err_l <= bound), (err_l, bound)
    phi = s.modes().cpu().numpy()
    pb = mode_bounds(window, ref, k, proj_eps)
    errs = np.array([metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, perm[i]]) for i in range(k)])
    assert np.all(errs <= pb[perm]), (errs, pb[perm])
    return err_s, err_l, errs


# ---------------------------------------------------------------- every slab form, ragged n

RAGGED_N = 13065   # 3 x 4096 + 777: a partial last slab for every slab size


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("iter_", [1, 2, 4])
def test_gram_slab_forms_ragged(monkeypatch, dtype, iter_):
    monkeypatch.setenv("DMD_GRAM_ITER", str(iter_))
    dmd = _dmd()
    n, m, r = RAGGED_N, 9, 5
    npdt = np.float32 if dtype == "f32" else np.float64
    v = gen.BlobVideo(height=105, width=125, n=n, blob_sigma=6.0)
    T = m + 5
    frames = v.frames(0, T).astype(npdt)
    X = torch.from_numpy(frames.T.copy()).cuda()
    keep = []
    with dmd.Stream(n, m, r, dtype=dtype) as s:
        for t in range(T):
            if t % 2:
                x, buf = misaligned_copy(X[t])
                keep.append(buf)
            else:
                x = X[t]
            s.push(x)
            check_gram(s, frames[:, max(0, t - m):t + 1])
            if t >= m + 3:
                check_window(s, frames[:, t - m:t + 1], m, r, phi_tol=2e-4 if dtype == "f32" else 1e-8)


@pytest.mark.parametrize("iter_", [1, 2, 4])
def test_batch_slab_forms_ragged(monkeypatch, iter_):
    """The grouped Gram pass of a batch tick in each slab form: every member
    equals the same stream alone bit for bit, and its Gram the oracle's."""
    monkeypatch.setenv("DMD_GRAM_ITER", str(iter_))
    dmd = _dmd()
    specs = [(RAGGED_N, 9, 5), (4097, 16, 6), (70001, 12, 6)]
    gens = [gen.MixStream(stream=300 + i, n=n, m=0, r=0, kind="video") for i, (n, m, r) in enumerate(specs)]
    T = max(m for _, m, _ in specs) + 3
    frames = [np.stack([g.frame(t) for t in range(T)], axis=1) for g in gens]
    dev = [torch.from_numpy(F.T.copy()).cuda() for F in frames]
    alone = []
    for (n, m, r), X in zip(specs, dev):
        with dmd.Stream(n, m, r) as s:
            for t in range(T):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            alone.append((s.gram(), lam, sig))
    streams = [dmd.Stream(n, m, r) for (n, m, r) in specs]
    with dmd.Batch(max_streams=4) as batch:
        for s in streams:
            batch.attach(s)
        for t in range(T):
            batch.tick(streams, [X[t] for X in dev])
        torch.cuda.synchronize()
        for i, s in enumerate(streams):
            n, m, r = specs[i]
            G = s.gram()
            lam, sig, _ = s.eigs()
            assert np.array_equal(G, alone[i][0]), i
            assert np.array_equal(lam, alone[i][1]) and np.array_equal(sig, alone[i][2]), i
            check_gram(s, frames[i][:, T - m - 1:])
        for s in streams:
            batch.detach(s)
    for s in streams:
        s.close()



def test_batch_at_serving_mix_extremes():
    """A batch tick at the ends of the serving mix's size range (n = 2,097,152
    and 65,536, with a ragged 1,048,579 between) in the slab forms the default
    launch shapes pick at those sizes: every member equals the same stream
    alone bit for bit, its Gram the oracle's, and the largest member's last
    window the oracle's exact DMD."""
    dmd = _dmd()
    specs = [(2_097_152, 16, 8), (65_536, 32, 16), (1_048_579, 16, 8)]
    gens = [gen.MixStream(stream=400 + i, n=n, m=0, r=0, kind="video") for i, (n, m, r) in enumerate(specs)]
    T = max(m for _, m, _ in specs) + 3
    frames = [np.stack([g.frame(t) for t in range(T)], axis=1) for g in gens]
    dev = [torch.from_numpy(F.T.copy()).cuda() for F in frames]
    alone = []
    for (n, m, r), X in zip(specs, dev):
        with dmd.Stream(n, m, r) as s:
            for t in range(T):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            alone.append((s.gram(), lam, sig))
    streams = [dmd.Stream(n, m, r) for (n, m, r) in specs]
    with dmd.Batch(max_streams=4) as batch:
        for s in streams:
            batch.attach(s)
        for t in range(T):
            batch.tick(streams, [X[t] for X in dev])
        torch.cuda.synchronize()
        for i, s in enumerate(streams):
            n, m, r = specs[i]
            lam, sig, _ = s.eigs()
            assert np.array_equal(s.gram(), alone[i][0]), i
            assert np.array_equal(lam, alone[i][1]) and np.array_equal(sig, alone[i][2]), i
            check_gram(s, frames[i][:, T - m - 1:])
        n, m, r = specs[0]
        check_window(streams[0], frames[0][:, T - m - 1:], m, r, phi_tol=2e-4)
        for s in streams:
            batch.detach(s)
    for s in streams:
        s.close()

# ---------------------------------------------------------------- 1920 x 1080 video

def test_full_hd_video_single_pushes():
    """n = 2,073,600 FP32, m = 64, r = 20: the Gram of the last four windows and
    the DMD (sigma, lambda, V, A~, W, Phi) of the last one."""
    dmd = _dmd()
    m, r = 64, 20
    v = gen.BlobVideo()
    n = v.n
    T = m + 4
    frames = pooled_frames(v, 0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r) as s:
        for t in range(T):
            s.push(X[t])
            if t >= m:
                check_gram(s, frames[:, t - m:t + 1])
        check_window(s, frames[:, T - m - 1:], m, r, phi_tol=2e-4)


# ---------------------------------------------------------------- 2^20 travelling waves, m = 256

WN, WM, WR, WT = 1 << 20, 256, 32, 500


@pytest.fixture(scope="module")
def waves():
    """The frames (FP32) and the oracle's results, shared by the FP32 and
    FP64 legs (FP64 data hold the same values, widened exactly)."""
    w = gen.TravelingWaves(n=WN, n_waves=8)
    return {"frames": pooled_frames(w, 0, WT), "gram": {}, "ref": None}


def check_gram_cached(s, cache, key, window):
    if key not in cache:
        cache[key] = oracle.gram(window)
    ref = cache[key]
    G = s.gram()
    assert G.shape == ref.shape
    d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert np.all(np.abs(G - ref) <= 1e-12 * d + 1e-300), np.max(np.abs(G - ref) / d)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_waves_streamed_full_size(waves, dtype):
    """500 streamed frames of n = 2^20 (FP32 data, or the same values as FP64
    data), m = 256, r = 32: the Gram of windows 0, 50, ..., 200 and of the
    last (243), and the DMD of the last window (r_eff = 16: the data have
    real rank 16).  FP32 projections accumulate 256 products in FP32:
    relative error up to m 2^-24 = 2^-16 of the cancellation factor."""
    dmd = _dmd()
    F = waves["frames"]
    torch_dt = torch.float32 if dtype == "f32" else torch.float64
    X = torch.from_numpy(F.T.copy()).to(device="cuda", dtype=torch_dt)
    last = WT - WM - 1
    checked = []
    with dmd.Stream(WN, WM, WR, dtype=dtype) as s:
        for t in range(WT):
            s.push(X[t])
            w = t - WM
            if w >= 0 and (w % 50 == 0 or w == last):
                check_gram_cached(s, waves["gram"], w, F[:, w:t + 1])
                checked.append(w)
        assert checked == [0, 50, 100, 150, 200, last]
        del X
        if waves["ref"] is None:
            Fw = oracle.as_fp64(F[:, last:])
            waves["ref"] = oracle.exact_dmd(Fw[:, :WM], Fw[:, 1:], WR)
        err_s, err_l, errs = check_dmd(s, F[:, last:], WM, WR, 2.0 ** -16 if dtype == "f32" else 1e-12,
                                       ref=waves["ref"])
    print(f"\n[waves {dtype}] sigma rel err max {err_s.max():.1e}, lambda rel err max {err_l.max():.1e}, "
          f"mode rel err max {errs.max():.1e}")


# ---------------------------------------------------------------- host-memory pushes

@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_host_memory_pushes_equal_device_pushes(dtype):
    """Snapshots in pageable or pinned host memory are staged on the device
    and give bit for bit the results of the same snapshots pushed from device
    memory (the staging buffer is counted in the stream's device bytes)."""
    dmd = _dmd()
    n, m, r = 2_073_600, 8, 4
    npdt = np.float32 if dtype == "f32" else np.float64
    v = gen.BlobVideo()
    T = m + 4
    frames = pooled_frames(v, 0, T).astype(npdt)
    host = torch.from_numpy(frames.T.copy())
    pinned = host.pin_memory()
    X = host.cuda()
    with dmd.Stream(n, m, r, dtype=dtype) as a, dmd.Stream(n, m, r, dtype=dtype) as b:
        before = b.info().device_bytes
        for t in range(T):
            a.push(X[t])
            b.push(host[t] if t % 2 == 0 else pinned[t])
        assert b.info().device_bytes == before + (n + 63) // 64 * 64 * frames.itemsize
        la, sa, _ = a.eigs()
        lb, sb, _ = b.eigs()
        assert np.array_equal(la, lb) and np.array_equal(sa, sb)
        assert np.array_equal(a.gram(), b.gram())
        assert torch.equal(a.modes(), b.modes())
        check_gram(b, frames[:, T - m - 1:])


def test_host_memory_sparse_pushes_equal_device_pushes():
    dmd = _dmd()
    fs = gen.FourierSparse(side=64, nnz=120, redraw=0.05)
    m, r = 12, 6
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=130) as a, \
            dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=130) as b:
        for t in range(m + 4):
            idx, val = fs.frame(t)
            a.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
            b.push_csr(torch.from_numpy(idx), torch.from_numpy(val))
        la, sa, _ = a.eigs()
        lb, sb, _ = b.eigs()
        assert np.array_equal(la, lb) and np.array_equal(sa, sb)
        assert np.array_equal(a.gram(), b.gram())
