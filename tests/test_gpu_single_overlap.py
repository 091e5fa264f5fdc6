"""Modes of single pushes beside the next push (dense streams).

Every solve leaves a copy of its state and mode coefficients; dmd_stream_modes
reads that copy and the solve's window only, so on a second stream it runs
while the next push (Gram update and solves) runs on the first.  The modes of
every step must equal those of the same calls on one stream, bit for bit
(same kernels on the same values), and match the oracle.
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


def run(X, n, m, r, dtype, two_streams, plan, max_block=1):
    """plan: list of "p" (push + modes), "b<k>" (block push of k), "n" (push
    without modes), "s" (a host read of the eigenvalues)."""
    dmd = _dmd()
    cur = torch.cuda.current_stream()
    A = torch.cuda.Stream() if two_streams else cur
    B = torch.cuda.Stream() if two_streams else cur
    A.wait_stream(cur)
    outs = []
    t = 0
    cdt = torch.complex128 if dtype == "f64" else torch.complex64
    with dmd.Stream(n, m, r, dtype=dtype, max_block=max_block) as s:
        for step in plan:
            if step[0] == "b":
                k = int(step[1:])
                s.push_block(X[t:t + k], stream=A)
                t += k
                continue
            s.push(X[t], stream=A)
            t += 1
            if step == "s":
                outs.append(("eigs", t, s.eigs()[0]))
            if step != "p" or t < m + 1:
                continue
            o = torch.zeros((r, n), dtype=cdt, device="cuda").T
            B.wait_stream(cur)                      # the zero fill is on the current stream
            s.modes(o, stream=B)
            outs.append(("modes", t, o))
        torch.cuda.synchronize()
        lam, sig, _ = s.eigs()
        assert s.sync() in (0, 1)
    return outs, (lam, sig), t


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_single_modes_beside_next_push(dtype):
    H, W, m, r = 60, 90, 20, 8
    n = H * W
    plan = ["p"] * (m + 1) + ["p"] * 12 + ["n", "p", "s", "p", "p", "n", "n", "p"] + ["p"] * 6
    T = len(plan)
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, T)
    if dtype == "f64":
        frames = frames.astype(np.float64)
    X = torch.from_numpy(frames.T.copy()).cuda()
    seq, fin_seq, _ = run(X, n, m, r, dtype, False, plan)
    ovl, fin_ovl, _ = run(X, n, m, r, dtype, True, plan)
    assert np.array_equal(fin_seq[0], fin_ovl[0]) and np.array_equal(fin_seq[1], fin_ovl[1])
    assert len(seq) == len(ovl)
    checked = 0
    tol = 2e-4 if dtype == "f32" else 1e-8
    for a, b in zip(seq, ovl):
        assert a[:2] == b[:2]
        if a[0] == "eigs":
            assert np.array_equal(a[2], b[2])
            continue
        pa, pb = a[2].cpu().numpy(), b[2].cpu().numpy()
        assert np.array_equal(pa, pb), a[1]
        t = a[1]
        Wn = frames[:, t - m - 1:t]
        ref = oracle.exact_dmd(oracle.as_fp64(Wn[:, :m]), oracle.as_fp64(Wn[:, 1:]), r)
        for i in range(ref.r_eff):
            e = min(metrics.phase_aligned_relerr(pb[:, i], ref.Phi[:, j]) for j in range(ref.r_eff))
            assert e < tol, (t, i, e)
        checked += 1
    assert checked > 20


def test_single_modes_beside_pushes_with_blocks():
    """A stream that also takes block pushes: single-push modes, block pushes
    and more single pushes interleaved on two streams equal one stream."""
    H, W, m, r = 48, 80, 16, 6
    n = H * W
    plan = ["b5", "b5", "b5", "b3", "p", "p", "b4", "p", "p", "p", "b2", "p", "s", "p"]
    T = sum(int(p[1:]) if p[0] == "b" else 1 for p in plan)
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    seq, fin_seq, _ = run(X, n, m, r, "f32", False, plan, max_block=5)
    ovl, fin_ovl, _ = run(X, n, m, r, "f32", True, plan, max_block=5)
    assert np.array_equal(fin_seq[0], fin_ovl[0])
    for a, b in zip(seq, ovl):
        assert a[:2] == b[:2]
        if a[0] == "eigs":
            assert np.array_equal(a[2], b[2])
        else:
            assert np.array_equal(a[2].cpu().numpy(), b[2].cpu().numpy()), a[1]


def test_single_modes_twice_on_two_streams():
    """The same solve's modes on two streams, then a push: both equal."""
    dmd = _dmd()
    H, W, m, r = 40, 50, 12, 5
    n = H * W
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, m + 4)
    X = torch.from_numpy(frames.T.copy()).cuda()
    A, B = torch.cuda.Stream(), torch.cuda.Stream()
    with dmd.Stream(n, m, r) as s:
        for t in range(m + 3):
            s.push(X[t])
        torch.cuda.synchronize()
        o1 = torch.zeros((r, n), dtype=torch.complex64, device="cuda").T
        o2 = torch.zeros((r, n), dtype=torch.complex64, device="cuda").T
        A.wait_stream(torch.cuda.current_stream())
        B.wait_stream(torch.cuda.current_stream())
        s.modes(o1, stream=A)
        s.modes(o2, stream=B)
        s.push(X[m + 3])                           # the next push may run beside both
        s.push(X[0])                               # the one after waits for both
        torch.cuda.synchronize()
        assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
