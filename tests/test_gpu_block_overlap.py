"""Block pushes on one stream and their projections on another.

The projection of block b reads only the ring columns of its windows and the
inputs packed after its solves, so it may run beside the Gram update and the
solves of block b + 1.  The same sequence of calls, once on a single stream and
once with pushes on stream A and projections on stream B (with single pushes
and reads in between), must give the same modes for every block, bit for bit
(same kernels, same inputs), and leave the outputs of unsolved windows
untouched.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_precision import EPS, mode_bounds

pytestmark = pytest.mark.gpu

SENTINEL = 7.0 + 7.0j


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def run_sequence(X, n, m, r, kb, plan, precision, two_streams):
    """plan: list of ("block", k) / ("single",) steps; returns the modes of
    every block step (or None before the window is full) and the final eigs."""
    dmd = _dmd()
    cur = torch.cuda.current_stream()
    A = torch.cuda.Stream() if two_streams else cur
    B = torch.cuda.Stream() if two_streams else cur
    A.wait_stream(cur)
    outs = []
    t = 0
    with dmd.Stream(n, m, r, max_block=kb, precision=precision) as s:
        for step in plan:
            if step[0] == "single":
                s.push(X[t], stream=A)
                t += 1
                lam, _, _ = s.eigs()               # a read between the pushes
                outs.append(("single", t, lam))
                continue
            k = step[1]
            s.push_block(X[t:t + k], stream=A)
            t += k
            if t < m + 1:
                outs.append(("block", t, k, None))
                continue
            o = torch.full((kb, r, n), SENTINEL, dtype=torch.complex64, device="cuda")
            B.wait_stream(cur)                      # the fill above is on the current stream
            s.block_modes(o, stream=B)
            outs.append(("block", t, k, o))
        torch.cuda.synchronize()
        final = s.eigs()
    return outs, final


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_overlapped_projection_equals_sequential(precision):
    H, W, m, r, kb = 90, 160, 24, 10, 5
    n = H * W
    plan = [("block", 3), ("block", 5), ("block", 5), ("block", 4), ("block", 5), ("block", 5),
            ("single",), ("block", 2), ("block", 5), ("block", 5), ("block", 1), ("block", 5),
            ("block", 5), ("block", 5)]
    T = sum(1 if p[0] == "single" else p[1] for p in plan)
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, T)
    X = torch.from_numpy(frames.T.copy()).cuda()
    seq, fin_seq = run_sequence(X, n, m, r, kb, plan, precision, two_streams=False)
    ovl, fin_ovl = run_sequence(X, n, m, r, kb, plan, precision, two_streams=True)
    assert np.array_equal(fin_seq[0], fin_ovl[0]) and np.array_equal(fin_seq[1], fin_ovl[1])
    checked = 0
    for a, b in zip(seq, ovl):
        assert a[:2] == b[:2]
        if a[0] == "single":
            assert np.array_equal(a[2], b[2])
            continue
        if a[3] is None:
            assert b[3] is None
            continue
        pa, pb = a[3].cpu().numpy(), b[3].cpu().numpy()
        assert np.array_equal(pa, pb), a[:3]
        # and the modes are right: every solved window against the oracle
        t, k = a[1], a[2]
        for w in range(kb):
            te = t - k + w
            if w >= k or te < m:
                assert np.all(pb[w] == SENTINEL)
                continue
            Wn = frames[:, te - m:te + 1]
            ref = oracle.exact_dmd(oracle.as_fp64(Wn[:, :m]), oracle.as_fp64(Wn[:, 1:]), r)
            kk = ref.r_eff
            bound = mode_bounds(Wn, ref, kk, EPS[precision])
            phi = pb[w][:kk].T
            for i in range(kk):
                # each GPU mode matches an oracle mode within that mode's bound
                e = [metrics.phase_aligned_relerr(phi[:, i], ref.Phi[:, j]) for j in range(kk)]
                j = int(np.argmin(e))
                assert e[j] <= bound[j], (t, w, i, e[j], bound[j])
            assert np.all(pb[w][kk:] == SENTINEL)
            checked += 1
    assert checked > 20


def test_block_modes_twice_on_two_streams():
    """Projecting the same block twice, on two different streams, gives the same modes."""
    dmd = _dmd()
    H, W, m, r, kb = 64, 100, 16, 8, 4
    n = H * W
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, m + 1 + 3 * kb)
    X = torch.from_numpy(frames.T.copy()).cuda()
    A, B = torch.cuda.Stream(), torch.cuda.Stream()
    with dmd.Stream(n, m, r, max_block=kb) as s:
        s.push_block(X[:kb])
        t = kb
        while t + kb <= X.shape[0]:
            s.push_block(X[t:t + kb])
            t += kb
        torch.cuda.synchronize()
        o1 = torch.zeros((kb, r, n), dtype=torch.complex64, device="cuda")
        o2 = torch.zeros((kb, r, n), dtype=torch.complex64, device="cuda")
        A.wait_stream(torch.cuda.current_stream())
        B.wait_stream(torch.cuda.current_stream())
        s.block_modes(o1, stream=A)
        s.block_modes(o2, stream=B)
        s.push(X[0], stream=A)                    # a single push after both: waits for both
        torch.cuda.synchronize()
        assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
