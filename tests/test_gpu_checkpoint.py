"""Checkpoint / resume (Sec. 5: persisting a stream).

A stream restored from a checkpoint holds the same window and Gram as the
saved one (in another ring position), so every later result is the same,
bit for bit: the same kernels run on the same values in the same order.  The
final windows are also checked against the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics
from test_gpu_dense import check_window

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def same_results(a, b):
    la, sa, _ = a.eigs()
    lb, sb, _ = b.eigs()
    assert np.array_equal(la, lb) and np.array_equal(sa, sb)
    assert np.array_equal(a.gram(), b.gram())
    assert torch.equal(a.modes(), b.modes())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_resume_dense_bitwise(dtype):
    dmd = _dmd()
    H, W, m, r = 64, 90, 20, 8
    n = H * W
    T0, T1 = m + 6, 7
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, T0 + T1)
    if dtype == "f64":
        frames = frames.astype(np.float64)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype=dtype) as a, dmd.Stream(n, m, r, dtype=dtype) as b:
        for t in range(T0):
            a.push(X[t])
        blob = a.save()
        b.restore(blob)
        same_results(a, b)
        for t in range(T0, T0 + T1):
            a.push(X[t])
            b.push(X[t])
            same_results(a, b)
        check_window(b, frames[:, -(m + 1):], m, r, phi_tol=2e-4 if dtype == "f32" else 1e-8)


def test_resume_partial_window_with_buildup():
    dmd = _dmd()
    n, m, r = 3000, 12, 5
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, m + 4).astype(np.float32)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, buildup=True) as a, dmd.Stream(n, m, r, buildup=True) as b:
        for t in range(5):
            a.push(X[t])
        b.restore(a.save())
        same_results(a, b)
        for t in range(5, m + 4):
            a.push(X[t])
            b.push(X[t])
            same_results(a, b)
    # a stream without the build-up option restores the partial window but
    # has nothing to report until it is full
    with dmd.Stream(n, m, r, buildup=True) as a, dmd.Stream(n, m, r) as c:
        for t in range(5):
            a.push(X[t])
        c.restore(a.save())
        with pytest.raises(dmd.DMDError) as ei:
            c.eigs()
        assert ei.value.code == dmd.E_NOT_READY
        assert np.array_equal(a.gram(), c.gram())


def test_resume_sparse_bitwise():
    dmd = _dmd()
    fs = gen.FourierSparse(side=64, nnz=120, redraw=0.05)
    m, r = 24, 8
    T0, T1 = m + 4, 5

    def push(s, t):
        idx, val = fs.frame(t)
        s.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())

    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=130) as a, \
            dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=130) as b:
        for t in range(T0):
            push(a, t)
        b.restore(a.save())
        same_results(a, b)
        for t in range(T0, T0 + T1):
            push(a, t)
            push(b, t)
            same_results(a, b)
        dense = np.stack([oracle.densify(*fs.frame(t), fs.n) for t in range(T0 + T1 - m - 1, T0 + T1)], axis=1)
        ref = oracle.exact_dmd(dense[:, :m], dense[:, 1:], r)
        lam, _, _ = b.eigs()
        assert metrics.eig_relerr(lam, ref.lam)[0].max() < 1e-8


def test_resume_block_stream_bitwise():
    dmd = _dmd()
    H, W, m, r, kb = 48, 80, 16, 6, 4
    n = H * W
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=3.0).frames(0, m + 1 + 6 * kb)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=kb) as a, dmd.Stream(n, m, r, max_block=kb) as b:
        t = 0
        while t < m + 1 + 2 * kb:
            k = min(kb, m + 1 + 2 * kb - t)
            a.push_block(X[t:t + k])
            t += k
        b.restore(a.save())
        same_results(a, b)
        while t + kb <= X.shape[0]:
            a.push_block(X[t:t + kb])
            b.push_block(X[t:t + kb])
            t += kb
            wa, _ = a.block_eigs()
            wb, _ = b.block_eigs()
            for (sa, la, ga), (sb, lb, gb) in zip(wa, wb):
                assert sa == sb and np.array_equal(la, lb) and np.array_equal(ga, gb)
            assert torch.equal(a.block_modes(), b.block_modes())


def test_restore_rejects_bad_checkpoints():
    dmd = _dmd()
    n, m, r = 2000, 8, 4
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, m + 2).astype(np.float32)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r) as a:
        for t in range(m + 2):
            a.push(X[t])
        blob = a.save()
        for bad, msg in [(blob[:40], "truncated"), (b"x" * len(blob), "not a checkpoint"),
                         (blob[:-8], "truncated")]:
            with dmd.Stream(n, m, r) as b:
                with pytest.raises(dmd.DMDError) as ei:
                    b.restore(bad)
                assert ei.value.code == dmd.E_INVAL
        for shape in [(n + 1, m, r), (n, m + 1, r), (n, m, r - 1)]:
            with dmd.Stream(*shape) as b:
                with pytest.raises(dmd.DMDError) as ei:
                    b.restore(blob)
                assert ei.value.code == dmd.E_INVAL
        with dmd.Stream(n, m, r, dtype="f64") as b:
            with pytest.raises(dmd.DMDError) as ei:
                b.restore(blob)
            assert ei.value.code == dmd.E_INVAL


def test_restore_rejects_bad_sparse_indices():
    """A sparse checkpoint whose indices break the push rule (strictly
    increasing in [0, n)) is refused on the host before any device copy, and
    the stream keeps its window."""
    import struct
    dmd = _dmd()
    fs = gen.FourierSparse(side=32, nnz=40, redraw=0.05)
    m, r = 6, 3
    with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=48) as a:
        for t in range(m + 2):
            idx, val = fs.frame(t)
            a.push_csr(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())
        blob = bytearray(a.save())
        G0 = a.gram()
        # header: magic[8], version, dtype, n (int64), m, r, count, max_nnz,
        # four counters, gram_bytes, data_bytes (int64)
        hdr = struct.calcsize("<8sii q 4i 4i qq")
        count = struct.unpack_from("<i", blob, 8 + 4 + 4 + 8 + 8)[0]
        gram_bytes = struct.unpack_from("<q", blob, hdr - 16)[0]
        data = hdr + gram_bytes
        nnz = struct.unpack_from(f"<{count}i", blob, data)
        second = data + 4 * count + 12 * nnz[0]   # indices of window snapshot 1
        for e, value in ((nnz[1] - 1, fs.n), (0, -1), (3, struct.unpack_from("<i", blob, second + 4 * 2)[0]),
                         (nnz[1] - 1, 2**31 - 1)):
            bad = bytearray(blob)
            struct.pack_into("<i", bad, second + 4 * e, value)
            with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=48) as b:
                with pytest.raises(dmd.DMDError) as ei:
                    b.restore(bytes(bad))
                assert ei.value.code == dmd.E_INVAL
            with pytest.raises(dmd.DMDError) as ei:
                a.restore(bytes(bad))
            assert ei.value.code == dmd.E_INVAL
            assert np.array_equal(a.gram(), G0)
        with dmd.Stream(fs.n, m, r, dtype="c64_csr", max_nnz=48) as b:
            b.restore(bytes(blob))                 # the unmodified checkpoint is accepted
            assert np.array_equal(b.gram(), G0)
