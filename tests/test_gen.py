"""Synthetic input generators: reproducible, independent per frame, right shapes."""

import numpy as np

import gen


def test_modal_frames_reproducible_and_real_rank():
    a = gen.ModalStream(n=256, noise=0.0)
    b = gen.ModalStream(n=256, noise=0.0)
    np.testing.assert_array_equal(a.frame(17), b.frame(17))
    F = a.frames(0, 20)
    s = np.linalg.svd(F, compute_uv=False)
    assert s[9] / s[0] > 1e-6 and s[10] / s[0] < 1e-12  # 5 complex modes -> real rank 10
    assert np.all(np.abs(a.lam) >= 0.98) and np.all(np.abs(a.lam) <= 1.0)


def test_video_frame_independent_of_history():
    v1 = gen.BlobVideo(height=60, width=80, blob_sigma=5.0)
    v2 = gen.BlobVideo(height=60, width=80, blob_sigma=5.0)
    f = v1.frame(40)
    assert f.dtype == np.float32 and f.shape == (4800,)
    _ = [v2.frame(t) for t in range(3)]
    np.testing.assert_array_equal(v2.frame(40), f)
    assert 0.0 <= v1.bg.min() and v1.bg.max() <= 1.0


def test_flow_rank_and_eigs():
    w = gen.TravelingWaves(n=64 * 64, n_waves=4, kmax=8)
    F = w.frames(0, 20).astype(np.float64)
    s = np.linalg.svd(F, compute_uv=False)
    assert s[7] / s[0] > 1e-3 and s[8] / s[0] < 1e-6  # 4 waves -> real rank 8
    assert np.allclose(np.abs(w.true_eigs()), 1.0)


def test_fourier_sparse_support_chain():
    fs = gen.FourierSparse(side=32, nnz=50, redraw=0.1)
    idx0, val0 = fs.frame(0)
    idx5, val5 = fs.frame(5)
    assert idx0.dtype == np.int32 and val0.dtype == np.complex64
    assert idx5.size == 50 and np.all(np.diff(idx5) > 0)
    assert set(idx5.tolist()) <= set(fs.pool.tolist())
    assert len(set(idx0.tolist()) - set(fs.support(1).tolist())) == 5
    other = gen.FourierSparse(side=32, nnz=50, redraw=0.1)
    np.testing.assert_array_equal(other.frame(5)[0], idx5)
    np.testing.assert_array_equal(other.frame(5)[1], val5)


def test_stream_mix_parameters():
    mix = gen.stream_mix(64)
    assert len(mix) == 64
    for s in mix:
        assert 65536 <= s.n <= 2097152
        assert s.m in (16, 32, 64, 128) and s.r == min(s.m // 2, 32)
    small = gen.MixStream(stream=0, n=5000, m=16, r=8, kind="video")
    assert small.frame(3).shape == (5000,)
    flow = gen.MixStream(stream=1, n=5000, m=16, r=8, kind="flow")
    assert flow.frame(3).shape == (5000,)
