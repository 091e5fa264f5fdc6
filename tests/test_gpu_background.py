"""GPU parity of the mode amplitudes and the background split (Sec. 3.3,
Algorithm 3) against the FP64 oracle.

Tolerances: b comes from the FP64 small solves (like lambda): 1e-7 relative
to max |b| (the solve of W Lambda b = alpha_1 adds the conditioning of W);
the background index must match; fg and |l| are one FP64 pass (1e-9 of
max |x|) or an FP32 pass with FP32 coefficients (2e-4 of max |x|, as the
FP32 projections).
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import background as bgo
from oracle import metrics

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


def check_split(s, W, m, r, tol_x):
    ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
    lam, sig, _ = s.eigs()
    err, perm = metrics.eig_relerr(lam, ref.lam)
    assert err.max() < 1e-8
    b, idx, _ = s.amplitudes()
    b_ref = bgo.amplitudes(ref)
    assert b.size == ref.r_eff
    assert np.max(np.abs(b - b_ref[perm])) < 1e-7 * np.max(np.abs(b_ref)), np.max(np.abs(b - b_ref[perm]))
    i_ref = bgo.background_index(ref.lam)
    assert perm[idx] == i_ref
    s_ref, bg_ref, _ = bgo.background_split(W, ref, b_ref)
    fg, bg = s.background()
    scale = np.max(np.abs(oracle.as_fp64(W)))
    assert np.max(np.abs(fg.cpu().numpy() - s_ref)) < tol_x * scale
    assert np.max(np.abs(bg.cpu().numpy() - bg_ref)) < tol_x * scale


@pytest.mark.parametrize("n", [4133, 1000])
def test_modal_fp64_amplitudes_and_background(n):
    dmd = _dmd()
    m, r = 16, 6
    frames = gen.ModalStream(n=n, noise=1e-3).frames(0, m + 4)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, dtype="f64") as s:
        for t in range(m):
            s.push(X[t])
        with pytest.raises(dmd.DMDError) as ei:
            s.amplitudes()
        assert ei.value.code == dmd.E_NOT_READY
        sentinel = torch.full((n,), 5.0, dtype=torch.float64, device="cuda")
        s.background(fg=sentinel, want_bg=False)
        assert torch.all(sentinel == 5.0).item()          # no full window yet: untouched
        for t in range(m, m + 4):
            s.push(X[t])
            check_split(s, frames[:, t - m:t + 1], m, r, 1e-9)


def test_background_closed_form_on_gpu():
    """Constant background plus a travelling wave: fg is the wave, bg the background."""
    dmd = _dmd()
    rng = np.random.default_rng(11)
    n, m = 5000, 10
    c = rng.uniform(0.5, 1.5, n)
    p1, p2 = rng.standard_normal((2, n))
    a, w, th = 3.0, 0.4, 0.3
    t = np.arange(m + 1)
    wave = a * (np.cos(w * t + th)[None, :] * p1[:, None] + np.sin(w * t + th)[None, :] * p2[:, None])
    F = c[:, None] + wave
    X = torch.from_numpy(F.T.copy()).cuda()
    with dmd.Stream(n, m, 3, dtype="f64") as s:
        for k in range(m + 1):
            s.push(X[k])
        lam, _, _ = s.eigs()
        b, idx, _ = s.amplitudes()
        assert abs(lam[idx] - 1.0) < 1e-9
        fg, bg = s.background()
        assert np.max(np.abs(bg.cpu().numpy() - c)) < 1e-8
        assert np.max(np.abs(fg.cpu().numpy() - wave[:, m])) < 1e-8


@pytest.mark.parametrize("prec,tol", [("default", 2e-4), ("fp64", 1e-9)])
def test_video_fp32_background(prec, tol):
    dmd = _dmd()
    H, W, m, r = 100, 130, 37, 12
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=4.0).frames(0, m + 3)
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(H * W, m, r, precision=prec) as s:
        for t in range(m + 3):
            s.push(X[t])
            if t >= m:
                check_split(s, frames[:, t - m:t + 1], m, r, tol)


def test_background_rejects_sparse_streams():
    dmd = _dmd()
    with dmd.Stream(1000, 8, 4, dtype="c64_csr", max_nnz=16) as s:
        with pytest.raises(dmd.DMDError) as ei:
            s.background(fg=torch.zeros(1000, dtype=torch.complex64, device="cuda"), want_bg=False)
        assert ei.value.code in (dmd.E_UNSUPPORTED,)
