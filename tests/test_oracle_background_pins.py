"""Pins of the oracle's mode amplitudes and background split (Sec. 3.3,
Algorithm 3) against closed forms and an independent route.

* Noiseless modal data lies exactly in the span of the DMD modes, so the
  amplitudes must reproduce every snapshot of the window: x_{j+1} = Phi
  Lambda^j b, the first (x_1 = Phi b, the defining equation of Sec. 3.3) and
  the newest (the exponent the background split uses).
* The paper's fast formula b = (W Lambda)^-1 alpha_1 must equal the
  least-squares amplitudes Phi^+ x_1 (the first formula of Sec. 3.3) there.
* A constant non-negative background plus one travelling wave (a conjugate
  pair of modes): the mode with lambda = 1 is the background, and the
  foreground of the newest snapshot is exactly the wave.
* Planted mistakes (column 0 of V instead of row 0, exponent m+1) fail.
"""

import numpy as np

import gen
import oracle
from oracle import background as bgo


def noiseless_modal(m=32):
    g = gen.ModalStream(n=4096, noise=0.0)
    F = g.frames(0, m + 1)
    res = oracle.exact_dmd(F[:, :m], F[:, 1:], 10)
    assert res.r_eff == 10
    return F, res


def test_amplitudes_reproduce_every_snapshot_of_the_window():
    F, res = noiseless_modal()
    m = F.shape[1] - 1
    b = bgo.amplitudes(res)
    scale = np.linalg.norm(F, axis=0).max()
    for j in range(m + 1):
        xj = res.Phi @ (res.lam ** j * b)
        assert np.linalg.norm(xj - F[:, j]) < 1e-9 * scale, j


def test_fast_amplitudes_equal_least_squares():
    F, res = noiseless_modal()
    b = bgo.amplitudes(res)
    b_ls = bgo.amplitudes_lstsq(res, F[:, 0])
    assert np.max(np.abs(b - b_ls)) < 1e-8 * np.max(np.abs(b_ls))


def test_background_split_closed_form():
    """x_t = c + a (cos(w t + th) p1 + sin(w t + th) p2), c >= 0: eigenvalues
    {1, e^{+-iw}}; the background is c and the foreground of the newest
    snapshot is the wave at t = m."""
    rng = np.random.default_rng(11)
    n, m = 500, 10
    c = rng.uniform(0.5, 1.5, n)
    p1, p2 = rng.standard_normal((2, n))
    a, w, th = 3.0, 0.4, 0.3
    t = np.arange(m + 1)
    wave = a * (np.cos(w * t + th)[None, :] * p1[:, None] + np.sin(w * t + th)[None, :] * p2[:, None])
    F = c[:, None] + wave
    res = oracle.exact_dmd(F[:, :m], F[:, 1:], 3)
    assert res.r_eff == 3
    assert np.allclose(np.sort(np.angle(res.lam)), [-w, 0.0, w], atol=1e-10)
    s, bg, i = bgo.background_split(F, res)
    assert abs(res.lam[i] - 1.0) < 1e-10
    assert np.max(np.abs(bg - c)) < 1e-9
    assert np.max(np.abs(s - wave[:, m])) < 1e-9


def test_background_index_rule():
    lam = np.array([0.5, 1.02, 0.99 * np.exp(0.1j), 0.0])
    assert bgo.background_index(lam) == 1
    assert bgo.background_index(np.array([1j, -1j])) == 0  # |log| = pi/2 both: lowest index


def test_planted_mistakes_are_caught():
    F, res = noiseless_modal()
    m = F.shape[1] - 1
    scale = np.linalg.norm(F[:, 0])
    k = res.r_eff
    # alpha_1 from column 0 of V (as the listing writes) instead of row 0
    alpha_col = res.sigma[:k] * np.conj(res.V[:k, 0])
    b_col = np.linalg.solve(res.W * res.lam[None, :], alpha_col)
    assert np.linalg.norm(res.Phi @ b_col - F[:, 0]) > 1e-3 * scale
    # the newest snapshot with exponent m+1 instead of m
    b = bgo.amplitudes(res)
    assert np.linalg.norm(res.Phi @ (res.lam ** (m + 1) * b) - F[:, m]) > 1e-3 * scale
