"""Pins of the FP64 oracle against facts fixed by the paper and by linear algebra.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a special case that reduces to a textbook result, or a brute-force
construction (explicit A = X' X^+ on tiny inputs, exact rational arithmetic).
"""

from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle
from oracle import metrics


# ---------------------------------------------------------------- Gram (Sec. 2.1, Sec. 3.1)

def test_gram_matches_exact_rational_dots():
    """Exact rational inner products of float32 data, correctly rounded, agree with
    the oracle's FP64 Gram to within the summation error bound n * 2^-53 * sum|x_i y_i|."""
    rng = np.random.default_rng(7)
    W = rng.standard_normal((48, 5)).astype(np.float32)
    G = oracle.gram(W)
    for i in range(5):
        for j in range(5):
            exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(W[:, i], W[:, j]))
            bound = 48 * 2.0 ** -53 * float(np.sum(np.abs(W[:, i].astype(np.float64) * W[:, j])))
            assert abs(G[i, j] - float(exact)) <= bound


def test_gram_complex_is_conjugate_linear_in_first_argument():
    x = np.array([1 + 2j, 3 - 1j])
    y = np.array([2 - 1j, 1j])
    G = oracle.gram(np.stack([x, y], axis=1))
    # <x, y> = conj(x) . y written out by hand
    hand = (1 - 2j) * (2 - 1j) + (3 + 1j) * (1j)
    assert G[0, 1] == pytest.approx(hand)
    assert G[1, 0] == pytest.approx(np.conj(hand))
    assert G[0, 0] == pytest.approx(1 + 4 + 9 + 1)


def test_streamed_gram_equals_full_recompute():
    """Sec. 3.1: after shifts only the newest row/column is new; the kept Gram
    must equal the Gram of the current window recomputed from scratch."""
    g = gen.ModalStream(n=300, noise=1e-3)
    s = oracle.StreamingMoS(m=7, r=4)
    for t in range(23):
        s.push(g.frame(t))
        W = s.window()
        assert W.shape[1] == min(t + 1, 8)
        full = W.T @ W
        assert np.max(np.abs(s.G - full)) <= 1e-13 * np.max(np.abs(full))
    # the window really is the last m+1 frames
    np.testing.assert_array_equal(s.window(), g.frames(23 - 8, 8))


def test_streamed_gram_complex_sparse():
    fs = gen.FourierSparse(side=16, nnz=20, redraw=0.1)
    s = oracle.StreamingMoS(m=5, r=3)
    for t in range(12):
        idx, val = fs.frame(t)
        s.push(oracle.densify(idx, val, fs.n))
    W = s.window()
    np.testing.assert_allclose(s.G, W.conj().T @ W, rtol=0, atol=1e-14 * np.abs(s.G).max())
    assert np.allclose(s.G, s.G.conj().T)


# ---------------------------------------------------------------- SVD (Sec. 2.1)

def test_orthogonal_columns_give_norms_as_singular_values():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 6)))
    norms = np.array([3.0, 0.5, 7.0, 1.0, 2.0, 0.25])
    X = Q * norms
    sigma, V, U = oracle.mos_svd(X)
    np.testing.assert_allclose(sigma, np.sort(norms)[::-1], rtol=1e-13)
    # V is a signed permutation; canonical sign makes it a permutation
    np.testing.assert_allclose(np.abs(V), np.abs(V).round(), atol=1e-12)
    assert np.all(V.max(axis=0) > 0.999)
    res = oracle.exact_dmd(X, X, r=6, r_eff=6)
    np.testing.assert_allclose(res.sigma, np.sort(norms)[::-1], rtol=1e-13)


def test_rank_one_singular_value():
    u = np.arange(1.0, 11.0)
    v = np.array([2.0, -1.0, 0.5, 3.0])
    sigma, V, U = oracle.mos_svd(np.outer(u, v), r=1)
    assert sigma[0] == pytest.approx(np.linalg.norm(u) * np.linalg.norm(v), rel=1e-14)
    assert np.all(sigma[1:] < 1e-6 * sigma[0])
    np.testing.assert_allclose(np.abs(V[:, 0]), np.abs(v) / np.linalg.norm(v), rtol=1e-13)


def test_mos_agrees_with_lapack_svd():
    """Two independent routines: eigh of X^*X (method of snapshots) and LAPACK SVD."""
    g = gen.ModalStream(n=500, noise=1e-2)
    X = g.frames(0, 12)
    sigma, V, U = oracle.mos_svd(X, r=10)
    s_ref = np.linalg.svd(X, compute_uv=False)
    np.testing.assert_allclose(sigma[:10], s_ref[:10], rtol=1e-10)
    # U orthonormal and X V = U Sigma (Sec. 2.1, step 2)
    np.testing.assert_allclose(U.T @ U, np.eye(10), atol=1e-10)
    np.testing.assert_allclose(X @ V, U * sigma[:10], atol=1e-10 * sigma[0])


def test_r_effective_rule():
    s = np.array([10.0, 1.0, 1e-3, 1e-9, 0.0])
    assert oracle.r_effective(s, 5, 1e-7) == 3
    assert oracle.r_effective(s, 2, 1e-7) == 2
    assert oracle.r_effective(s, 5, 0.0) == 4
    assert oracle.r_effective(np.zeros(3), 3, 0.0) == 0


# ---------------------------------------------------------------- DMD (Sec. 2.2)

def test_closed_form_modal_eigenvalues_and_modes():
    """Noiseless sum of 5 complex modes: exact DMD recovers {lambda_k, conj lambda_k}
    and modes parallel to phi_k / conj(phi_k)."""
    g = gen.ModalStream(n=4096, noise=0.0)
    F = g.frames(0, 33)
    res = oracle.exact_dmd(F[:, :32], F[:, 1:], r=10)
    assert res.r_eff == 10
    assert res.sigma[10] / res.sigma[0] < 1e-14
    true = g.true_eigs()
    err, perm = metrics.eig_relerr(res.lam, true)
    assert err.max() < 1e-12
    true_modes = np.concatenate([g.phi, g.phi.conj()], axis=1)
    for i in range(10):
        assert metrics.sin_angle(res.Phi[:, i], true_modes[:, perm[i]]) < 1e-10


def test_rotation_worked_example():
    """x1=(1,0), x2=(0,1), x3=(-1,0): X' = A0 X with A0 the 90-degree rotation, so the
    DMD eigenvalues are +-i and the mode of lambda is (1, -lambda)/sqrt(2)."""
    F = np.array([[1.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    res = oracle.exact_dmd(F[:, :2], F[:, 1:], r=2, r_eff=2)
    np.testing.assert_allclose(np.sort_complex(res.lam), np.array([-1j, 1j]), atol=1e-15)
    for lam, phi in zip(res.lam, res.Phi.T):
        expect = np.array([1.0, -lam]) / np.sqrt(2.0)  # A0 (1, -lam) = (lam, 1) = lam (1, -lam)
        assert metrics.sin_angle(phi, expect) < 1e-14


def test_linear_system_recovers_operator_spectrum():
    """x_{t+1} = A0 x_t with n=8 < m=12: X X^+ = I, so A = X' X^+ = A0 and the
    rank-8 DMD spectrum is eig(A0)."""
    rng = np.random.default_rng(11)
    A0 = rng.standard_normal((8, 8)) / np.sqrt(8) * 0.9
    xs = [rng.standard_normal(8)]
    for _ in range(12):
        xs.append(A0 @ xs[-1])
    F = np.stack(xs, axis=1)
    res = oracle.exact_dmd(F[:, :12], F[:, 1:], r=8, r_eff=8)
    err, _ = metrics.eig_relerr(res.lam, np.linalg.eigvals(A0))
    assert err.max() < 1e-8
    for lam, phi in zip(res.lam, res.Phi.T):
        assert np.linalg.norm(A0 @ phi - lam * phi) < 1e-8 * np.linalg.norm(phi)


def test_bruteforce_explicit_operator():
    """Tiny n: the nonzero eigenvalues of the explicit A = X' pinv(X) equal Lambda and
    each column of Phi is an eigenvector of A (Sec. 2.2)."""
    rng = np.random.default_rng(5)
    n, m = 16, 6
    F = rng.standard_normal((n, m + 1))
    X, Xp = F[:, :m], F[:, 1:]
    A = Xp @ np.linalg.pinv(X)
    res = oracle.exact_dmd(X, Xp, r=m, r_eff=m)
    evA = np.linalg.eigvals(A)
    evA = evA[np.argsort(-np.abs(evA))][:m]
    err, _ = metrics.eig_relerr(res.lam, evA)
    assert err.max() < 1e-10
    for lam, phi in zip(res.lam, res.Phi.T):
        assert np.linalg.norm(A @ phi - lam * phi) < 1e-10 * np.linalg.norm(phi) * max(1, abs(lam))


def test_eigen_relation_at_scale():
    """A phi = lambda phi with A applied implicitly as X' V Sigma^-1 U^* (n = 20000)."""
    v = gen.BlobVideo(height=100, width=200, blob_sigma=6.0)
    F = v.frames(0, 17).astype(np.float64)
    res = oracle.exact_dmd(F[:, :16], F[:, 1:], r=8, r_eff=8, pod=True)
    for lam, phi in zip(res.lam, res.Phi.T):
        Aphi = F[:, 1:] @ (res.V / res.sigma[:8]) @ (res.U.conj().T @ phi)
        assert np.linalg.norm(Aphi - lam * phi) < 1e-9 * np.linalg.norm(phi)


def test_unitary_invariance_fourier_vs_space():
    """Sec. 3.5: SVD and DMD are invariant under a unitary transform.  DMD of
    Fourier coefficients and of the same fields in space give equal sigma and
    Lambda; the modes map by the (orthonormal) 2-D FFT."""
    fs = gen.FourierSparse(side=24, nnz=40, redraw=0.05)
    m = 10
    Fk = np.stack([oracle.densify(*fs.frame(t), fs.n) for t in range(m + 1)], axis=1)
    Fx = np.stack([np.fft.ifft2(Fk[:, j].reshape(24, 24), norm="ortho").reshape(-1)
                   for j in range(m + 1)], axis=1)
    a = oracle.exact_dmd(Fk[:, :m], Fk[:, 1:], r=6, r_eff=6)
    b = oracle.exact_dmd(Fx[:, :m], Fx[:, 1:], r=6, r_eff=6)
    np.testing.assert_allclose(a.sigma[:6], b.sigma[:6], rtol=1e-12)
    err, perm = metrics.eig_relerr(b.lam, a.lam)
    assert err.max() < 1e-10
    for i in range(6):
        mapped = np.fft.fft2(b.Phi[:, i].reshape(24, 24), norm="ortho").reshape(-1)
        assert metrics.phase_aligned_relerr(mapped, a.Phi[:, perm[i]]) < 1e-9


def test_streaming_algorithms_match_standard_dmd():
    """Algorithms 1-2 (streamed Gram, eig, A~ from Gram blocks) reproduce the SVD-route
    exact DMD on every window of a noisy stream."""
    g = gen.ModalStream(n=2000, noise=1e-3, stream=3)
    m, r = 12, 10
    s = oracle.StreamingMoS(m, r)
    for t in range(30):
        s.push(g.frame(t))
        if not s.ready():
            continue
        W = s.window()
        ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
        got = s.dmd()
        assert got.r_eff == ref.r_eff == r
        assert metrics.sigma_relerr(got.sigma[:r], ref.sigma[:r]).max() < 1e-9
        err, perm = metrics.eig_relerr(got.lam, ref.lam)
        assert err.max() < 1e-8
        for i in range(r):
            assert metrics.phase_aligned_relerr(got.Phi[:, i], ref.Phi[:, perm[i]]) < 1e-6


def test_conventions_sorted_and_canonical():
    g = gen.ModalStream(n=1000, noise=1e-3, stream=2)
    F = g.frames(0, 21)
    res = oracle.exact_dmd(F[:, :20], F[:, 1:], r=10)
    mod = np.abs(res.lam)
    assert np.all(np.diff(mod) <= 1e-12)
    for j in range(res.r_eff):
        w = res.W[:, j]
        assert np.linalg.norm(w) == pytest.approx(1.0, rel=1e-14)
        i = np.argmax(np.abs(w))
        assert abs(w[i].imag) < 1e-15 and w[i].real > 0


# ---------------------------------------------------------------- planted mistakes

def _closed_form_error(dmd_fn):
    g = gen.ModalStream(n=512, noise=0.0, stream=9)
    F = g.frames(0, 17)
    lam = dmd_fn(F[:, :16], F[:, 1:])
    err, _ = metrics.eig_relerr(lam, g.true_eigs())
    return err.max()


def _oracle_lam(X, Xp):
    return oracle.exact_dmd(X, Xp, r=10, r_eff=10).lam


def test_planted_mistakes_are_caught():
    """The closed-form pin fails for plausible slips in the DMD formula."""
    assert _closed_form_error(_oracle_lam) < 1e-10

    def wrong_operand(X, Xp):  # X in place of X' in A~
        U, s, Vh = np.linalg.svd(X, full_matrices=False)
        At = U[:, :10].T @ X @ Vh[:10].T / s[:10]
        return np.linalg.eigvals(At)

    def dropped_sigma(X, Xp):  # Sigma^-1 left out
        U, s, Vh = np.linalg.svd(X, full_matrices=False)
        At = U[:, :10].T @ Xp @ Vh[:10].T
        return np.linalg.eigvals(At)

    def transposed_v(X, Xp):  # V^* used where V belongs
        U, s, Vh = np.linalg.svd(X, full_matrices=False)
        At = U[:, :10].T @ Xp @ Vh[:, :10] / s[:10]
        return np.linalg.eigvals(At)

    for bad in (wrong_operand, dropped_sigma, transposed_v):
        assert _closed_form_error(bad) > 1e-3


def test_planted_gram_mistake_is_caught():
    """A Gram without the conjugate breaks Hermitian symmetry on complex data."""
    fs = gen.FourierSparse(side=16, nnz=20)
    W = np.stack([oracle.densify(*fs.frame(t), fs.n) for t in range(4)], axis=1)
    good = oracle.gram(W)
    bad = W.T @ W
    assert np.allclose(good, good.conj().T)
    assert not np.allclose(bad, bad.conj().T)
