"""Pins of the error metrics that the GPU parity tests rely on, and of the
oracle's POD-mode helper.

Each metric is checked against values worked out by hand (so that a metric
returning 0, dropping a normalisation or using the wrong phase fails), and
the eigenvalue-sensitivity bound against planted Gram perturbations.
"""

import math

import numpy as np
import pytest

import gen
import oracle
from oracle import metrics


# ---------------------------------------------------------------- sigma_relerr

def test_sigma_relerr_hand_values():
    err = metrics.sigma_relerr([1.1, 2.0], [1.0, 4.0, 9.0])   # reference longer: truncated
    np.testing.assert_allclose(err, [0.1, 0.5], rtol=1e-15)
    assert metrics.sigma_relerr([3.0], [3.0])[0] == 0.0
    # relative to the reference, not to the estimate
    assert metrics.sigma_relerr([2.0], [1.0])[0] == pytest.approx(1.0)
    assert metrics.sigma_relerr([1.0], [2.0])[0] == pytest.approx(0.5)


# ---------------------------------------------------------------- phase_aligned_relerr

def test_phase_aligned_relerr_hand_values():
    a = np.array([3.0, 4.0])
    # a pure phase is removed exactly
    assert metrics.phase_aligned_relerr(a * np.exp(0.7j), a) == pytest.approx(0.0, abs=1e-15)
    # orthogonal vectors: no phase helps, ||b - a|| / ||a|| = sqrt(2)
    assert metrics.phase_aligned_relerr([1.0, 0.0], [0.0, 1.0]) == pytest.approx(math.sqrt(2.0))
    # the scale is not removed: b = 2i a -> |2| - 1 = 1
    assert metrics.phase_aligned_relerr(2j * a, a) == pytest.approx(1.0)
    # b = (3, 4i), a = (3, 4): the best phase leaves
    # ||b||^2 + ||a||^2 - 2 |<b, a>| = 50 - 2 |9 - 16i| = 50 - 2 sqrt(337)
    want = math.sqrt(50.0 - 2.0 * math.sqrt(337.0)) / 5.0
    assert metrics.phase_aligned_relerr([3.0, 4j], a) == pytest.approx(want, rel=1e-13)
    # a component along a only: b = (1, 1), a = (1, 0) -> 1
    assert metrics.phase_aligned_relerr([1.0, 1.0], [1.0, 0.0]) == pytest.approx(1.0)


# ---------------------------------------------------------------- sin_angle

def test_sin_angle_hand_values():
    assert metrics.sin_angle([1.0, 0.0], [1.0, 1.0]) == pytest.approx(1.0 / math.sqrt(2.0))
    assert metrics.sin_angle([1.0, 0.0, 0.0], [0.0, 2.0, 0.0]) == pytest.approx(1.0)
    # complex multiples span the same line
    assert metrics.sin_angle([1.0, 1j], [1j, -1.0]) == pytest.approx(0.0, abs=1e-15)
    for t in (0.1, 0.5, 1.2, 2.5):
        assert metrics.sin_angle([1.0, 0.0], [math.cos(t), math.sin(t)]) == pytest.approx(abs(math.sin(t)))
    # scale-free in both arguments
    assert metrics.sin_angle([5.0, 0.0], [0.3, 0.3]) == pytest.approx(1.0 / math.sqrt(2.0))


# ---------------------------------------------------------------- eig_relerr / match_eigs

def test_eig_relerr_hand_values():
    lam_hat = np.array([1.1, 2j])
    lam = np.array([2j * (1 + 1e-3), 1.0])
    err, perm = metrics.eig_relerr(lam_hat, lam)
    assert list(perm) == [1, 0]
    np.testing.assert_allclose(err, [0.1, 1e-3 / (1 + 1e-3)], rtol=1e-12)
    with pytest.raises(ValueError):
        metrics.match_eigs([1, 2, 3], [1, 2])


# ---------------------------------------------------------------- eig_sensitivity

def test_eig_sensitivity_hand_value_diagonal():
    """Diagonal A~ (W = I): kappa_i = sigma_1^2 / (sigma_i^2 |lambda_i|)."""
    sig = np.array([4.0, 2.0, 1.0])
    lam = np.array([0.9, 0.5j, -0.25])
    ref = oracle.DMDResult(sigma=sig, r_eff=3, V=np.eye(3), Atilde=np.diag(lam), lam=lam,
                           W=np.eye(3, dtype=complex), Phi=None)
    np.testing.assert_allclose(metrics.eig_sensitivity(ref), 16.0 / (sig ** 2 * np.abs(lam)), rtol=1e-14)


def test_eig_sensitivity_bounds_planted_gram_perturbations():
    """Perturb the window's Gram by eps sigma_1^2 (random symmetric) and redo
    the small solves of Algorithm 2: every eigenvalue moves by at most a small
    multiple of eps kappa_i, and the bound is attained within a factor 100
    (it is not vacuous)."""
    rng = np.random.default_rng(5)
    v = gen.BlobVideo(height=40, width=60, blob_sigma=4.0)
    m, r = 16, 8
    F = oracle.as_fp64(v.frames(0, m + 1))
    G = oracle.gram(F)
    ref = oracle.dmd_from_gram(G, m, r)
    kap = metrics.eig_sensitivity(ref)
    eps = 1e-12
    worst = 0.0
    for _ in range(6):
        E = rng.uniform(-1.0, 1.0, G.shape)
        E = 0.5 * (E + E.T)
        pert = oracle.dmd_from_gram(G + eps * ref.sigma[0] ** 2 * E, m, r, r_eff=ref.r_eff)
        err, perm = metrics.eig_relerr(pert.lam, ref.lam)
        ratio = err / (eps * kap[perm])
        assert ratio.max() < 4.0, ratio.max()
        worst = max(worst, ratio.max())
    assert worst > 1e-2


# ---------------------------------------------------------------- pod_modes

def test_pod_modes_equal_lapack_left_singular_vectors():
    """U = X V Sigma^-1 (Sec. 2.1, step 2) from the method of snapshots equals
    LAPACK's left singular vectors of X up to each column's sign, and is
    orthonormal."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((500, 7)) @ np.diag([9.0, 5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    sigma, V, _ = oracle.mos_svd(X)
    U = oracle.pod_modes(X, V[:, :5], sigma)
    Ul, sl, _ = np.linalg.svd(X, full_matrices=False)
    for j in range(5):
        sgn = np.sign(Ul[:, j] @ U[:, j])
        np.testing.assert_allclose(U[:, j], sgn * Ul[:, j], atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(5), atol=1e-12)
    np.testing.assert_allclose(sigma[:5], sl[:5], rtol=1e-12)
