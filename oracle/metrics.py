"""Error metrics between a computed DMD and the oracle's (test infrastructure)."""

import numpy as np
from scipy.optimize import linear_sum_assignment
from scipy.linalg import subspace_angles


def sigma_relerr(s_hat, s) -> np.ndarray:
    s_hat = np.asarray(s_hat, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)[: s_hat.size]
    return np.abs(s_hat - s) / np.abs(s)


def match_eigs(lam_hat, lam) -> np.ndarray:
    """perm such that lam_hat[i] pairs with lam[perm[i]] (min total |difference|)."""
    lam_hat = np.asarray(lam_hat)
    lam = np.asarray(lam)
    if lam_hat.size > lam.size:
        raise ValueError(f"cannot match {lam_hat.size} eigenvalues to {lam.size}")
    cost = np.abs(lam_hat[:, None] - lam[None, :])
    row, col = linear_sum_assignment(cost)
    perm = np.empty(lam_hat.size, dtype=np.int64)
    perm[row] = col
    return perm


def eig_relerr(lam_hat, lam):
    perm = match_eigs(lam_hat, lam)
    lam = np.asarray(lam)[perm]
    return np.abs(np.asarray(lam_hat) - lam) / np.abs(lam), perm


def sin_angle(a, b) -> float:
    """Sine of the angle between the lines spanned by vectors a and b."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    return float(np.linalg.norm(b - a * np.vdot(a, b)))


def phase_aligned_relerr(b, a) -> float:
    """||b e^{i t} - a|| / ||a|| with the phase t that minimises it."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    c = np.vdot(b, a)
    ph = c / abs(c) if c != 0 else 1.0
    return float(np.linalg.norm(b * ph - a) / np.linalg.norm(a))


def max_subspace_angle(A, B) -> float:
    return float(np.max(subspace_angles(np.asarray(A), np.asarray(B))))


def rel_fro(A_hat, A) -> float:
    A = np.asarray(A)
    return float(np.linalg.norm(np.asarray(A_hat) - A) / np.linalg.norm(A))


def max_rel_entry(A_hat, A, scale=None) -> float:
    """max |A_hat - A| / scale (scale defaults to max |A|)."""
    A = np.asarray(A)
    s = np.max(np.abs(A)) if scale is None else scale
    return float(np.max(np.abs(np.asarray(A_hat) - A)) / s)
