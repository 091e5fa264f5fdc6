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


def eig_sensitivity(ref) -> np.ndarray:
    """First-order relative sensitivity of each DMD eigenvalue of `ref` (a
    DMDResult) to an absolute perturbation of the window's inner products of
    size sigma_1^2, i.e. |d lambda_i| / |lambda_i| <= eps * kappa_i to first
    order when every Gram entry moves by at most eps * sigma_1^2.

    The method of snapshots forms A~ = Sigma^-1 V^* X^* X' V Sigma^-1 from the
    Gram (Sec. 3.1, Algorithm 2), so a Gram perturbation dG moves entry (j, k)
    of A~ by about dG_jk / (sigma_j sigma_k); with right eigenvectors W and
    left eigenvectors Y = W^-1 (rows), first-order perturbation theory of a
    simple eigenvalue gives
        |d lambda_i| <= sum_jk |Y_ij| |dA~_jk| |W_ki|
                     <= eps sigma_1^2 (sum_j |Y_ij| / sigma_j) (sum_k |W_ki| / sigma_k).
    Returned in the order of ref.lam."""
    k = int(ref.r_eff)
    s = np.asarray(ref.sigma, dtype=np.float64)[:k]
    W = np.asarray(ref.W)
    Y = np.linalg.inv(W)
    left = np.abs(Y) @ (1.0 / s)
    right = (1.0 / s) @ np.abs(W)
    return s[0] ** 2 * left * right / np.abs(np.asarray(ref.lam))
