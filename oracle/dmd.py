"""Plain FP64 implementations of the method-of-snapshots SVD and exact DMD.

Test infrastructure only (see the package docstring).  Every routine here is
the textbook definition written out with NumPy; the only library steps are
matrix products, ``numpy.linalg.svd``, ``eigh`` and ``eig``.
"""

from dataclasses import dataclass
from typing import Optional

import numpy as np


def as_fp64(x) -> np.ndarray:
    """Widen to float64 / complex128 (exact for float32 / complex64 input)."""
    x = np.asarray(x)
    return x.astype(np.complex128) if np.iscomplexobj(x) else x.astype(np.float64)


def densify(idx, val, n) -> np.ndarray:
    """Dense complex128 vector of length n from sorted CSR (idx, val)."""
    x = np.zeros(int(n), dtype=np.complex128)
    x[np.asarray(idx, dtype=np.int64)] = np.asarray(val, dtype=np.complex128)
    return x


def gram(W) -> np.ndarray:
    """All inner products <w_i, w_j> = w_i^* w_j of the columns of W.

    This is the matrix X^* X of the method of snapshots (Sec. 2.1, step 1) and
    the first-step branch of Algorithm 1.
    """
    W = as_fp64(W)
    return W.conj().T @ W


def default_rcond(eps_acc: float = 2.0 ** -52) -> float:
    """Rank cut-off relative to sigma_1 for a Gram accumulated with unit round-off eps_acc.

    The Gram carries an absolute error of order eps_acc * sigma_1^2, so
    sigma_k below ~sqrt(eps_acc) * sigma_1 cannot be resolved (the method of
    snapshots squares the condition number, Sec. 2.1).
    """
    return 10.0 * np.sqrt(eps_acc)


def r_effective(sigma, r: int, rcond: float) -> int:
    """Number of leading singular values (at most r) above rcond * sigma_1."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.size == 0 or not sigma[0] > 0:
        return 0
    thr = rcond * sigma[0]
    k = 0
    while k < min(int(r), sigma.size) and sigma[k] > thr:
        k += 1
    return k


def canonical_columns(M, normalize: bool = True) -> np.ndarray:
    """Scale each column to unit 2-norm and rotate its phase so that the entry of
    largest modulus (first one on ties) is real and positive."""
    M = np.array(M, dtype=np.complex128 if np.iscomplexobj(M) else np.float64, copy=True)
    for j in range(M.shape[1]):
        col = M[:, j]
        if normalize:
            nrm = np.linalg.norm(col)
            if nrm > 0:
                col = col / nrm
        i = int(np.argmax(np.abs(col)))
        a = col[i]
        if a != 0:
            col = col * (np.conj(a) / abs(a))
        M[:, j] = col
    return M


def column_phases(M) -> np.ndarray:
    """Unit-modulus factors d_j with canonical_columns(M, normalize=False) == M * d."""
    M = np.asarray(M)
    d = np.ones(M.shape[1], dtype=np.complex128 if np.iscomplexobj(M) else np.float64)
    for j in range(M.shape[1]):
        a = M[int(np.argmax(np.abs(M[:, j]))), j]
        if a != 0:
            d[j] = np.conj(a) / abs(a)
    return d


def sort_eigs(lam, W):
    """Order eigenpairs by descending |lambda|, ties by ascending arg(lambda)."""
    lam = np.asarray(lam)
    order = np.lexsort((np.angle(lam), -np.abs(lam)))
    return lam[order], np.asarray(W)[:, order]


@dataclass
class DMDResult:
    sigma: np.ndarray          # singular values of X, descending (all of them)
    r_eff: int                 # truncation rank used
    V: np.ndarray              # m x r_eff right singular vectors (canonical columns)
    Atilde: np.ndarray         # r_eff x r_eff projected operator
    lam: np.ndarray            # r_eff DMD eigenvalues, sorted
    W: np.ndarray              # r_eff x r_eff eigenvectors of Atilde (canonical columns)
    Phi: Optional[np.ndarray]  # n x r_eff DMD modes X' V Sigma^-1 W
    U: Optional[np.ndarray] = None  # n x r_eff POD modes X V Sigma^-1


def mos_svd(X, r: Optional[int] = None):
    """Method-of-snapshots SVD (Sec. 2.1): X^* X V = V Lambda, sigma = sqrt|Lambda|,
    U = X V Sigma^-1.  Returns (sigma, V, U) with sigma descending, V canonical,
    truncated to the r leading triplets when r is given."""
    X = as_fp64(X)
    ev, V = np.linalg.eigh(gram(X))
    sigma = np.sqrt(np.abs(ev))
    order = np.argsort(-sigma, kind="stable")
    sigma, V = sigma[order], V[:, order]
    V = canonical_columns(V)
    k = V.shape[1] if r is None else int(r)
    U = X @ (V[:, :k] / sigma[:k])
    return sigma, V[:, :k], U


def exact_dmd(X, Xp, r: int, r_eff: Optional[int] = None, rcond: Optional[float] = None,
              modes: bool = True, pod: bool = False) -> DMDResult:
    """Exact DMD of the pair (X, X') by the SVD route (Sec. 2.2).

    X = U Sigma V^*  (thin SVD, LAPACK), truncated to k = r_eff leading triplets;
    A~  = U^* X' V Sigma^-1          (Eq. Atilde)
    A~ W = W Lambda                  (eigendecomposition of A~)
    Phi = X' V Sigma^-1 W            (Eq. Phi)
    k defaults to r_effective(sigma, r, rcond).
    """
    X = as_fp64(X)
    Xp = as_fp64(Xp)
    U, s, Vh = np.linalg.svd(X, full_matrices=False)
    if r_eff is None:
        r_eff = r_effective(s, r, default_rcond() if rcond is None else rcond)
    k = int(r_eff)
    V = Vh[:k].conj().T
    d = column_phases(V)
    V = V * d
    U = U[:, :k] * d
    s_k = s[:k]
    At = U.conj().T @ Xp @ V / s_k
    lam, W = np.linalg.eig(At)
    lam, W = sort_eigs(lam, W)
    W = canonical_columns(W)
    Phi = (Xp @ (V / s_k)) @ W if modes else None
    return DMDResult(sigma=s, r_eff=k, V=V, Atilde=At, lam=lam, W=W, Phi=Phi,
                     U=U if pod else None)


def dmd_from_gram(Gw, m: int, r: int, r_eff: Optional[int] = None,
                  rcond: Optional[float] = None, window=None) -> DMDResult:
    """Streaming-DMD small solves (Algorithm 2) from the (m+1) x (m+1) Gram of a window.

    xtx = G[0:m, 0:m] is the Gram of X, xty = G[0:m, 1:m+1] = X^* X'.
    eig(xtx) -> sigma = sort(sqrt|s|) with V permuted alike (Algorithm 1);
    vsi = V Sigma^-1; A~ = vsi^* xty vsi; A~ W = W Lambda; Phi = X' vsi W.
    """
    Gw = np.asarray(Gw)
    xtx = Gw[:m, :m]
    xty = Gw[:m, 1:m + 1]
    ev, V = np.linalg.eigh(xtx)
    sigma = np.sqrt(np.abs(ev))
    order = np.argsort(-sigma, kind="stable")
    sigma, V = sigma[order], V[:, order]
    V = canonical_columns(V)
    if r_eff is None:
        r_eff = r_effective(sigma, r, default_rcond() if rcond is None else rcond)
    k = int(r_eff)
    vsi = V[:, :k] / sigma[:k]
    At = vsi.conj().T @ xty @ vsi
    lam, W = np.linalg.eig(At)
    lam, W = sort_eigs(lam, W)
    W = canonical_columns(W)
    Phi = None
    if window is not None:
        Xp = as_fp64(window)[:, 1:m + 1]
        Phi = Xp @ (vsi @ W)
    return DMDResult(sigma=sigma, r_eff=k, V=V[:, :k], Atilde=At, lam=lam, W=W, Phi=Phi)


def pod_modes(X, V, sigma) -> np.ndarray:
    """U = X V Sigma^-1 (Sec. 2.1, step 2) for the given leading triplets."""
    V = np.asarray(V)
    k = V.shape[1]
    return as_fp64(X) @ (V / np.asarray(sigma)[:k])


class StreamingMoS:
    """Streaming method-of-snapshots SVD/DMD (Algorithms 1 and 2), FP64.

    The window holds the last m+1 snapshots; X is its first m columns and X'
    its last m.  The Gram of the whole window is kept: on each push the
    oldest snapshot's row and column are dropped (the shift of Algorithm 1),
    the inner products among the surviving snapshots are reused, and only the
    new snapshot's inner products with the window are computed (Sec. 3.1).
    G[0:m, 0:m] is Algorithm 1's xtx and G[0:m, 1:m+1] Algorithm 2's xty, so
    one new column serves both.  Before the window is full the Gram grows by
    appending (nothing is evicted).
    """

    def __init__(self, m: int, r: int, rcond: Optional[float] = None):
        self.m = int(m)
        self.r = int(r)
        self.rcond = default_rcond() if rcond is None else float(rcond)
        self.cols = []
        self.G = np.zeros((0, 0))
        self.count = 0

    def push(self, x) -> None:
        x = as_fp64(x).reshape(-1)
        if len(self.cols) == self.m + 1:
            self.cols.pop(0)
            self.G = self.G[1:, 1:]
        self.cols.append(x)
        g = np.array([np.vdot(c, x) for c in self.cols])  # <x_j, x_new> = x_j^* x_new
        k = len(self.cols)
        dt = np.complex128 if (np.iscomplexobj(self.G) or np.iscomplexobj(g)) else np.float64
        Gn = np.zeros((k, k), dtype=dt)
        Gn[:k - 1, :k - 1] = self.G
        Gn[:, k - 1] = g
        Gn[k - 1, :] = g.conj()
        self.G = Gn
        self.count += 1

    def ready(self) -> bool:
        return len(self.cols) == self.m + 1

    def window(self) -> np.ndarray:
        return np.stack(self.cols, axis=1)

    def dmd(self, r_eff: Optional[int] = None, modes: bool = True) -> DMDResult:
        if not self.ready():
            raise RuntimeError("window not full")
        return dmd_from_gram(self.G, self.m, self.r, r_eff=r_eff, rcond=self.rcond,
                             window=self.window() if modes else None)
