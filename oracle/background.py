"""Mode amplitudes and streaming background subtraction (Sec. 3.3, Algorithm 3).

Test infrastructure only, like the rest of this package.

Readings (the paper is ambiguous here):
* alpha_1, the POD coefficients of the first snapshot x_1, are U_r^* x_1.
  With U = X V Sigma^-1 and X^* X = V Sigma^2 V^* this is Sigma_r V_r^* e_1,
  i.e. alpha_1[k] = sigma_k conj(V[0, k]) -- the first *row* of V (Algorithm 3
  writes column 0).
* The background mode is argmin_i |log lambda_i| (Algorithm 3; the complex
  logarithm's modulus, i.e. the eigenvalue closest to 1 on the log scale),
  lowest index on ties.
* Snapshot j of the window (j = 0 for x_1) is reconstructed as
  Phi Lambda^j b, so the newest snapshot x_{m+1} of an (m+1)-column window
  uses lambda^m (Algorithm 3's streaming branch raises lambda to the number of
  window columns, one more).
"""

import numpy as np

from .dmd import DMDResult, as_fp64


def amplitudes(res: DMDResult) -> np.ndarray:
    """b = (W Lambda)^-1 alpha_1 (Sec. 3.3): from x_1 = Phi b, U alpha_1 =
    X' V Sigma^-1 W b, so alpha_1 = A~ W b = W Lambda b."""
    k = res.r_eff
    alpha1 = res.sigma[:k] * np.conj(res.V[0, :k])
    WL = res.W * res.lam[None, :]
    return np.linalg.solve(WL, alpha1)


def amplitudes_lstsq(res: DMDResult, x1) -> np.ndarray:
    """The least-squares amplitudes b = Phi^+ x_1 (the first formula of Sec. 3.3)."""
    return np.linalg.lstsq(res.Phi, as_fp64(x1).astype(np.complex128), rcond=None)[0]


def background_index(lam) -> int:
    """argmin_i |log lambda_i| (Algorithm 3), lowest index on ties; lambda = 0 never wins."""
    lam = np.asarray(lam, dtype=np.complex128)
    with np.errstate(divide="ignore"):
        d = np.abs(np.log(lam))
    return int(np.argmin(d))


def background_split(window, res: DMDResult, b=None):
    """Background and foreground of the newest snapshot of an (m+1)-column window.

    l = b_i lambda_i^m phi_i with i the background mode, s = x_{m+1} - |l|
    (Algorithm 3, streaming branch).  Returns (s, |l|, i)."""
    W = as_fp64(window)
    m = W.shape[1] - 1
    if b is None:
        b = amplitudes(res)
    i = background_index(res.lam)
    l = b[i] * res.lam[i] ** m * res.Phi[:, i]
    bg = np.abs(l)
    return W[:, m] - bg, bg, i
