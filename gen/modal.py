"""Sum of damped/oscillating complex modes observed as real snapshots.

x_t = sum_k Re(b_k * lambda_k**t * phi_k) + N(0, noise**2),  t = 0, 1, ...

with |lambda_k| ~ U[0.98, 1], arg lambda_k ~ U[0, pi], phi_k complex Gaussian
vectors scaled to unit 2-norm and b_k ~ CN(0, 1).  Each complex mode spans a
real 2-D subspace, so K modes give real rank 2K; the exact DMD of the
noiseless data has eigenvalues {lambda_k, conj(lambda_k)}.  ``noise`` is the
standard deviation of the additive Gaussian noise.
"""

import numpy as np

from .common import frame_rng, static_rng

CFG_ID = 1


class ModalStream:
    def __init__(self, n=4096, n_modes=5, noise=1e-3, stream=0, dtype=np.float64,
                 lam_abs=(0.98, 1.0), lam_arg=(0.0, np.pi)):
        self.n = int(n)
        self.n_modes = int(n_modes)
        self.noise = float(noise)
        self.stream = int(stream)
        self.dtype = np.dtype(dtype)
        rng = static_rng(CFG_ID, stream)
        mod = rng.uniform(lam_abs[0], lam_abs[1], self.n_modes)
        arg = rng.uniform(lam_arg[0], lam_arg[1], self.n_modes)
        self.lam = mod * np.exp(1j * arg)
        a = rng.standard_normal((self.n, self.n_modes))
        b = rng.standard_normal((self.n, self.n_modes))
        phi = a + 1j * b
        self.phi = phi / np.linalg.norm(phi, axis=0, keepdims=True)
        self.b = (rng.standard_normal(self.n_modes)
                  + 1j * rng.standard_normal(self.n_modes)) / np.sqrt(2.0)

    def frame(self, t: int) -> np.ndarray:
        coeff = self.b * self.lam ** int(t)
        x = (self.phi @ coeff).real
        if self.noise > 0:
            x = x + self.noise * frame_rng(CFG_ID, self.stream, t).standard_normal(self.n)
        return x.astype(self.dtype)

    def frames(self, t0: int, count: int) -> np.ndarray:
        """Frames t0 .. t0+count-1 as an (n, count) column-major-like array."""
        return np.stack([self.frame(t) for t in range(t0, t0 + count)], axis=1)

    def true_eigs(self) -> np.ndarray:
        """The 2K DMD eigenvalues of the noiseless stream."""
        return np.concatenate([self.lam, self.lam.conj()])
