"""Synthetic 2-D flow: a sum of travelling Fourier waves.

Stand-in for the scientific-computing streams of the paper (Sec. 1, Sec. 3.5).
On an L x L periodic grid (pixel index y * L + x, truncated to n entries)

    x_t(x, y) = sum_{k=0}^{K-1} A_k cos(2 pi (kx_k x + ky_k y) / L - w_k t + th_k)

with A_k = 10^(-k/2) (so sigma_1 / sigma_2K ~ 10^((K-1)/2)), distinct integer
wave vectors (components in [-kmax, kmax], nonzero, no two equal up to sign),
w_k ~ U[0.05, 3.0] and th_k ~ U[0, 2 pi).  Each wave is a complex pair with
DMD eigenvalues exp(-i w_k) and exp(+i w_k); the data have real rank 2K.
Frames are noiseless and stored as float32.
"""

import numpy as np

from .common import static_rng

CFG_ID = 3


class TravelingWaves:
    def __init__(self, n=1 << 20, n_waves=8, kmax=16, omega=(0.05, 3.0), stream=0,
                 cfg_id=CFG_ID, side=None):
        self.n = int(n)
        self.L = int(side) if side is not None else 1 << int(np.ceil(np.log2(np.sqrt(self.n))))
        assert self.L * self.L >= self.n
        self.stream = int(stream)
        self.K = int(n_waves)
        rng = static_rng(cfg_id, stream)
        kv = []
        seen = set()
        while len(kv) < self.K:
            k = tuple(int(v) for v in rng.integers(-kmax, kmax + 1, 2))
            neg = (-k[0], -k[1])
            if k == (0, 0) or k in seen or neg in seen or k == neg:
                continue
            seen.add(k)
            kv.append(k)
        self.kvec = np.array(kv, dtype=np.int64)
        self.amp = 10.0 ** (-np.arange(self.K) / 2.0)
        self.omega = rng.uniform(omega[0], omega[1], self.K)
        self.theta = rng.uniform(0.0, 2 * np.pi, self.K)
        coord = np.arange(self.L, dtype=np.float64)
        # separable complex exponentials exp(i 2 pi k x / L) for each wave
        self._ex = np.exp(2j * np.pi * np.outer(self.kvec[:, 0], coord) / self.L)
        self._ey = np.exp(2j * np.pi * np.outer(self.kvec[:, 1], coord) / self.L)

    def frame(self, t: int) -> np.ndarray:
        img = np.zeros((self.L, self.L), dtype=np.float64)
        for k in range(self.K):
            ph = self.amp[k] * np.exp(1j * (self.theta[k] - self.omega[k] * t))
            img += (ph * np.outer(self._ey[k], self._ex[k])).real
        return img.reshape(-1)[: self.n].astype(np.float32)

    def frames(self, t0: int, count: int) -> np.ndarray:
        return np.stack([self.frame(t) for t in range(t0, t0 + count)], axis=1)

    def true_eigs(self) -> np.ndarray:
        return np.concatenate([np.exp(-1j * self.omega), np.exp(1j * self.omega)])
