"""Fourier-sparse snapshots in CSR form (complex64).

Stand-in for streams that arrive compressed in the Fourier domain (Sec. 3.5).
The grid is N x N with FFT index ordering; linear index l = iy * N + ix holds
wave vector (kx, ky) with kx = ix if ix < N/2 else ix - N (same for ky).

* Candidate pool: the 2 * nnz indices of lowest |k| (ties: lower linear index).
* Initial support: the nnz lowest-|k| indices.
* Each frame t >= 1 replaces ``round(redraw * nnz)`` support indices, chosen
  uniformly, with as many pool indices not in the support, chosen uniformly.
* Values: index l carries a_l * exp(i w_l t) with a_l ~ CN(0, 1) *
  max(|k|, 1)^(-5/3) (fixed per stream) and w_l = 2 pi (k . u) / N for a fixed
  advection velocity u (frozen-flow advection).

A frame is returned as ``(idx, val)``: sorted unique int32 indices and their
complex64 values.  The support chain is simulated once from t = 0, so any
frame can be regenerated on its own.
"""

import numpy as np

from .common import frame_rng, static_rng

CFG_ID = 4


class FourierSparse:
    def __init__(self, side=512, nnz=2621, redraw=0.05, velocity=(3.0, 1.7),
                 stream=0, cfg_id=CFG_ID):
        self.N = int(side)
        self.n = self.N * self.N
        self.nnz = int(nnz)
        self.n_redraw = int(round(redraw * self.nnz))
        self.stream = int(stream)
        self.cfg_id = int(cfg_id)
        ix = np.arange(self.N)
        kk = np.where(ix < self.N // 2, ix, ix - self.N)
        ky, kx = np.meshgrid(kk, kk, indexing="ij")
        kx = kx.reshape(-1).astype(np.float64)
        ky = ky.reshape(-1).astype(np.float64)
        kabs = np.hypot(kx, ky)
        lin = np.arange(self.n)
        order = np.lexsort((lin, kabs))
        self.pool = np.sort(order[: 2 * self.nnz])
        rng = static_rng(self.cfg_id, stream)
        pk = np.maximum(kabs[self.pool], 1.0)
        a = (rng.standard_normal(self.pool.size) + 1j * rng.standard_normal(self.pool.size)) / np.sqrt(2.0)
        self._amp = np.zeros(self.n, dtype=np.complex128)
        self._amp[self.pool] = a * pk ** (-5.0 / 3.0)
        u = np.asarray(velocity, dtype=np.float64)
        self._omega = np.zeros(self.n, dtype=np.float64)
        self._omega[self.pool] = 2 * np.pi * (kx[self.pool] * u[0] + ky[self.pool] * u[1]) / self.N
        self._supports = [np.sort(order[: self.nnz]).astype(np.int32)]

    def support(self, t: int) -> np.ndarray:
        while len(self._supports) <= t:
            s = len(self._supports)
            cur = self._supports[-1]
            rng = frame_rng(self.cfg_id, self.stream, s)
            drop = rng.choice(cur.size, self.n_redraw, replace=False)
            free = np.setdiff1d(self.pool, cur, assume_unique=True)
            add = rng.choice(free, self.n_redraw, replace=False)
            keep = np.delete(cur, drop)
            self._supports.append(np.sort(np.concatenate([keep, add])).astype(np.int32))
        return self._supports[t]

    def frame(self, t: int):
        idx = self.support(t)
        val = self._amp[idx] * np.exp(1j * self._omega[idx] * t)
        return idx.copy(), val.astype(np.complex64)

    def frame_dense(self, t: int) -> np.ndarray:
        idx, val = self.frame(t)
        x = np.zeros(self.n, dtype=np.complex64)
        x[idx] = val
        return x
