"""Synthetic greyscale video: smooth background + moving Gaussian blobs + noise.

Stand-in for the paper's surveillance-video experiments (Sec. 4).  Frame t is

    bg(y, x) + sum_b amp * exp(-(dx_b(t)^2 + dy_b(t)^2) / (2 s^2)) + N(0, noise^2)

* bg: U[0, 1] noise smoothed by a periodic Gaussian filter of std ``bg_sigma``
  pixels, then min-max scaled to [0, 1].
* blobs: Gaussian profile of std ``blob_sigma`` pixels, amplitude ``amp``,
  start position uniform over the frame, direction uniform, speed
  U[speed_lo, speed_hi] px/frame, periodic wrap; dx, dy are wrapped distances.
* noise: standard deviation ``noise`` (per pixel).

Pixels are stored row-major (index y * W + x) as float32.
"""

import numpy as np
from scipy.ndimage import gaussian_filter

from .common import frame_rng, static_rng

CFG_ID = 2


class BlobVideo:
    def __init__(self, height=1080, width=1920, n_blobs=4, blob_sigma=30.0,
                 amp=1.0, bg_sigma=20.0, noise=0.01, speed=(1.0, 4.0),
                 stream=0, n=None, cfg_id=CFG_ID):
        self.H, self.W = int(height), int(width)
        self.n = self.H * self.W if n is None else int(n)
        assert self.n <= self.H * self.W
        self.stream = int(stream)
        self.cfg_id = int(cfg_id)
        self.blob_sigma = float(blob_sigma)
        self.amp = float(amp)
        self.noise = float(noise)
        rng = static_rng(self.cfg_id, stream)
        raw = rng.uniform(0.0, 1.0, (self.H, self.W))
        bg = gaussian_filter(raw, sigma=bg_sigma, mode="wrap")
        bg = (bg - bg.min()) / (bg.max() - bg.min())
        self.bg = bg
        self.pos0 = np.stack([rng.uniform(0, self.H, n_blobs),
                              rng.uniform(0, self.W, n_blobs)], axis=1)
        ang = rng.uniform(0.0, 2 * np.pi, n_blobs)
        spd = rng.uniform(speed[0], speed[1], n_blobs)
        self.vel = np.stack([spd * np.sin(ang), spd * np.cos(ang)], axis=1)

    def _wrapped_profile(self, centre: float, size: int) -> np.ndarray:
        d = np.arange(size, dtype=np.float64) - centre
        d = (d + size / 2.0) % size - size / 2.0
        return np.exp(-d * d / (2.0 * self.blob_sigma ** 2))

    def frame(self, t: int) -> np.ndarray:
        img = self.bg.copy()
        for b in range(self.pos0.shape[0]):
            cy, cx = self.pos0[b] + t * self.vel[b]
            gy = self._wrapped_profile(cy % self.H, self.H)
            gx = self._wrapped_profile(cx % self.W, self.W)
            img += self.amp * np.outer(gy, gx)
        x = img.reshape(-1)[: self.n]
        if self.noise > 0:
            x = x + self.noise * frame_rng(self.cfg_id, self.stream, t).standard_normal(self.n)
        return x.astype(np.float32)

    def frames(self, t0: int, count: int) -> np.ndarray:
        return np.stack([self.frame(t) for t in range(t0, t0 + count)], axis=1)
