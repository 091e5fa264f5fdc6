"""Many-stream serving mix: uneven snapshot lengths and windows.

Each stream s draws (from its own static generator)
  n ~ round(exp(U[ln 65536, ln 2097152])),  m ~ U{16, 32, 64, 128},
  r = min(m // 2, 32),
and alternates between blob video (grid width 2^ceil(log2 sqrt n), rows
enough to hold n pixels, truncated to n) and travelling-wave flow (same grid
rule).  Frame arrivals are a Poisson process with the given aggregate rate,
split evenly over streams.
"""

import math
from dataclasses import dataclass, field

import numpy as np

from .common import static_rng
from .video import BlobVideo
from .flow import TravelingWaves

CFG_ID = 5


@dataclass
class MixStream:
    stream: int
    n: int
    m: int
    r: int
    kind: str
    _gen: object = field(default=None, repr=False)

    def generator(self):
        if self._gen is None:
            width = 1 << int(math.ceil(math.log2(math.sqrt(self.n))))
            if self.kind == "video":
                height = -(-self.n // width)
                self._gen = BlobVideo(height=height, width=width, n=self.n,
                                      stream=self.stream, cfg_id=CFG_ID)
            else:
                self._gen = TravelingWaves(n=self.n, stream=self.stream,
                                           cfg_id=CFG_ID, side=width)
        return self._gen

    def frame(self, t: int) -> np.ndarray:
        return self.generator().frame(t)


def stream_mix(count=64, n_range=(65536, 2097152), windows=(16, 32, 64, 128)):
    out = []
    for s in range(count):
        rng = static_rng(CFG_ID, 1000 + s)
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        m = int(windows[int(rng.integers(0, len(windows)))])
        r = min(m // 2, 32)
        kind = "video" if s % 2 == 0 else "flow"
        out.append(MixStream(stream=s, n=n, m=m, r=r, kind=kind))
    return out


def poisson_arrivals(count_streams: int, rate_total: float, duration: float, seed_stream=0):
    """Sorted (time, stream) arrival events of a Poisson process."""
    rng = static_rng(CFG_ID, 10_000 + seed_stream)
    n_events = rng.poisson(rate_total * duration)
    times = np.sort(rng.uniform(0.0, duration, n_events))
    streams = rng.integers(0, count_streams, n_events)
    return times, streams
