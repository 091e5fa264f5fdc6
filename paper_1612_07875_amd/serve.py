"""Continuous-batching request loop over the library's batched tick.

Frames of many streams arrive at arbitrary times.  Each loop iteration takes,
for every admitted stream, its oldest pending frame (one per stream per tick,
in arrival order) and advances all of them with one `dmd_batch_tick`; frames
that arrive while a tick runs wait for the next one.  Streams are admitted
while their device footprint fits the batch's HBM budget; a stream that does
not fit waits in a queue and is admitted when others close.

The scheduling logic is independent of the GPU: it talks to an executor with
three methods, so it can be exercised with a mock executor on the CPU.

    executor.open(sid, spec) -> bool      admit (False: over budget)
    executor.close(sid)
    executor.tick([(sid, frame_index)]) -> handle
    executor.done(handle) -> bool         (non-blocking completion query)
    executor.wait(handle)
"""

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class StreamSpec:
    n: int
    m: int
    r: int
    precision: str = "default"   # projections: "default" (FP32), "bf16x3", ...


@dataclass
class FrameRecord:
    sid: int
    index: int
    arrival: float
    start: Optional[float] = None
    done: Optional[float] = None


@dataclass
class ServeStats:
    frames: int
    elapsed: float
    updates_per_s: float
    p50_ms: float
    p99_ms: float
    max_ms: float
    ticks: int
    mean_batch: float
    admitted: int
    refused_at_first: int
    latencies_ms: List[float] = field(default_factory=list, repr=False)


class Server:
    def __init__(self, executor, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.clock = clock
        self.sleep = sleep
        self.pending: Dict[int, collections.deque] = {}
        self.active = set()
        self.waiting = collections.deque()       # (sid, spec) not yet admitted
        self.specs: Dict[int, StreamSpec] = {}
        self.records: List[FrameRecord] = []
        self.inflight = collections.deque()      # (handle, [FrameRecord])
        self.next_index: Dict[int, int] = {}
        self.ticks = 0
        self.batch_sizes: List[int] = []
        self.refused = 0

    # ------------------------------------------------------------ streams
    def open(self, sid: int, spec: StreamSpec) -> bool:
        self.specs[sid] = spec
        self.pending.setdefault(sid, collections.deque())
        self.next_index.setdefault(sid, 0)
        if not self.waiting and self.ex.open(sid, spec):
            self.active.add(sid)
            return True
        self.refused += 1
        self.waiting.append(sid)
        return False

    def close(self, sid: int) -> None:
        if sid in self.active:
            self._drain()
            self.ex.close(sid)
            self.active.discard(sid)
        self._admit_waiting()

    def _admit_waiting(self) -> None:
        while self.waiting:
            sid = self.waiting[0]
            if not self.ex.open(sid, self.specs[sid]):
                break
            self.waiting.popleft()
            self.active.add(sid)

    # ------------------------------------------------------------ frames
    def arrive(self, sid: int, t: float) -> None:
        rec = FrameRecord(sid=sid, index=self.next_index[sid], arrival=t)
        self.next_index[sid] += 1
        self.pending[sid].append(rec)
        self.records.append(rec)

    def step(self) -> int:
        """Launch one tick over every admitted stream with a pending frame."""
        self._poll()
        batch = [self.pending[sid].popleft() for sid in sorted(self.active) if self.pending[sid]]
        if not batch:
            return 0
        now = self.clock()
        for rec in batch:
            rec.start = now
        handle = self.ex.tick([(rec.sid, rec.index) for rec in batch])
        self.inflight.append((handle, batch))
        self.ticks += 1
        self.batch_sizes.append(len(batch))
        return len(batch)

    def _poll(self) -> None:
        while self.inflight and self.ex.done(self.inflight[0][0]):
            _, recs = self.inflight.popleft()
            now = self.clock()
            for rec in recs:
                rec.done = now

    def _drain(self) -> None:
        while self.inflight:
            handle, recs = self.inflight.popleft()
            self.ex.wait(handle)
            now = self.clock()
            for rec in recs:
                rec.done = now

    # ------------------------------------------------------------ driver
    def run(self, arrivals, t0: Optional[float] = None, idle_sleep: float = 50e-6) -> ServeStats:
        """arrivals: iterable of (time offset in s, sid) sorted by time."""
        arrivals = list(arrivals)
        t0 = self.clock() if t0 is None else t0
        k = 0
        while k < len(arrivals) or any(self.pending[s] for s in self.active) or self.inflight:
            now = self.clock() - t0
            while k < len(arrivals) and arrivals[k][0] <= now:
                self.arrive(arrivals[k][1], t0 + arrivals[k][0])
                k += 1
            launched = self.step()
            if launched == 0:
                self._poll()
                if k < len(arrivals) and not self.inflight:
                    wait = arrivals[k][0] - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 1e-3))
                elif self.inflight:
                    self.sleep(idle_sleep)
        self._drain()
        return self.stats(t0)

    def stats(self, t0: float) -> ServeStats:
        done = [r for r in self.records if r.done is not None]
        lat = np.array([1000.0 * (r.done - r.arrival) for r in done]) if done else np.zeros(1)
        end = max((r.done for r in done), default=t0)
        elapsed = max(end - t0, 1e-9)
        return ServeStats(
            frames=len(done), elapsed=elapsed, updates_per_s=len(done) / elapsed,
            p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
            max_ms=float(lat.max()), ticks=self.ticks,
            mean_batch=float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            admitted=len(self.active), refused_at_first=self.refused, latencies_ms=list(lat))


def stream_footprint(spec: StreamSpec, modes: bool, footprint_fn) -> int:
    """HBM bytes one admitted stream holds: what the library allocates for it
    (footprint_fn(n, m, r, precision=...), nothing allocated) plus, when the
    modes are kept, the executor's resident n x r complex64 mode buffer."""
    lib = int(footprint_fn(spec.n, spec.m, spec.r, precision=spec.precision))
    celem = 16 if spec.precision == "fp64" else 8   # complex128 or complex64 modes
    return lib + (celem * spec.n * spec.r if modes else 0)


class GPUExecutor:
    """Executor backed by libdmdstream: one Stream per sid in one Batch.
    Frame `index` of stream `sid` is read from frames[sid][index % len].
    With modes=True every update also projects the window's DMD modes into a
    resident per-stream buffer (in the stream's precision).  graphs > 0 runs
    each tick as one HIP graph launch (tick shapes cached, see Batch).

    Admission: a stream is admitted while the executor's total footprint
    (library memory plus mode buffers, counted before anything is allocated)
    stays within hbm_budget (0: 90 % of the device memory free at start); a
    stream that does not fit, or whose allocation fails, is refused and waits
    in the server's queue."""

    def __init__(self, frames: Dict[int, "object"], hbm_budget: int = 0, max_streams: int = 1024,
                 modes: bool = False, graphs: int = 0):
        import torch
        from .binding import Batch, DMDError, Stream, E_NOMEM, footprint
        self.torch = torch
        self.Stream = Stream
        self.DMDError = DMDError
        self.E_NOMEM = E_NOMEM
        self.footprint = footprint
        self.frames = frames
        if hbm_budget <= 0:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.used = 0
        self.charged = {}
        # the executor holds the budget (it also counts the mode buffers), so
        # the batch itself admits whatever the executor passes on
        self.batch = Batch(max_streams=max_streams, hbm_budget=1 << 62, graphs=graphs)
        self.streams = {}
        self.want_modes = modes
        self.modes = {}

    def open(self, sid, spec) -> bool:
        need = stream_footprint(spec, self.want_modes, self.footprint)
        if self.used + need > self.budget:
            return False
        try:
            s = self.Stream(spec.n, spec.m, spec.r, precision=spec.precision)
        except self.DMDError as e:
            if e.code == self.E_NOMEM:
                return False
            raise
        try:
            self.batch.attach(s)
            if self.want_modes:
                self.modes[sid] = self.torch.zeros((spec.r, spec.n), dtype=s.mode_dtype, device="cuda").T
        except self.DMDError as e:
            s.close()
            if e.code == self.E_NOMEM:
                return False
            raise
        except self.torch.cuda.OutOfMemoryError:
            self.batch.detach(s)
            s.close()
            return False
        self.streams[sid] = s
        self.used += need
        self.charged[sid] = need
        return True

    def close(self, sid) -> None:
        s = self.streams.pop(sid)
        self.modes.pop(sid, None)
        self.batch.detach(s)
        s.close()
        self.used -= self.charged.pop(sid)

    def tick(self, items):
        ss = [self.streams[sid] for sid, _ in items]
        xs = [self.frames[sid][idx % self.frames[sid].shape[0]] for sid, idx in items]
        if self.want_modes:
            self.batch.tick(ss, xs, modes=[self.modes[sid] for sid, _ in items])
        else:
            self.batch.tick(ss, xs)
        ev = self.torch.cuda.Event()
        ev.record()
        return ev

    def done(self, handle) -> bool:
        return handle.query()

    def wait(self, handle) -> None:
        handle.synchronize()

    def shutdown(self) -> None:
        for sid in list(self.streams):
            self.close(sid)
        self.batch.close()
