"""Continuous-batching request loop over the library's batched tick.

Frames of many streams arrive at arbitrary times.  Each loop iteration takes,
for every admitted stream, its oldest pending frame (one per stream per tick,
in arrival order) and advances all of them with one `dmd_batch_tick`; frames
that arrive while a tick runs wait for the next one.  Streams are admitted
while their device footprint fits the batch's HBM budget; a stream that does
not fit waits in a queue and is admitted when others close.

Lanes: an executor may put streams into lanes (executor.lane(sid)), whose
ticks run on device queues of their own.  A loop iteration then launches one
tick per lane with pending frames, and a tick completes on its own: streams
whose small solves are short (small windows) do not wait behind the ticks of
streams with large windows.  A stream stays in one lane, so its frames are
still processed in arrival order.

The scheduling logic is independent of the GPU: it talks to an executor with
these methods, so it can be exercised with a mock executor on the CPU.

    executor.open(sid, spec) -> bool      admit (False: over budget)
    executor.close(sid)
    executor.tick([(sid, frame_index)]) -> handle   (one lane's streams)
    executor.done(handle) -> bool         (non-blocking completion query)
    executor.wait(handle)
    executor.lane(sid) -> int             (optional; no method: one lane)
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
    """max_inflight: ticks a lane may have on the device at once.  1 (the
    default): the frames that arrive while a lane's tick runs wait for it and
    go into that lane's next tick together.  None: no limit, every loop
    iteration launches a tick for each lane with pending frames, queued on
    the device behind the running ones (measured on the 64-stream mix: p50
    4.7 ms against 1.5 ms with one tick in flight)."""

    def __init__(self, executor, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, max_inflight: Optional[int] = 1):
        self.ex = executor
        self.max_inflight = max_inflight
        self.clock = clock
        self.sleep = sleep
        self.pending: Dict[int, collections.deque] = {}
        self.active = set()
        self.waiting = collections.deque()       # (sid, spec) not yet admitted
        self.specs: Dict[int, StreamSpec] = {}
        self.records: List[FrameRecord] = []
        self.inflight = collections.deque()      # (handle, [FrameRecord], lane)
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
        """Launch one tick per lane over every admitted stream with a pending
        frame."""
        self._poll()
        lane_of = getattr(self.ex, "lane", None)
        busy = collections.Counter(lane for _, _, lane in self.inflight)
        lanes: Dict[int, List[FrameRecord]] = collections.OrderedDict()
        for sid in sorted(self.active):
            if not self.pending[sid]:
                continue
            lane = lane_of(sid) if lane_of else 0
            if self.max_inflight is not None and busy[lane] >= self.max_inflight:
                continue
            lanes.setdefault(lane, []).append(self.pending[sid].popleft())
        if not lanes:
            return 0
        now = self.clock()
        total = 0
        for lane, recs in lanes.items():
            for rec in recs:
                rec.start = now
            handle = self.ex.tick([(rec.sid, rec.index) for rec in recs])
            self.inflight.append((handle, recs, lane))
            self.ticks += 1
            self.batch_sizes.append(len(recs))
            total += len(recs)
        return total

    def _poll(self) -> None:
        # ticks of different lanes complete in any order
        if not self.inflight:
            return
        now = None
        keep = collections.deque()
        for entry in self.inflight:
            handle, recs, _ = entry
            if self.ex.done(handle):
                now = self.clock() if now is None else now
                for rec in recs:
                    rec.done = now
            else:
                keep.append(entry)
        self.inflight = keep

    def _drain(self) -> None:
        while self.inflight:
            handle, recs, _ = self.inflight.popleft()
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
    """Executor backed by libdmdstream: one Stream per sid, in the Batch of its
    lane.  Frame `index` of stream `sid` is read from frames[sid][index % len].
    With modes=True every update also projects the window's DMD modes into a
    resident per-stream buffer (in the stream's precision).  graphs > 0 runs
    each tick as one HIP graph launch (tick shapes cached, see Batch).

    Lanes: lane_split = (m0, m1, ...) increasing puts a stream with m <= m0 in
    lane 0, m0 < m <= m1 in lane 1, ..., and the rest in the last lane, each
    lane with a Batch and a HIP stream (default priority) of its own, so that
    the ticks of small windows run beside those of large ones instead of
    behind them (a tick lasts as long as its slowest member's single-CU
    solves).  An int is one threshold; None: one lane.

    Admission: a stream is admitted while the executor's total footprint
    (library memory plus mode buffers, counted before anything is allocated)
    stays within hbm_budget (0: 90 % of the device memory free at start); a
    stream that does not fit, or whose allocation fails, is refused and waits
    in the server's queue."""

    def __init__(self, frames: Dict[int, "object"], hbm_budget: int = 0, max_streams: int = 1024,
                 modes: bool = False, graphs: int = 0, lane_split=(32, 64)):
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
        # the batches themselves admit whatever the executor passes on
        if lane_split is None:
            lane_split = ()
        elif isinstance(lane_split, int):
            lane_split = (lane_split,)
        self.lane_split = tuple(sorted(lane_split))
        nlanes = len(self.lane_split) + 1
        self.batches = [Batch(max_streams=max_streams, hbm_budget=1 << 62, graphs=graphs) for _ in range(nlanes)]
        self.queues = [torch.cuda.Stream() for _ in range(nlanes)]
        self.lanes = {}
        self.streams = {}
        self.want_modes = modes
        self.modes = {}

    def lane(self, sid) -> int:
        return self.lanes[sid]

    def _lane_of(self, spec) -> int:
        return sum(1 for m0 in self.lane_split if spec.m > m0)

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
        lane = self._lane_of(spec)
        batch = self.batches[lane]
        try:
            batch.attach(s)
            if self.want_modes:
                self.modes[sid] = self.torch.zeros((spec.r, spec.n), dtype=s.mode_dtype, device="cuda").T
        except self.DMDError as e:
            s.close()
            if e.code == self.E_NOMEM:
                return False
            raise
        except self.torch.cuda.OutOfMemoryError:
            batch.detach(s)
            s.close()
            return False
        # the lane's queue runs after what the program enqueued so far (the
        # frames and the zeroed mode buffer)
        self.queues[lane].wait_stream(self.torch.cuda.current_stream())
        self.streams[sid] = s
        self.lanes[sid] = lane
        self.used += need
        self.charged[sid] = need
        return True

    def close(self, sid) -> None:
        # (the server drains every tick before it closes a stream)
        s = self.streams.pop(sid)
        self.modes.pop(sid, None)
        self.batches[self.lanes.pop(sid)].detach(s)
        s.close()
        self.used -= self.charged.pop(sid)

    def tick(self, items):
        lane = self.lanes[items[0][0]]
        if any(self.lanes[sid] != lane for sid, _ in items):
            raise ValueError("a tick takes the streams of one lane")
        ss = [self.streams[sid] for sid, _ in items]
        xs = [self.frames[sid][idx % self.frames[sid].shape[0]] for sid, idx in items]
        q = self.queues[lane]
        if self.want_modes:
            self.batches[lane].tick(ss, xs, modes=[self.modes[sid] for sid, _ in items], stream=q)
        else:
            self.batches[lane].tick(ss, xs, stream=q)
        ev = self.torch.cuda.Event()
        ev.record(q)
        return ev

    def done(self, handle) -> bool:
        return handle.query()

    def wait(self, handle) -> None:
        handle.synchronize()

    def shutdown(self) -> None:
        for q in self.queues:
            q.synchronize()
        for sid in list(self.streams):
            self.close(sid)
        for b in self.batches:
            b.close()
