"""Scheduling logic of the continuous-batching server, on the CPU with a mock
executor (modelled tick durations, admission by a byte budget) and a fake clock."""

import pytest

from paper_1612_07875_amd.serve import Server, StreamSpec


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class MockExecutor:
    def __init__(self, clock, budget, tick_s=1e-3, per_item_s=1e-4):
        self.clock, self.budget = clock, budget
        self.used = 0
        self.open_ids = {}
        self.ticks = []
        self.tick_s, self.per_item_s = tick_s, per_item_s
        self.busy_until = 0.0

    def footprint(self, spec):
        return spec.n * (spec.m + 2) * 4

    def open(self, sid, spec):
        f = self.footprint(spec)
        if self.used + f > self.budget:
            return False
        self.used += f
        self.open_ids[sid] = f
        return True

    def close(self, sid):
        self.used -= self.open_ids.pop(sid)

    def tick(self, items):
        # ticks run back to back on one device queue
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + self.tick_s + self.per_item_s * len(items)
        self.ticks.append(list(items))
        return self.busy_until

    def done(self, h):
        return self.clock() >= h

    def wait(self, h):
        if self.clock.t < h:
            self.clock.t = h


def make(budget=10**9, **kw):
    clock = FakeClock()
    ex = MockExecutor(clock, budget, **kw)
    return Server(ex, clock=clock, sleep=clock.sleep), ex, clock


def test_one_frame_per_stream_per_tick_in_arrival_order():
    srv, ex, clock = make()
    srv.open(0, StreamSpec(1000, 8, 4))
    srv.open(1, StreamSpec(1000, 8, 4))
    st = srv.run([(0.0, 0), (0.0, 0), (0.0, 1), (0.0, 0)])
    assert st.frames == 4
    assert ex.ticks[0] == [(0, 0), (1, 0)]
    assert ex.ticks[1] == [(0, 1)]
    assert ex.ticks[2] == [(0, 2)]


def test_admission_queue_by_budget():
    spec = StreamSpec(1000, 8, 4)
    srv, ex, clock = make(budget=2 * 1000 * 10 * 4)
    assert srv.open(0, spec) and srv.open(1, spec)
    assert not srv.open(2, spec)          # over budget: waits
    assert 2 not in srv.active and srv.refused == 1
    srv.close(0)                          # frees its share
    assert 2 in srv.active and 0 not in srv.active


def test_frames_arriving_during_a_tick_go_to_the_next_tick():
    srv, ex, clock = make(tick_s=5e-3, per_item_s=0.0)
    for sid in range(3):
        srv.open(sid, StreamSpec(100, 4, 2))
    # stream 0 at t=0; streams 1, 2 arrive while that tick runs (t=1 ms, 2 ms)
    st = srv.run([(0.0, 0), (1e-3, 1), (2e-3, 2)])
    assert st.frames == 3
    assert ex.ticks[0] == [(0, 0)]
    assert sorted(sum(ex.ticks[1:], [])) == [(1, 0), (2, 0)]
    assert st.ticks >= 2


def test_latency_accounting_under_light_load():
    srv, ex, clock = make(tick_s=2e-3, per_item_s=0.0)
    srv.open(0, StreamSpec(100, 4, 2))
    arrivals = [(0.01 * k, 0) for k in range(20)]   # far apart: no queueing
    st = srv.run(arrivals)
    assert st.frames == 20
    assert st.p50_ms == pytest.approx(2.0, abs=0.2)
    assert st.p99_ms < 2.5


def test_backlog_raises_latency_but_keeps_order():
    srv, ex, clock = make(tick_s=1e-3, per_item_s=0.0)
    srv.open(0, StreamSpec(100, 4, 2))
    st = srv.run([(0.0, 0)] * 10)                     # burst of 10 frames of one stream
    assert [t[0][1] for t in ex.ticks] == list(range(10))
    assert st.max_ms == pytest.approx(10.0, abs=0.5)  # the last waits for 9 earlier ticks


def test_stream_footprint_counts_library_and_mode_buffers():
    """Admission charges what the library allocates plus the resident modes
    (n x r complex64, complex128 for FP64 projections), before allocating."""
    from paper_1612_07875_amd.serve import stream_footprint
    calls = []

    def lib_bytes(n, m, r, precision="default"):
        calls.append((n, m, r, precision))
        return 1000 * m

    spec = StreamSpec(n=500, m=16, r=8)
    assert stream_footprint(spec, False, lib_bytes) == 16000
    assert stream_footprint(spec, True, lib_bytes) == 16000 + 8 * 500 * 8
    assert stream_footprint(StreamSpec(500, 16, 8, precision="fp64"), True, lib_bytes) == 16000 + 16 * 500 * 8
    assert calls[0] == (500, 16, 8, "default")


class LaneExecutor(MockExecutor):
    """Two device queues: streams with m <= 8 in lane 0, the rest in lane 1,
    whose ticks take `slow_s` (large windows: long single-CU solves)."""

    def __init__(self, clock, budget, slow_s=10e-3, **kw):
        super().__init__(clock, budget, **kw)
        self.specs = {}
        self.busy = [0.0, 0.0]
        self.slow_s = slow_s

    def open(self, sid, spec):
        self.specs[sid] = spec
        return super().open(sid, spec)

    def lane(self, sid):
        return 0 if self.specs[sid].m <= 8 else 1

    def tick(self, items):
        lanes = {self.lane(sid) for sid, _ in items}
        assert len(lanes) == 1, "a tick takes the streams of one lane"
        q = lanes.pop()
        start = max(self.clock(), self.busy[q])
        self.busy[q] = start + (self.tick_s if q == 0 else self.slow_s)
        self.ticks.append(list(items))
        return self.busy[q]


def test_lanes_tick_separately_and_small_windows_do_not_wait():
    clock = FakeClock()
    ex = LaneExecutor(clock, 10**9, tick_s=1e-3, slow_s=10e-3)
    srv = Server(ex, clock=clock, sleep=clock.sleep)
    srv.open(0, StreamSpec(100, 8, 4))      # lane 0
    srv.open(1, StreamSpec(100, 128, 32))   # lane 1
    # both streams get a frame every 2 ms for 20 ms
    arrivals = sorted([(2e-3 * k, 0) for k in range(10)] + [(2e-3 * k, 1) for k in range(10)])
    st = srv.run(arrivals)
    assert st.frames == 20
    # one lane per tick, and each stream's frames in order
    for t in ex.ticks:
        assert len({ex.lane(sid) for sid, _ in t}) == 1
    for sid in (0, 1):
        idx = [i for t in ex.ticks for s, i in t if s == sid]
        assert idx == list(range(10))
    lat0 = [1000 * (r.done - r.arrival) for r in srv.records if r.sid == 0]
    lat1 = [1000 * (r.done - r.arrival) for r in srv.records if r.sid == 1]
    # the small window's frames complete with their own 1 ms ticks, although
    # the large window's lane is backlogged (10 ms ticks every 2 ms)
    assert max(lat0) < 1.5
    assert max(lat1) > 50.0


def test_one_lane_executor_keeps_one_tick_per_step():
    srv, ex, clock = make(tick_s=1e-3, per_item_s=0.0)   # MockExecutor has no lane(): one lane
    srv.open(0, StreamSpec(100, 8, 4))
    srv.open(1, StreamSpec(100, 128, 32))
    srv.run([(0.0, 0), (0.0, 1)])
    assert ex.ticks[0] == [(0, 0), (1, 0)]


def test_one_tick_in_flight_per_lane_batches_the_frames_that_wait():
    clock = FakeClock()
    ex = LaneExecutor(clock, 10**9, tick_s=1e-3, slow_s=10e-3)
    srv = Server(ex, clock=clock, sleep=clock.sleep, max_inflight=1)
    for sid in range(3):
        srv.open(sid, StreamSpec(100, 8, 4))   # lane 0
    srv.open(3, StreamSpec(100, 128, 32))      # lane 1
    st = srv.run([(0.0, 0), (0.0, 3), (2e-4, 1), (4e-4, 2), (5e-4, 3)])
    assert st.frames == 5
    lane0 = [t for t in ex.ticks if ex.lane(t[0][0]) == 0]
    lane1 = [t for t in ex.ticks if ex.lane(t[0][0]) == 1]
    # streams 1 and 2 arrived while stream 0's tick ran: one tick together
    assert lane0 == [[(0, 0)], [(1, 0), (2, 0)]]
    # stream 3's second frame waited for its lane's first tick
    assert lane1 == [[(3, 0)], [(3, 1)]]
    rec = {(r.sid, r.index): r for r in srv.records}
    assert rec[(1, 0)].done == pytest.approx(2e-3, abs=1e-4)     # behind stream 0's tick, not stream 3's
    assert rec[(3, 1)].done == pytest.approx(20e-3, abs=1e-4)
