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
