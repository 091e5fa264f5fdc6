"""The serving loop end to end on the GPU: frames of several streams arrive
at random times, each loop iteration advances every admitted stream with a
pending frame in one batched tick (with its modes), streams over the HBM
budget wait until others close.  Every stream's results -- served in the mix,
admitted late or not -- must equal the same frames pushed through a stream
of its own, bit for bit (same kernels, same per-stream order), and match
the oracle."""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics

pytestmark = pytest.mark.gpu

# the second stream takes the large slab form of the Gram pass (n >= 2^20)
SPECS = [(6000, 8, 4), (1_100_003, 16, 8), (4000, 24, 10), (12000, 16, 6), (7000, 8, 3), (5000, 12, 5)]


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


# lane_split (8, 12): streams with m <= 8, 8 < m <= 12 and m > 12 tick in three
# lanes (each a batch and a HIP stream of its own) that run side by side
@pytest.mark.parametrize("lane_split", [None, (8, 12)])
def test_served_equals_alone_with_admission_queue(lane_split):
    dmd = _dmd()
    from paper_1612_07875_amd.serve import GPUExecutor, Server, StreamSpec, stream_footprint
    from test_gpu_batch import eig_bound
    T = {sid: m + 6 for sid, (n, m, r) in enumerate(SPECS)}
    host = {sid: np.stack([gen.MixStream(stream=500 + sid, n=n, m=0, r=0, kind="video").frame(t)
                           for t in range(T[sid])]) for sid, (n, m, r) in enumerate(SPECS)}
    frames = {sid: torch.from_numpy(h).cuda() for sid, h in host.items()}
    # footprints (library memory + resident modes, counted before anything
    # is allocated): the budget admits the first four streams only
    foot = []
    for n, m, r in SPECS:
        with dmd.Stream(n, m, r) as s:
            assert dmd.footprint(n, m, r) == int(s.info().device_bytes)
        foot.append(stream_footprint(StreamSpec(n, m, r), True, dmd.footprint))
        assert foot[-1] == dmd.footprint(n, m, r) + 8 * n * r
    budget = sum(foot[:4]) + 1024
    ex = GPUExecutor(frames, hbm_budget=budget, modes=True, lane_split=lane_split)
    assert len({ex._lane_of(StreamSpec(n, m, r)) for n, m, r in SPECS}) == (3 if lane_split else 1)
    srv = Server(ex)
    admitted = [srv.open(sid, StreamSpec(n, m, r)) for sid, (n, m, r) in enumerate(SPECS)]
    assert admitted == [True, True, True, True, False, False]
    rng = np.random.default_rng(3)
    arrivals = sorted((float(rng.uniform(0.0, 0.05)), sid) for sid in range(len(SPECS)) for _ in range(T[sid]))
    srv.run(arrivals)
    results = {}

    def grab(sid):
        s = ex.streams[sid]
        lam, sig, rc = s.eigs()
        results[sid] = (lam, sig, ex.modes[sid].cpu().numpy()[:, :lam.size], s.gram())

    for sid in range(4):
        grab(sid)
    for sid in (4, 5):
        assert sid not in ex.streams                     # still waiting for room
    srv.close(0)
    srv.close(1)                                          # room for the two waiting streams
    assert 4 in ex.streams and 5 in ex.streams
    srv.run([])                                           # their queued frames
    for sid in (4, 5):
        grab(sid)
    ex.shutdown()
    torch.cuda.synchronize()
    for sid, (n, m, r) in enumerate(SPECS):
        with dmd.Stream(n, m, r) as s:
            for t in range(T[sid]):
                s.push(frames[sid][t])
            lam, sig, _ = s.eigs()
            phi = s.modes().cpu().numpy()[:, :lam.size]
            G = s.gram()
        a = results[sid]
        assert np.array_equal(a[0], lam) and np.array_equal(a[1], sig), sid
        assert np.array_equal(a[2], phi), sid
        assert np.array_equal(a[3], G), sid
        W = oracle.as_fp64(host[sid][-(m + 1):].T)
        ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
        err, perm = metrics.eig_relerr(lam, ref.lam)
        bound = eig_bound(ref)[perm]
        assert np.all(err <= bound), (sid, err, bound)
