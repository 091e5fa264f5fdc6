"""Batched ticks: many streams of uneven n, m, r advanced by one grouped launch
per phase.  Each stream's results in the mix must equal the results of the
same stream advanced alone, bit for bit (same kernels, same per-stream
reduction order), and match the FP64 oracle like any single stream.
"""

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import metrics

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


MIX = [  # (n, m, r, kind)
    (20000, 16, 8, "video"),
    (33333, 32, 16, "flow"),
    (70001, 64, 20, "video"),
    (9000, 128, 24, "flow"),
    (131072, 24, 12, "video"),
    (50000, 33, 10, "flow"),
]


def make_gen(i, n, kind):
    return gen.MixStream(stream=100 + i, n=n, m=0, r=0, kind=kind)


def test_batch_equals_alone_bitwise_and_oracle():
    dmd = _dmd()
    T_extra = 3
    gens = [make_gen(i, n, kind) for i, (n, m, r, kind) in enumerate(MIX)]
    frames = [np.stack([g.frame(t) for t in range(m + 1 + T_extra)], axis=1)
              for g, (n, m, r, kind) in zip(gens, MIX)]
    dev = [torch.from_numpy(F.T.copy()).cuda() for F in frames]

    # alone
    alone = []
    for (n, m, r, kind), X in zip(MIX, dev):
        with dmd.Stream(n, m, r) as s:
            for t in range(X.shape[0]):
                s.push(X[t])
            lam, sig, _ = s.eigs()
            alone.append((s.gram(), lam, sig, s.modes().cpu().numpy()))

    # in the mix: streams joining at different ticks, one tick per frame index
    streams = [dmd.Stream(n, m, r) for (n, m, r, kind) in MIX]
    batch = dmd.Batch(max_streams=16)
    for s in streams:
        batch.attach(s)
    T = max(X.shape[0] for X in dev)
    outs = [torch.zeros((s.r, s.n), dtype=torch.complex64, device="cuda").T for s in streams]
    for t in range(T):
        # stream i starts at tick T - len_i so that all finish together
        act = [i for i, X in enumerate(dev) if t >= T - X.shape[0]]
        batch.tick([streams[i] for i in act], [dev[i][t - (T - dev[i].shape[0])] for i in act],
                   modes=[outs[i] for i in act])
    torch.cuda.synchronize()
    for i, s in enumerate(streams):
        lam, sig, _ = s.eigs()
        G = s.gram()
        phi = outs[i].cpu().numpy()
        a = alone[i]
        assert np.array_equal(G, a[0]), i
        assert np.array_equal(lam, a[1]) and np.array_equal(sig, a[2]), i
        k = lam.size
        assert np.array_equal(phi[:, :k], a[3][:, :k]), i
        # oracle parity of the final window
        n, m, r, kind = MIX[i]
        W = frames[i][:, -(m + 1):]
        ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
        assert k == ref.r_eff
        # the method of snapshots squares the condition number: tolerances
        # grow with (sigma_1 / sigma_k)^2 (the oracle's own MoS and SVD
        # routes differ by that much on the flow streams' weakest waves)
        kap2 = (ref.sigma[0] / ref.sigma[:k]) ** 2
        assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= 1e-11 + 1e-13 * kap2)
        err, perm = metrics.eig_relerr(lam, ref.lam)
        assert err.max() < max(1e-6, 1e-15 * kap2.max()), (i, err.max())
    batch.close()
    for s in streams:
        s.close()


def test_batch_admission_by_hbm_budget():
    dmd = _dmd()
    a = dmd.Stream(100000, 32, 8)
    b = dmd.Stream(100000, 32, 8)
    fa = a.info().device_bytes
    with dmd.Batch(max_streams=4, hbm_budget=int(1.5 * fa)) as batch:
        batch.attach(a)
        with pytest.raises(dmd.DMDError) as ei:
            batch.attach(b)
        assert ei.value.code == dmd.E_NOMEM
        n, used, budget = batch.info()
        assert n == 1 and used == fa
        batch.detach(a)
        batch.attach(b)          # admitted once the other left
        assert batch.info()[0] == 1
    a.close()
    b.close()


def test_batch_rejects_unsupported_members():
    dmd = _dmd()
    with dmd.Batch(max_streams=2) as batch:
        s64 = dmd.Stream(1000, 8, 4, dtype="f64")
        with pytest.raises(dmd.DMDError) as ei:
            batch.attach(s64)
        assert ei.value.code == dmd.E_UNSUPPORTED
        s = dmd.Stream(1000, 8, 4)
        batch.attach(s)
        with pytest.raises(dmd.DMDError):
            batch.attach(s)      # twice
        other = dmd.Stream(1000, 8, 4)
        x = torch.zeros(1000, device="cuda")
        with pytest.raises(dmd.DMDError):
            batch.tick([other], [x])  # not attached
        s64.close()
        s.close()
        other.close()
