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
    (1_500_001, 16, 8, "video"),   # large slab form of the Gram pass, ragged tail
]


def eig_bound(ref):
    """Per-eigenvalue bound on the relative error of lambda_i, in ref's order.

    The method of snapshots works from the FP64 Gram, whose entries carry
    rounding of order u sigma_1^2 (u = 2^-52), and the oracle takes the SVD
    route; metrics.eig_sensitivity gives each eigenvalue's first-order
    sensitivity kappa_i to such a perturbation.  On the CPU the oracle's own
    Gram route (StreamingMoS) and SVD route differ by at most 0.46 u kappa_i
    over these mixes; 32 u kappa_i leaves a margin of 70 for the GPU's
    different summation order."""
    return 1e-13 + 32 * 2.0 ** -52 * metrics.eig_sensitivity(ref)


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
        # grow with (sigma_1 / sigma_k)^2 for sigma_k and with each
        # eigenvalue's own sensitivity for lambda_i
        kap2 = (ref.sigma[0] / ref.sigma[:k]) ** 2
        assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= 1e-11 + 1e-13 * kap2)
        err, perm = metrics.eig_relerr(lam, ref.lam)
        bound = eig_bound(ref)[perm]
        assert np.all(err <= bound), (i, err, bound)
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
        # members solve on every tick; sparse members use the tridiagonal solver
        for kw in ({"auto_solve": False}, {"dtype": "c64_csr", "max_nnz": 16, "eig_solver": "jacobi"}):
            bad = dmd.Stream(1024, 8, 4, **kw)
            with pytest.raises(dmd.DMDError) as ei:
                batch.attach(bad)
            assert ei.value.code == dmd.E_UNSUPPORTED, kw
            bad.close()
        s64 = dmd.Stream(1000, 8, 4, dtype="f64")
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


@pytest.mark.parametrize("graphs", [1, 3, 64])
def test_graph_ticks_equal_eager_ticks(graphs):
    """Ticks replayed as HIP graphs give the eager ticks' results, bit for bit.

    Streams join at different ticks and modes are asked for on some ticks
    only, so several tick shapes occur (with graphs = 1 and 3 the cache
    evicts and recaptures); between replays the program runs eager work of
    its own (a plain stream push, a torch reduction) and synchronizes.
    """
    dmd = _dmd()
    mix = [MIX[0], MIX[1], MIX[4], MIX[5]]
    T = 48
    gens = [make_gen(i, n, kind) for i, (n, m, r, kind) in enumerate(mix)]
    dev = [torch.from_numpy(np.stack([g.frame(t) for t in range(T)], axis=0)).cuda() for g in gens]
    start = [0, 3, 9, 9]

    def run(graph_cache, side):
        streams = [dmd.Stream(n, m, r) for (n, m, r, kind) in mix]
        batch = dmd.Batch(max_streams=8, graphs=graph_cache)
        for s in streams:
            batch.attach(s)
        outs = [torch.zeros((s.r, s.n), dtype=torch.complex64, device="cuda").T for s in streams]
        trace = []
        for t in range(T):
            act = [i for i in range(len(mix)) if t >= start[i]]
            want_modes = t % 3 != 1
            batch.tick([streams[i] for i in act], [dev[i][t - start[i]] for i in act],
                       modes=[outs[i] for i in act] if want_modes else None)
            if side is not None:
                side.push(dev[0][t])
                torch.cuda.synchronize()
                _ = float(dev[1][t].abs().sum())
            torch.cuda.synchronize()
            rec = []
            for i in act:
                s = streams[i]
                G = s.gram()
                try:
                    lam, sig, _ = s.eigs()
                except dmd.DMDError as e:
                    assert e.code == dmd.E_NOT_READY
                    rec.append((G, None, None, None))
                    continue
                phi = outs[i].cpu().numpy()[:, :lam.size] if want_modes else None
                rec.append((G, lam, sig, phi))
            trace.append(rec)
        batch.close()
        for s in streams:
            s.close()
        return trace

    eager = run(0, None)
    with dmd.Stream(*mix[0][:3]) as side:
        graphed = run(graphs, side)
    ready = 0
    for t, (re, rg) in enumerate(zip(eager, graphed)):
        for i, (a, b) in enumerate(zip(re, rg)):
            assert np.array_equal(a[0], b[0]), (t, i)
            if a[1] is None:
                assert b[1] is None, (t, i)
                continue
            ready += 1
            assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), (t, i)
            if a[3] is not None:
                assert np.array_equal(a[3], b[3]), (t, i)
    assert ready > 40


def test_graph_option_checks():
    dmd = _dmd()
    for bad in (-1, 257):
        with pytest.raises(dmd.DMDError) as ei:
            dmd.Batch(max_streams=4, graphs=bad)
        assert ei.value.code == dmd.E_INVAL


# Heterogeneous members (dmd_batch_tick_frames): FP32 streams with FP32 or
# split-BF16 projections share the grouped launches; FP64 streams (FP64 data,
# or FP32 data with FP64 projections) and sparse complex streams (Sec. 3.5)
# run their own Gram / ingest and projection kernels inside the tick; every
# member's small solves are grouped, real and Hermitian windows of both sizes.
HETERO = [  # (kind, n or (side, nnz), m, r, options)
    ("video", 20000, 16, 8, {}),
    ("flow", 33333, 32, 12, {"precision": "bf16x3"}),
    ("video", 50001, 24, 10, {"dtype": "f64"}),
    ("flow", 40000, 64, 16, {"precision": "fp64"}),
    ("video", 9000, 80, 12, {}),                     # real window above 64: solve from global memory
    ("sparse", (64, 80), 16, 6, {}),                 # Hermitian window in LDS
    ("sparse", (48, 61), 40, 8, {}),                 # Hermitian window above 32
]


def _hetero_frames(i, kind, size, m, T):
    """Frames (device) and their FP64 values (host) of member i."""
    if kind == "sparse":
        side, nnz = size
        fs = gen.FourierSparse(side=side, nnz=nnz, redraw=0.05)
        dev, host = [], []
        for t in range(T):
            idx, val = fs.frame(t)
            dev.append((torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda()))
            host.append(oracle.densify(idx, val, fs.n))
        return fs.n, dev, np.stack(host, axis=1)
    g = make_gen(200 + i, size, kind)
    F = np.stack([g.frame(t) for t in range(T)], axis=1).astype(np.float32)
    return size, F, F.astype(np.float64)


def _open(dmd, kind, n, m, r, opts, nnz):
    if kind == "sparse":
        return dmd.Stream(n, m, r, dtype="c64_csr", max_nnz=nnz + 5)
    return dmd.Stream(n, m, r, **opts)


@pytest.mark.parametrize("graphs", [0, 2])
def test_batch_mixed_members_equal_alone_and_oracle(graphs):
    dmd = _dmd()
    T_extra = 3
    members = []
    for i, (kind, size, m, r, opts) in enumerate(HETERO):
        T = m + 1 + T_extra
        n, F, host = _hetero_frames(i, kind, size, m, T)
        if kind == "sparse":
            frames = F
        else:
            elem = torch.float64 if opts.get("dtype") == "f64" else torch.float32
            X = torch.from_numpy(F.T.copy()).to(elem).cuda()
            frames = [X[t] for t in range(T)]
        nnz = size[1] if kind == "sparse" else 0
        members.append((kind, n, m, r, opts, nnz, frames, host))

    def push_one(s, kind, f):
        if kind == "sparse":
            s.push_csr(*f)
        else:
            s.push(f)

    alone = []
    for kind, n, m, r, opts, nnz, frames, host in members:
        with _open(dmd, kind, n, m, r, opts, nnz) as s:
            for f in frames:
                push_one(s, kind, f)
            lam, sig, _ = s.eigs()
            alone.append((s.gram(), lam, sig, s.modes().cpu().numpy()))

    streams = [_open(dmd, kind, n, m, r, opts, nnz) for kind, n, m, r, opts, nnz, frames, host in members]
    batch = dmd.Batch(max_streams=16, graphs=graphs)
    for s in streams:
        batch.attach(s)
    # dmd_batch_tick takes dense members only
    sp = [i for i, mb in enumerate(members) if mb[0] == "sparse"][0]
    with pytest.raises(dmd.DMDError) as ei:
        batch.tick([streams[sp]], [torch.zeros(streams[sp].n, dtype=torch.complex64, device="cuda")])
    assert ei.value.code == dmd.E_INVAL
    T = max(len(mb[6]) for mb in members)
    outs = [torch.zeros((s.r, s.n), dtype=s.mode_dtype, device="cuda").T for s in streams]
    for t in range(T):
        act = [i for i, mb in enumerate(members) if t >= T - len(mb[6])]
        batch.tick_frames([streams[i] for i in act], [members[i][6][t - (T - len(members[i][6]))] for i in act],
                          modes=[outs[i] for i in act])
    torch.cuda.synchronize()
    for i, s in enumerate(streams):
        kind, n, m, r, opts, nnz, frames, host = members[i]
        lam, sig, _ = s.eigs()
        G = s.gram()
        phi = outs[i].cpu().numpy()
        a = alone[i]
        assert np.array_equal(G, a[0]), i
        assert np.array_equal(lam, a[1]) and np.array_equal(sig, a[2]), i
        k = lam.size
        assert np.array_equal(phi[:, :k], a[3][:, :k]), i
        W = host[:, -(m + 1):]
        ref = oracle.exact_dmd(W[:, :m], W[:, 1:], r)
        assert k == ref.r_eff, i
        kap2 = (ref.sigma[0] / ref.sigma[:k]) ** 2
        assert np.all(metrics.sigma_relerr(sig, ref.sigma[:k]) <= 1e-11 + 1e-13 * kap2), i
        err, perm = metrics.eig_relerr(lam, ref.lam)
        bound = eig_bound(ref)[perm]
        assert np.all(err <= bound), (i, err, bound)
    batch.close()
    for s in streams:
        s.close()
