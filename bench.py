#!/usr/bin/env python3
"""Streaming-DMD window updates on one MI355X.

Workload: synthetic blob video, 1920 x 1080 greyscale FP32 frames
(n = 2,073,600), window m = 64, truncation rank r = 20.  Frames are generated
on the host and copied to HBM before timing.

Every window update runs the whole hot path through the C ABI:
  ingest + Gram -- the new frame(s) and their inner products with the window
                   (FP64 accumulation), Gram update;
  solve         -- FP64 Jacobi eig of X^* X, sigma, A~, Hessenberg-QR eig of
                   A~, projection coefficients (all on the GPU);
  modes         -- Phi = X' V Sigma^-1 W (n x r complex64) into a resident buffer.

--mode block (default): one step = one push of k frames (multi-column update,
  Sec. 5) whose k windows are all solved (side by side) and projected; the
  value counts k window updates per step.
--mode single: one step = one frame.
--mode modal: plain streaming DMD in FP64: n = 4096 real snapshots of five
  damped modes plus noise, m = 32, r = 10, 64 frames (32 windows); the 64
  frames are streamed again after a reset until >= 1,000 window updates are
  timed; one step = one push + FP64 solves + FP64 modes; per-frame latency
  p50/p99 over the same updates.
--mode waves: the precision-study workload: n = 2^20 travelling waves, m = 256,
  r = 32, FP32 data (and a second leg with the same values as FP64 data);
  one step = one push + FP64 solves + modes; also the whole-window Gram
  (Algorithm 1's first step, 257 columns) timed in FP64, FP32 and split-BF16
  MFMA products against the matrix-core roofline of each.
--mode sparse: the sparse (Fourier-coefficient) configuration: 512 x 512
  complex64 coefficients at 1 % (2,621 per frame, lowest wavenumbers, 5 %
  redrawn per frame), m = 128, r = 24; one step = one sparse push + solves +
  modes.  A second leg pushes 512 x 512 spatial frames through the device
  Fourier ingest (same support size) and is reported under "fourier_ingest";
  a third advances --sparse-streams such streams by one batch tick per step
  and is reported under "batched".

Prints one JSON line (see the repository's benchmark contract).
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix, published
BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix, published

H, W, M, R = 1080, 1920, 64, 20
COPY_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=("block", "single", "sparse", "modal", "waves"), default="block",
                    help="block: k frames per step (multi-column update, every window solved and projected); "
                         "single: one frame per step")
    ap.add_argument("--block", type=int, default=32, help="frames per block in block mode (1..64)")
    ap.add_argument("--rank", type=int, default=R, help="truncation rank r (the workload's is 20)")
    ap.add_argument("--precision", choices=("fp32", "bf16x3"), default="fp32",
                    help="arithmetic of the mode projections: FP32 MFMA, or three BF16 MFMA products "
                         "(hi*hi + hi*lo + lo*hi) with FP32 accumulation")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20 blocks / 100 frames)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 2 blocks / 10 frames)")
    ap.add_argument("--latency-frames", type=int, default=400, help="single-frame pushes timed one by one")
    ap.add_argument("--latency-blocks", type=int, default=20, help="block mode: blocks timed one by one")
    ap.add_argument("--cpu-windows", type=int, default=4, help="windows in the oracle's timed sample")
    ap.add_argument("--sparse-streams", type=int, default=16,
                    help="sparse mode: streams in the batched leg (0: no batched leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="block mode, FP32: skip the comparison run with split-BF16 projections")
    ap.add_argument("--serve", action="store_true",
                    help="run the 64-stream serving mix (Poisson arrivals) instead of the single-stream workload")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="aggregate frames/s")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB (5 times) and print its bandwidth: the "
                         "calibration kernel for the HBM byte counters")
    return ap.parse_args()


def copy_probe():
    """A plain copy of COPY_BYTES (read COPY_BYTES, write COPY_BYTES) per launch."""
    import torch
    torch.cuda.set_device(0)
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(5):
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    best = min(times)
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 6,
                      "best_us": round(best * 1e6, 1),
                      "copy_GBps": round(2 * COPY_BYTES / best / 1e9, 1)}), flush=True)


def defaults(args):
    if args.steps is None:
        args.steps = {"block": 20, "modal": 1024, "waves": 60}.get(args.mode, 100)
    if args.warmup is None:
        args.warmup = {"block": 2, "modal": 32}.get(args.mode, 10)
    if not 1 <= args.block <= 64:
        raise SystemExit("--block must be in [1, 64]")
    return args


def kernel_source_hash(name: str) -> str:
    path = os.path.join(ROOT, "paper_1612_07875_amd", "csrc", name)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel: str, source: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(kernel)
    if not rec or rec.get("source_sha256_16") != kernel_source_hash(source):
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """BLAS threads the oracle uses, the host's logical CPU count and CPU model."""
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count() or 1
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return int(threads), int(os.cpu_count() or 1), model


def cpu_baseline(frames_host, windows: int, m=None, r=None, n=None):
    """The FP64 oracle (exact DMD by LAPACK SVD, with modes) on a bounded
    sample: the paper's non-streaming CPU baseline (Sec. 4, "CPU")."""
    import numpy as np
    import oracle

    m = M if m is None else m
    r = R if r is None else r
    n = frames_host.shape[1] if n is None else n
    threads, nproc, model = host_cpu()
    t0 = time.perf_counter()
    for w in range(windows):
        F = frames_host[w:w + m + 1]
        X = np.ascontiguousarray(F[:m].T)
        Xp = np.ascontiguousarray(F[1:].T)
        oracle.exact_dmd(X, Xp, r)
    dt = time.perf_counter() - t0
    return {
        "value": windows / dt,
        "unit": "window updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{windows} windows of the same workload (n={n}, m={m}, r={r}); "
                  f"FP64 exact DMD by LAPACK thin SVD with modes; {dt:.1f} s",
        "nproc": nproc, "cpu_model": model,
    }


def cpu_baseline_streaming(frames_host, frames: int, m=None, r=None, n=None):
    """The oracle's streaming method of snapshots in FP64 (Algorithms 1-2: one
    new Gram column per frame, eigh, A~, eig, modes): the paper's streaming
    CPU baseline (Sec. 4, "SCPU"), timed per frame after its window fills."""
    import oracle

    m = M if m is None else m
    r = R if r is None else r
    n = frames_host.shape[1] if n is None else n
    threads, nproc, model = host_cpu()
    s = oracle.StreamingMoS(m, r)
    for t in range(m + 1):
        s.push(frames_host[t])
    s.dmd()
    t0 = time.perf_counter()
    for t in range(m + 1, m + 1 + frames):
        s.push(frames_host[t])
        s.dmd()
    dt = time.perf_counter() - t0
    return {
        "value": frames / dt,
        "unit": "window updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{frames} streamed frames of the same workload (n={n}, m={m}, r={r}) after the window "
                  f"filled; FP64 streaming method of snapshots (new Gram column, eigh, A~, eig, modes); {dt:.1f} s",
        "nproc": nproc, "cpu_model": model,
    }


def serve_bench(args):
    """Many streams of uneven n and m behind the continuous-batching server."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import gen
    from gen.mix import poisson_arrivals
    from paper_1612_07875_amd.serve import GPUExecutor, Server, StreamSpec

    torch.cuda.set_device(0)
    mix = gen.stream_mix(args.serve_streams)
    t_gen = time.perf_counter()

    def pool(s):
        P = s.m + 9  # window fill plus a few frames; later frames cycle through the pool
        return np.stack([s.frame(t) for t in range(P)])

    with ThreadPoolExecutor(max_workers=16) as ex:
        host = list(ex.map(pool, mix))
    frames = {s.stream: torch.from_numpy(h).cuda() for s, h in zip(mix, host)}
    del host
    torch.cuda.synchronize()
    print(f"[serve] generated frame pools for {len(mix)} streams in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    times, sids = poisson_arrivals(len(mix), args.serve_rate, args.serve_seconds)
    arrivals = [(float(t), mix[int(k)].stream) for t, k in zip(times, sids)]

    def serving(lane_split, max_inflight=1):
        ex_gpu = GPUExecutor(frames, lane_split=lane_split)
        srv = Server(ex_gpu, max_inflight=max_inflight)
        for s in mix:
            srv.open(s.stream, StreamSpec(s.n, s.m, s.r))
        # fill every window (backlogged burst), untimed
        srv.run(sorted((0.0, s.stream) for s in mix for _ in range(s.m + 1)))
        srv.records.clear()
        srv.batch_sizes.clear()
        srv.ticks = 0
        # Poisson arrivals at the target rate
        st = srv.run(arrivals)
        print(f"[serve] lanes split at m = {lane_split}, ticks in flight per lane {max_inflight}: poisson run, "
              f"{st.frames} frames in {st.elapsed:.1f} s, p50 {st.p50_ms:.2f} ms, p99 {st.p99_ms:.2f} ms, "
              f"mean batch {st.mean_batch:.2f}", file=sys.stderr, flush=True)
        # saturation: every stream backlogged
        srv.records.clear()
        srv.batch_sizes.clear()
        srv.ticks = 0
        sat = srv.run(sorted((0.0, s.stream) for s in mix for _ in range(8)))
        ex_gpu.shutdown()
        torch.cuda.synchronize()
        return st, sat

    print("[serve] frames resident", file=sys.stderr, flush=True)
    st, sat = serving((32, 64), 1)
    st3, sat3 = serving((32, 64), None)
    st2, sat2 = serving(64, None)
    st1, sat1 = serving(None, None)
    modes_cmp = None if args.no_split else modes_saturation(mix, frames, GPUExecutor, Server, StreamSpec)
    footprint = sum((s.m + 2) * s.n * 4 for s in mix)
    out = {
        "metric": "DMD window updates/s + Gram HBM GB/s vs roofline; p99 frame latency",
        "value": round(st.updates_per_s, 2),
        "unit": "window updates/s",
        "n_gpus": 1, "steps": st.frames, "warmup": sum(s.m + 1 for s in mix),
        "ms_per_step": round(1000.0 * st.elapsed / max(st.frames, 1), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving mix: {len(mix)} streams, n log-uniform in [65536, 2097152], "
                               f"m in {{16,32,64,128}}, r = min(m/2, 32), blob video / travelling waves; "
                               f"Poisson arrivals {args.serve_rate:.0f} frames/s for {args.serve_seconds:.0f} s; "
                               f"each update = Gram column + FP64 solves (no modes; modes_saturation "
                               f"adds them); three lanes (m <= 32, m = 64, m = 128), each with its own "
                               f"batch and HIP stream, one tick in flight per lane",
                   "streams": len(mix), "ring_bytes": footprint},
        "latency_ms": {"p50": round(st.p50_ms, 3), "p99": round(st.p99_ms, 3), "max": round(st.max_ms, 3)},
        "mean_batch": round(st.mean_batch, 2), "ticks": st.ticks,
        "saturation": {"updates_per_s": round(sat.updates_per_s, 1), "frames": sat.frames,
                       "mean_batch": round(sat.mean_batch, 2), "p99_ms": round(sat.p99_ms, 2)},
        "three_lanes_unlimited": {"note": "the same arrivals and lanes, with no limit on the ticks in flight",
                                  "updates_per_s": round(st3.updates_per_s, 2),
                                  "latency_ms": {"p50": round(st3.p50_ms, 3), "p99": round(st3.p99_ms, 3),
                                                 "max": round(st3.max_ms, 3)},
                                  "mean_batch": round(st3.mean_batch, 2),
                                  "saturation_updates_per_s": round(sat3.updates_per_s, 1)},
        "two_lanes": {"note": "the same arrivals in two lanes (m <= 64, m = 128), no limit on the ticks in flight",
                      "updates_per_s": round(st2.updates_per_s, 2),
                      "latency_ms": {"p50": round(st2.p50_ms, 3), "p99": round(st2.p99_ms, 3),
                                     "max": round(st2.max_ms, 3)},
                      "mean_batch": round(st2.mean_batch, 2),
                      "saturation_updates_per_s": round(sat2.updates_per_s, 1)},
        "one_lane": {"note": "the same arrivals with every stream in one batch on one HIP stream, no limit "
                             "on the ticks in flight",
                     "updates_per_s": round(st1.updates_per_s, 2),
                     "latency_ms": {"p50": round(st1.p50_ms, 3), "p99": round(st1.p99_ms, 3),
                                    "max": round(st1.max_ms, 3)},
                     "mean_batch": round(st1.mean_batch, 2),
                     "saturation_updates_per_s": round(sat1.updates_per_s, 1)},
    }
    if modes_cmp is not None:
        out["modes_saturation"] = modes_cmp
    print(json.dumps(out), flush=True)


def modes_saturation(mix, frames, GPUExecutor, Server, StreamSpec, sat_frames=6):
    """Every stream backlogged, every update with its modes: plain per-stream
    FP32 (one stream after another, no batching) against batched ticks with
    FP32 and with split-BF16 projections."""
    import torch

    import paper_1612_07875_amd as dmd

    res = {}
    # plain per-stream FP32: each stream on its own, push + modes per frame
    streams = {s.stream: dmd.Stream(s.n, s.m, s.r) for s in mix}
    outs = {s.stream: torch.zeros((s.r, s.n), dtype=torch.complex64, device="cuda").T for s in mix}
    for s in mix:
        X = frames[s.stream]
        for t in range(s.m + 1):
            streams[s.stream].push(X[t % X.shape[0]])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(sat_frames):
        for s in mix:
            X = frames[s.stream]
            h = streams[s.stream]
            h.push(X[(s.m + 1 + f) % X.shape[0]])
            h.modes(outs[s.stream])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["per_stream_fp32"] = round(sat_frames * len(mix) / el, 1)
    for h in streams.values():
        h.close()
    del outs
    torch.cuda.synchronize()
    for prec, key, graphs in (("default", "batched_fp32", 0), ("default", "batched_fp32_graph", 8),
                              ("bf16x3", "batched_bf16x3", 0)):
        ex = GPUExecutor(frames, modes=True, graphs=graphs)
        srv = Server(ex)
        for s in mix:
            srv.open(s.stream, StreamSpec(s.n, s.m, s.r, precision=prec))
        srv.run(sorted((0.0, s.stream) for s in mix for _ in range(s.m + 1)))
        srv.records.clear()
        srv.batch_sizes.clear()
        srv.ticks = 0
        st = srv.run(sorted((0.0, s.stream) for s in mix for _ in range(sat_frames)))
        res[key] = round(st.updates_per_s, 1)
        ex.shutdown()
        torch.cuda.synchronize()
    print(f"[serve] modes at saturation: {res}", file=sys.stderr, flush=True)
    res["note"] = ("every stream backlogged, each update with its DMD modes; per_stream_fp32 runs the "
                   "streams one after another without batching; _graph replays each tick as one HIP graph")
    return res


def make_frames(T, keep):
    """T frames of the blob video on the device (generated on the host in
    parallel, outside any timed region); the first `keep` also kept on the host."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import gen

    n = H * W
    video = gen.BlobVideo(height=H, width=W)
    frames = torch.empty((T, n), dtype=torch.float32, device="cuda")
    host_keep = []
    t_gen = time.perf_counter()
    with ThreadPoolExecutor(max_workers=16) as ex:
        for t0 in range(0, T, 64):
            chunk = list(ex.map(video.frame, range(t0, min(T, t0 + 64))))
            for i, f in enumerate(chunk):
                frames[t0 + i].copy_(torch.from_numpy(f))
                if t0 + i < keep:
                    host_keep.append(f)
    torch.cuda.synchronize()
    print(f"[bench] generated {T} frames in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    return frames, host_keep


def kernel_table(dmd, names):
    out = {}
    for name in names:
        cnt, ms = dmd.profile_read(name)
        if cnt:
            out[name] = {"launches": cnt, "avg_us": 1000.0 * ms / cnt}
    return out


def roofline_of(kernels, bytes_per, source_of, mfma=None, traffic_key=None):
    """Roofline of the dominant kernel (longest average launch) among those
    with algorithmic bytes: bound by HBM or, where `mfma` gives its matrix-core
    work (flops per launch, the peak of its dtype), by whichever roof needs
    more time."""
    mfma = mfma or {}
    dom = max(bytes_per, key=lambda k: kernels.get(k, {}).get("avg_us", 0.0))
    avg_s = kernels[dom]["avg_us"] * 1e-6
    for k in bytes_per:
        if k in kernels:
            kernels[k]["algorithmic_bytes"] = bytes_per[k]
            kernels[k]["algorithmic_GBps"] = round(bytes_per[k] / (kernels[k]["avg_us"] * 1e-6) / 1e9, 1)
            if k in mfma:
                kernels[k]["mfma_flops"] = mfma[k][0]
                kernels[k]["mfma_TFLOPs"] = round(mfma[k][0] / (kernels[k]["avg_us"] * 1e-6) / 1e12, 2)
    t_hbm = bytes_per[dom] / (HBM_PEAK_GBS * 1e9)
    out = {"kernel": dom, "algorithmic_bytes_per_launch": bytes_per[dom],
           "avg_launch_us": round(kernels[dom]["avg_us"], 2),
           "floors_us": {"hbm": round(t_hbm * 1e6, 1)}}
    if dom in mfma:
        flops, peak_tf, kind = mfma[dom]
        t_mfma = flops / (peak_tf * 1e12)
        out["floors_us"]["mfma"] = round(t_mfma * 1e6, 1)
        out["mfma_work"] = kind
        if t_mfma > t_hbm:
            achieved = flops / avg_s / 1e12
            out.update({"bound": "mfma", "achieved": round(achieved, 2), "peak": peak_tf, "unit": "TFLOP/s",
                        "frac": round(achieved / peak_tf, 4),
                        "traffic": traffic_for((traffic_key or {}).get(dom, dom), source_of[dom])})
            return out
    achieved = bytes_per[dom] / avg_s / 1e9
    out.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for((traffic_key or {}).get(dom, dom), source_of[dom])})
    return out


LAT_WARM = 3  # untimed single frames before the latency frames


def single_latency(s, frames, t, L, phi, dmd):
    """Push -> modes latency of L single frames on one stream (nothing else
    running), after LAT_WARM untimed ones, and the per-kernel times of those
    L frames."""
    import numpy as np
    import torch
    if L > 0:
        for _ in range(LAT_WARM):
            s.push(frames[t])
            s.modes(phi)
            t += 1
        torch.cuda.synchronize()
    lat = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dmd.profile_enable(True)
    dmd.profile_reset()
    for _ in range(L):
        e0.record()
        s.push(frames[t])
        s.modes(phi)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
        t += 1
    dmd.profile_enable(False)
    kern = kernel_table(dmd, ("gram_columns", "project_modes", "solve_sym", "solve_eig"))
    dmd.profile_reset()
    if not lat:
        return None, t, kern
    lat = np.array(lat)
    return {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
            "frames": int(L)}, t, kern


def gram_alone_line(kern, n, kb):
    """HBM rate of the streaming Gram updates timed with nothing beside them
    (the latency runs): one frame ((m+2) n 4 bytes) and, in block mode, one
    block of kb frames ((m+1+2kb) n 4 bytes)."""
    out = {}
    sizes = [("gram_columns", (M + 2) * n * 4)]
    if kb is not None:
        sizes.append(("gram_block", (M + 1 + 2 * kb) * n * 4))
    for name, nbytes in sizes:
        if name in kern:
            us = kern[name]["avg_us"]
            gbs = nbytes / (us * 1e-6) / 1e9
            out[name] = {"avg_us": round(us, 2), "algorithmic_GBps": round(gbs, 1),
                         "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def bench_single(args):
    """One frame per step: push + FP64 solves + modes of that window."""
    import numpy as np
    import torch

    import paper_1612_07875_amd as dmd

    n = H * W
    K, Wu, L = args.steps, args.warmup, args.latency_frames
    T = M + 1 + Wu + K + L + LAT_WARM
    keep = M + 1 + (args.cpu_windows if not args.no_cpu_baseline else 0)
    frames, host_keep = make_frames(T, keep)

    s = dmd.Stream(n, M, R, dtype="f32", precision=args.precision)
    phi = torch.zeros((R, n), dtype=torch.complex64, device="cuda").T
    # pushes on one stream, modes on another: the modes of frame t run beside
    # the push of frame t + 1 (its Gram update and solves)
    sp, sm = bench_streams(torch)
    sp.wait_stream(torch.cuda.current_stream())
    sm.wait_stream(torch.cuda.current_stream())
    for t in range(M + 1):
        s.push(frames[t], stream=sp)
    t = M + 1
    for _ in range(Wu):
        s.push(frames[t], stream=sp)
        s.modes(phi, stream=sm)
        t += 1
    torch.cuda.synchronize()

    dmd.profile_enable(True)
    dmd.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        s.push(frames[t], stream=sp)
        s.modes(phi, stream=sm)
        t += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dmd.profile_enable(False)
    kernels = kernel_table(dmd, ("gram_columns", "gram_finalize", "solve_sym", "solve_eig", "project_modes"))
    dmd.profile_reset()
    print(f"[bench] timed {K} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    latency, t, alone = single_latency(s, frames, t, L, phi, dmd)
    gram_alone = gram_alone_line(alone, n, None)
    lam, sig, rc = s.eigs()
    r_eff = lam.size
    info = s.info()
    s.close()
    roofline = roofline_of(
        kernels,
        {"gram_columns": (M + 2) * n * 4,             # read m kept columns + new frame, write the frame
         "project_modes": M * n * 4 + n * r_eff * 8},  # read X', write Phi (complex64)
        {"gram_columns": "gram_push.hip", "project_modes": "project.hip"},
        {"project_modes": ((3.0 if args.precision == "bf16x3" else 1.0) * 2.0 * n * M * 2 * r_eff,
                           BF16_MFMA_TFLOPS if args.precision == "bf16x3" else FP32_MFMA_TFLOPS, args.precision)})
    out = result_line(K / elapsed, K, Wu, elapsed, "f32", {
        "workload": "blob video 1920x1080 FP32 (n=2073600), m=64, r=20; single-frame mode: "
                    "step = push of one frame + FP64 solves + modes of its window (the modes of "
                    "frame t run beside the push of frame t+1)",
        "n": n, "m": M, "r": R, "r_eff": int(r_eff), "frames_per_step": 1,
        "precision": precision_note(args)})
    out.update({"roofline": roofline, "kernels": kernels,
                "gram_GBps": kernels.get("gram_columns", {}).get("algorithmic_GBps"), "gram_alone": gram_alone,
                "latency_ms": latency, "jacobi_sweeps": int(info.sweeps), "qr_iters": int(info.qr_iters)})
    return out, host_keep


_STREAMS = None


def bench_streams(torch):
    """The push and projection streams, created once: every timed leg runs on
    the same pair of HIP streams (and so the same hardware queues)."""
    global _STREAMS
    if _STREAMS is None:
        _STREAMS = (torch.cuda.Stream(), torch.cuda.Stream())
    return _STREAMS


def timed_blocks(dmd, torch, frames, n, kb, K, Wu, precision):
    """Fill a window with block pushes, then Wu untimed and K timed steps of
    one block push + the modes of all its windows.  Pushes (Gram update +
    solves) go on one stream and projections on another, so the projection of
    block b overlaps the Gram update and solves of block b + 1."""
    fill = M + 1
    s = dmd.Stream(n, M, R, dtype="f32", max_block=kb, precision=precision)
    phis = torch.zeros((kb, R, n), dtype=torch.complex64, device="cuda")
    sp, sm = bench_streams(torch)
    sp.wait_stream(torch.cuda.current_stream())
    sm.wait_stream(torch.cuda.current_stream())
    t = 0
    while t < fill:                      # the window fills with block pushes as well
        k = min(kb, fill - t)
        s.push_block(frames[t:t + k], stream=sp)
        t += k
    for _ in range(Wu):
        s.push_block(frames[t:t + kb], stream=sp)
        s.block_modes(phis, stream=sm)
        t += kb
    torch.cuda.synchronize()

    dmd.profile_enable(True)
    dmd.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        s.push_block(frames[t:t + kb], stream=sp)
        s.block_modes(phis, stream=sm)
        t += kb
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dmd.profile_enable(False)
    kernels = kernel_table(dmd, ("gram_block", "block_solve", "pack_block", "project_block"))
    dmd.profile_reset()
    wins, _ = s.block_eigs()
    bad = [w for w in wins if w[0] not in (0, 1)]
    if bad:
        raise RuntimeError(f"a window of the last block was not solved: status {bad[0][0]}")
    r_effs = [int(w[1].size) for w in wins]
    return s, phis, t, elapsed, kernels, r_effs


def block_roofline(kernels, n, kb, r_effs, precision):
    """Algorithmic bytes and flops of the block kernels (per launch)."""
    kc_total = sum(2 * r for r in r_effs)           # real output columns over the k windows
    flops = 2.0 * n * M * kc_total                   # project_block: X' (n x m) times m x kc per window
    mfma = {"project_block": (flops, FP32_MFMA_TFLOPS, "fp32")}
    if precision == "bf16x3":                        # three BF16 products per FP32 product
        mfma = {"project_block": (3 * flops, BF16_MFMA_TFLOPS, "bf16x3")}
    return roofline_of(
        kernels,
        {"gram_block": (M + 1 + kb) * n * 4 + kb * n * 4,                 # read window + block, write the block
         "project_block": (M + kb - 1) * n * 4 + n * 8 * (kc_total // 2)},  # read the union of X', write k Phi
        {"gram_block": "gram_block.hip", "project_block": "project.hip"},
        mfma, {"project_block": "project_block_bf16x3"} if precision == "bf16x3" else None)


def gram_back_to_back(frames, n, dmd, reps=20):
    """The one-frame Gram pass (`k_gram_columns` + finalize) over consecutive
    pushes with the solves switched off: the kernel's own HBM rate with
    nothing between its launches, against (m+2) n 4 bytes per launch."""
    import torch
    s = dmd.Stream(n, M, R, dtype="f32", auto_solve=False)
    try:
        t = 0
        for _ in range(M + 1):
            s.push(frames[t])
            t += 1
        torch.cuda.synchronize()
        dmd.profile_enable(True)
        dmd.profile_reset()
        for _ in range(reps):
            s.push(frames[t % len(frames)])
            t += 1
        torch.cuda.synchronize()
        dmd.profile_enable(False)
        cnt, ms = dmd.profile_read("gram_columns")
        dmd.profile_reset()
    finally:
        s.close()
    if not cnt:
        return None
    us = 1000.0 * ms / cnt
    gbs = (M + 2) * n * 4 / (us * 1e-6) / 1e9
    return {"avg_us": round(us, 2), "algorithmic_GBps": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "launches": int(cnt)}


def background_alone(s, n, dmd, reps=10):
    """Background subtraction of the newest snapshot (foreground and |l|),
    timed alone after single-frame pushes: its HBM rate against the roofline,
    m n 4 bytes read (the columns of X') and 2 n elements written."""
    import torch
    fg = torch.empty(n, dtype=s.pod_dtype, device="cuda")
    bg = torch.empty_like(fg)
    s.background(fg, bg)
    torch.cuda.synchronize()
    dmd.profile_enable(True)
    dmd.profile_reset()
    for _ in range(reps):
        s.background(fg, bg)
    torch.cuda.synchronize()
    dmd.profile_enable(False)
    cnt, ms = dmd.profile_read("background")
    dmd.profile_reset()
    if not cnt:
        return None
    us = 1000.0 * ms / cnt
    nbytes = (M * 4 + 2 * fg.element_size()) * n
    gbs = nbytes / (us * 1e-6) / 1e9
    return {"avg_us": round(us, 2), "algorithmic_bytes": nbytes, "algorithmic_GBps": round(gbs, 1),
            "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def bench_block(args):
    """k frames per step (multi-column update): one block push, the FP64
    solves of all k windows side by side, and the modes of all k windows."""
    import numpy as np
    import torch

    import paper_1612_07875_amd as dmd

    n = H * W
    kb = args.block
    K, Wu, L = args.steps, args.warmup, args.latency_frames
    LB = args.latency_blocks
    fill = M + 1
    T = fill + (Wu + K + LB) * kb + L + LAT_WARM
    keep = M + 1 + (args.cpu_windows if not args.no_cpu_baseline else 0)
    frames, host_keep = make_frames(T, keep)

    split = None
    if args.precision == "fp32" and not args.no_split:
        # the same workload with split-BF16 projections, for comparison
        s2, _, _, el2, kern2, re2 = timed_blocks(dmd, torch, frames, n, kb, K, Wu, "bf16x3")
        s2.close()
        torch.cuda.synchronize()
        split = {"value": round(kb * K / el2, 2), "ms_per_step": round(1000.0 * el2 / K, 4),
                 "kernels": kern2, "roofline": block_roofline(kern2, n, kb, re2, "bf16x3")}
        print(f"[bench] split-BF16: {kb * K / el2:.1f} window updates/s", file=sys.stderr, flush=True)

    s, phis, t, elapsed, kernels, r_effs = timed_blocks(dmd, torch, frames, n, kb, K, Wu, args.precision)
    print(f"[bench] timed {K} blocks of {kb} frames in {elapsed:.3f} s", file=sys.stderr, flush=True)
    r_eff = min(r_effs)

    # block latency: enqueue of a block -> all k windows' modes written (one stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    blat = []
    dmd.profile_enable(True)
    dmd.profile_reset()
    for _ in range(LB):
        e0.record()
        s.push_block(frames[t:t + kb])
        s.block_modes(phis)
        e1.record()
        e1.synchronize()
        blat.append(e0.elapsed_time(e1))
        t += kb
    dmd.profile_enable(False)
    alone = kernel_table(dmd, ("gram_block", "project_block"))
    dmd.profile_reset()
    latency, t, alone1 = single_latency(s, frames, t, L, phis[0].T, dmd)
    alone.update(alone1)
    gram_alone = gram_alone_line(alone, n, kb)
    background = background_alone(s, n, dmd) if L > 0 else None
    info = s.info()
    s.close()
    if L > 0:
        gram_alone["gram_columns_back_to_back"] = gram_back_to_back(frames, n, dmd)
    roofline = block_roofline(kernels, n, kb, r_effs, args.precision)
    out = result_line(kb * K / elapsed, K, Wu, elapsed, "f32", {
        "workload": f"blob video 1920x1080 FP32 (n=2073600), m=64, r=20; block mode: step = one push of "
                    f"{kb} frames (multi-column update) + FP64 solves of all {kb} windows + modes of all {kb} windows",
        "n": n, "m": M, "r": R, "r_eff": int(r_eff), "frames_per_step": kb,
        "precision": precision_note(args)})
    blat = np.array(blat) if blat else None
    out.update({"roofline": roofline, "kernels": kernels,
                "gram_GBps": kernels.get("gram_block", {}).get("algorithmic_GBps"), "gram_alone": gram_alone,
                "block_latency_ms": ({"p50": round(float(np.percentile(blat, 50)), 3),
                                      "p99": round(float(np.percentile(blat, 99)), 3), "blocks": int(LB)}
                                     if blat is not None else None),
                "latency_ms": latency, "latency_note": "latency_ms: single-frame pushes (push -> modes) on "
                                                       "the same stream after the timed blocks and "
                                                       f"{LAT_WARM} untimed single frames",
                "background_alone": background,
                "jacobi_sweeps": int(info.sweeps), "qr_iters": int(info.qr_iters)})
    if split is not None:
        out["split_bf16"] = split
    return out, host_keep


def bench_sparse(args):
    """The sparse configuration (and the spatial -> Fourier ingest feeding it)."""
    import numpy as np
    import torch

    import gen
    import paper_1612_07875_amd as dmd

    side, nnz, m, r = 512, 2621, 128, 24
    n = side * side
    K, Wu = args.steps, args.warmup
    T = m + 1 + Wu + K
    fs = gen.FourierSparse(side=side, nnz=nnz, redraw=0.05)
    t0 = time.perf_counter()
    pairs = [fs.frame(t) for t in range(T)]
    idx = [torch.from_numpy(i).cuda() for i, _ in pairs]
    val = [torch.from_numpy(v).cuda() for _, v in pairs]
    video = gen.BlobVideo(height=side, width=side, blob_sigma=12.0)
    spatial = torch.from_numpy(np.stack([video.frame(t) for t in range(T)]).reshape(T, side, side)).cuda()
    torch.cuda.synchronize()
    print(f"[bench] generated {T} sparse and {T} spatial frames in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    def leg(push, names):
        s = dmd.Stream(n, m, r, dtype="c64_csr", max_nnz=nnz)
        phi = torch.zeros((r, n), dtype=torch.complex64, device="cuda").T
        if push == "fourier":
            s.fourier_setup(side, side, nnz)
        do = (lambda t: s.push_fourier(spatial[t])) if push == "fourier" else (lambda t: s.push_csr(idx[t], val[t]))
        for t in range(m + 1 + Wu):
            do(t)
            s.modes(phi)
        torch.cuda.synchronize()
        dmd.profile_enable(True)
        dmd.profile_reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for t in range(m + 1 + Wu, T):
            do(t)
            s.modes(phi)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        dmd.profile_enable(False)
        kern = kernel_table(dmd, names)
        dmd.profile_reset()
        lam, sig, _ = s.eigs()
        s.close()
        return el, kern, int(lam.size)

    def batched_leg(B, L=1):
        # B streams of the same shape, stream b fed the frames from b on (distinct
        # windows), in L lanes (batches of B / L streams, each ticking on a HIP
        # stream of its own); one step = one tick per lane, which pushes a frame
        # into every stream of the lane and writes every stream's modes
        streams = [dmd.Stream(n, m, r, dtype="c64_csr", max_nnz=nnz) for _ in range(B)]
        outs = [torch.zeros((r, n), dtype=torch.complex64, device="cuda").T for _ in range(B)]
        lanes = [list(range(q, B, L)) for q in range(L)]
        queues = [torch.cuda.Stream() for _ in range(L)]
        for q in queues:
            q.wait_stream(torch.cuda.current_stream())
        batches = [dmd.Batch(max_streams=B) for _ in range(L)]
        try:
            for lane, batch in zip(lanes, batches):
                for b in lane:
                    batch.attach(streams[b])

            def tick(t):
                for lane, batch, q in zip(lanes, batches, queues):
                    batch.tick_frames([streams[b] for b in lane],
                                      [(idx[(t + b) % T], val[(t + b) % T]) for b in lane],
                                      modes=[outs[b] for b in lane], stream=q)

            for t in range(m + 1 + Wu):
                tick(t)
            torch.cuda.synchronize()
            dmd.profile_enable(True)
            dmd.profile_reset()
            t1 = time.perf_counter()
            for t in range(m + 1 + Wu, T):
                tick(t)
            torch.cuda.synchronize()
            el_b = time.perf_counter() - t1
            dmd.profile_enable(False)
            kern_b = kernel_table(dmd, ("batch_gram", "batch_solve", "batch_project"))
            dmd.profile_reset()
        finally:
            for batch in batches:
                batch.close()
        r_effs = [int(st.eigs()[0].size) for st in streams]
        for st in streams:
            st.close()
        return el_b, kern_b, r_effs

    names = ("csr_gram", "solve_sym", "solve_eig", "csr_project")
    el, kern, r_eff = leg("csr", names)
    el_f, kern_f, r_eff_f = leg("fourier", ("fourier",) + names)
    B = args.sparse_streams
    el_b, kern_b, r_effs_b = batched_leg(B) if B > 0 else (None, None, None)
    BL, LL = 3 * B, 3
    el_l, kern_l, r_effs_l = batched_leg(BL, LL) if B > 0 else (None, None, None)
    # the sparse Gram pass reads the window's coefficients once: (m+1) nnz (4 + 8) bytes
    roofline = roofline_of(kern, {"csr_gram": (m + 1) * nnz * 12}, {"csr_gram": "csr.hip"})
    out = result_line(K / el, K, Wu, el, "c64", {
        "workload": "Fourier-sparse frames: n = 512^2 complex64 coefficients at 1 % (2,621 per frame, "
                    "lowest wavenumbers, 5 % redrawn per frame), m = 128, r = 24; step = sparse push + FP64 "
                    "Hermitian solves + modes (dense n x r complex64 output)",
        "n": n, "nnz": nnz, "m": m, "r": r, "r_eff": r_eff, "frames_per_step": 1,
        "precision": "FP64 Gram accumulation, FP64 solves, FP32 sparse projection"})
    out.update({"roofline": roofline, "kernels": kern,
                "roofline_note": "latency-bound: one update reads 4 MB; the solves of the 128 x 128 "
                                 "Hermitian window dominate",
                "fourier_ingest": {"value": round(K / el_f, 2), "unit": "window updates/s",
                                   "ms_per_step": round(1000.0 * el_f / K, 4), "r_eff": r_eff_f,
                                   "workload": "512 x 512 FP32 spatial frames (blob video) -> unitary 2-D DFT at "
                                               "the 2,621 lowest-|k| bins on the device -> the same sparse path",
                                   "kernels": kern_f}})
    if B > 0:
        out["batched"] = {
            "value": round(B * K / el_b, 2), "unit": "window updates/s", "streams": B,
            "ms_per_tick": round(1000.0 * el_b / K, 4), "r_eff": sorted(set(r_effs_b)),
            "workload": f"{B} sparse streams of the same shape, one dmd_batch_tick_frames per step (a frame "
                        "into every stream, grouped Hermitian solves, every stream's modes)",
            "kernels": kern_b}
        out["batched_lanes"] = {
            "value": round(BL * K / el_l, 2), "unit": "window updates/s", "streams": BL, "lanes": LL,
            "ms_per_step": round(1000.0 * el_l / K, 4), "r_eff": sorted(set(r_effs_l)),
            "workload": f"{BL} sparse streams in {LL} lanes of {BL // LL} (a batch on a HIP stream of its own "
                        "each); one step = one tick per lane"}
    return out, None


def bench_modal(args):
    """Plain streaming DMD in FP64 (n = 4096, m = 32, r = 10, 64 frames):
    latency-bound; every timed update is one of the 32 windows of the 64
    frames (the stream is reset and the frames streamed again)."""
    import numpy as np
    import torch

    import gen
    import paper_1612_07875_amd as dmd

    n, m, r, T = 4096, 32, 10, 64
    g = gen.ModalStream(n=n, noise=1e-3)
    host = np.ascontiguousarray(g.frames(0, T).T)          # (T, n) FP64
    frames = torch.from_numpy(host).cuda()
    per_pass = T - m                                         # window updates per pass
    passes = max(1, -(-args.steps // per_pass))
    warm = max(1, -(-args.warmup // per_pass))
    s = dmd.Stream(n, m, r, dtype="f64")
    phi = torch.zeros((r, n), dtype=torch.complex128, device="cuda").T
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def fill():
        s.reset()
        for t in range(m):
            s.push(frames[t])
        torch.cuda.synchronize()

    for _ in range(warm):
        fill()
        for t in range(m, T):
            s.push(frames[t])
            s.modes(phi)
        torch.cuda.synchronize()
    # throughput: the steady-state updates of each pass back to back.  The
    # step is a few short kernels, so the per-kernel HIP events of the
    # profile (two per launch) would add host time to every step: the
    # timed passes run without them, and the kernel table comes from the
    # same passes repeated with the profile on (profiled_ms_per_step).
    def timed_passes():
        el = 0.0
        for _ in range(passes):
            fill()
            t0 = time.perf_counter()
            for t in range(m, T):
                s.push(frames[t])
                s.modes(phi)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
        return el

    elapsed = timed_passes()
    dmd.profile_enable(True)
    dmd.profile_reset()
    elapsed_prof = timed_passes()
    dmd.profile_enable(False)
    kernels = kernel_table(dmd, ("gram_columns", "gram_finalize", "solve_sym", "solve_eig", "project_modes"))
    dmd.profile_reset()
    K = passes * per_pass
    # latency: push -> modes of each update, one at a time
    lat = []
    for _ in range(passes):
        fill()
        for t in range(m, T):
            e0.record()
            s.push(frames[t])
            s.modes(phi)
            e1.record()
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
    lam, sig, _ = s.eigs()
    r_eff = int(lam.size)
    s.close()
    lat = np.array(lat)
    roofline = roofline_of(
        kernels, {"gram_columns": (m + 2) * n * 8, "project_modes": m * n * 8 + n * r_eff * 16},
        {"gram_columns": "gram_push.hip", "project_modes": "project.hip"})
    out = result_line(K / elapsed, K, warm * per_pass, elapsed, "f64", {
        "workload": "modal stream FP64: n=4096, five damped complex modes + N(0, 1e-3^2) noise, m=32, r=10, "
                    "64 frames (32 windows) streamed again after a reset; step = push + FP64 solves + FP64 modes",
        "n": n, "m": m, "r": r, "r_eff": r_eff, "frames_per_step": 1,
        "precision": "FP64 data, Gram, solves and projections"})
    out.update({"roofline": roofline, "kernels": kernels,
                "roofline_note": "latency-bound: the 1.08 MB window stays in cache; the single-CU FP64 solves set "
                                 "the step; kernel times from a second pass with per-kernel events",
                "profiled_ms_per_step": round(1000.0 * elapsed_prof / K, 4),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                               "p99": round(float(np.percentile(lat, 99)), 4), "frames": int(lat.size)}})
    return out, host, (m, r)


def bench_waves(args):
    """The precision-study workload streamed: n = 2^20 travelling waves,
    m = 256, r = 32; FP32 data and the same values as FP64 data.  Plus the
    whole-window Gram (257 columns) in each product precision."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import gen
    import paper_1612_07875_amd as dmd

    n, m, r = 1 << 20, 256, 32
    K, Wu = args.steps, args.warmup
    T = m + 1 + Wu + K
    w = gen.TravelingWaves(n=n, n_waves=8)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=16) as ex:
        host = np.stack(list(ex.map(w.frame, range(T))))      # (T, n) FP32
    print(f"[bench] generated {T} frames in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    def leg(dtype):
        X = torch.from_numpy(host).to(device="cuda", dtype=torch.float32 if dtype == "f32" else torch.float64)
        s = dmd.Stream(n, m, r, dtype=dtype)
        phi = torch.zeros((r, n), dtype=s.mode_dtype, device="cuda").T
        sp, sm = bench_streams(torch)
        sp.wait_stream(torch.cuda.current_stream())
        sm.wait_stream(torch.cuda.current_stream())
        for t in range(m + 1 + Wu):
            s.push(X[t], stream=sp)
            if t > m:
                s.modes(phi, stream=sm)
        torch.cuda.synchronize()
        dmd.profile_enable(True)
        dmd.profile_reset()
        t1 = time.perf_counter()
        for t in range(m + 1 + Wu, T):
            s.push(X[t], stream=sp)
            s.modes(phi, stream=sm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        dmd.profile_enable(False)
        kern = kernel_table(dmd, ("gram_columns", "gram_finalize", "solve_sym", "solve_eig", "project_modes"))
        dmd.profile_reset()
        lam, _, _ = s.eigs()
        s.close()
        del X
        torch.cuda.synchronize()
        return el, kern, int(lam.size)

    el32, kern32, re32 = leg("f32")
    el64, kern64, re64 = leg("f64")
    eb = 4
    roofline = roofline_of(
        kern32, {"gram_columns": (m + 2) * n * eb, "project_modes": m * n * eb + n * re32 * 8},
        {"gram_columns": "gram_push.hip", "project_modes": "project.hip"},
        {"project_modes": (2.0 * n * m * 2 * re32, FP32_MFMA_TFLOPS, "fp32")})
    g64 = kern64.get("gram_columns", {})
    if g64:
        g64["algorithmic_bytes"] = (m + 2) * n * 8
        g64["algorithmic_GBps"] = round(g64["algorithmic_bytes"] / (g64["avg_us"] * 1e-6) / 1e9, 1)
    # whole-window Gram (257 columns) per product precision, back to back
    Xw = torch.from_numpy(host[:m + 1]).cuda()
    Xw64 = Xw.double()
    G = torch.empty((m + 1, m + 1), dtype=torch.float64, device="cuda")
    k = m + 1
    flops = float(n) * k * (k + 1)                          # the k (k + 1) / 2 distinct entries, 2 n flops each
    whole = {}
    for name, X_, prec, peak, mult in (("fp64", Xw64, "default", 78.6, 1.0), ("fp32", Xw, "default",
                                        FP32_MFMA_TFLOPS, 1.0), ("bf16x3", Xw, "bf16x3", BF16_MFMA_TFLOPS, 3.0)):
        dmd.window_gram(X_, precision=prec, out=G)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        a.record()
        for _ in range(reps):
            dmd.window_gram(X_, precision=prec, out=G)
        b.record()
        b.synchronize()
        us = a.elapsed_time(b) * 1000.0 / reps
        nbytes = k * n * X_.element_size()
        whole[name] = {"avg_us": round(us, 1), "algorithmic_flops": flops * mult,
                       "achieved_TFLOPs": round(flops * mult / (us * 1e-6) / 1e12, 2), "peak_TFLOPs": peak,
                       "frac_of_mfma_peak": round(flops * mult / (us * 1e-6) / 1e12 / peak, 4),
                       "algorithmic_GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                       "frac_of_hbm_peak": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    del Xw, Xw64
    out = result_line(K / el32, K, Wu, el32, "f32", {
        "workload": "travelling waves n=2^20 FP32 (8 waves, amplitudes 10^(-k/2)), m=256, r=32; step = push + "
                    "FP64 solves + FP32 modes (modes of frame t beside the push of t+1)",
        "n": n, "m": m, "r": r, "r_eff": re32, "frames_per_step": 1,
        "precision": "FP64 Gram accumulation, FP64 solves, FP32 modes"})
    out.update({"roofline": roofline, "kernels": kern32,
                "gram_GBps": kern32.get("gram_columns", {}).get("algorithmic_GBps"),
                "fp64_data": {"value": round(K / el64, 2), "unit": "window updates/s",
                              "ms_per_step": round(1000.0 * el64 / K, 4), "r_eff": re64, "kernels": kern64},
                "whole_gram": whole,
                "whole_gram_note": "dmd_window_gram of the first 257 frames (1.08 GB FP32 / 2.16 GB FP64), "
                                   "10 calls back to back; algorithmic flops n k (k+1), three times that for "
                                   "split-BF16"})
    return out, host, (m, r)


def precision_note(args):
    modes = "FP32 modes" if args.precision == "fp32" else "BF16x3 modes (FP32 accumulation)"
    return "FP64 Gram accumulation, FP64 solves, " + modes


def result_line(value, K, Wu, elapsed, dtype, config):
    return {
        "metric": "DMD window updates/s + Gram HBM GB/s vs roofline; p99 frame latency",
        "value": round(value, 2),
        "unit": "window updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": round(1000.0 * elapsed / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }


def main():
    global R
    args = defaults(parse())
    R = args.rank
    if args.copy_probe and args.gpus == 1:
        copy_probe()
        return
    if args.serve and args.gpus == 1:
        serve_bench(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    mr = None
    if args.mode == "single":
        out, host_keep = bench_single(args)
    elif args.mode == "sparse":
        out, host_keep = bench_sparse(args)
    elif args.mode == "modal":
        out, host_keep, mr = bench_modal(args)
    elif args.mode == "waves":
        out, host_keep, mr = bench_waves(args)
    else:
        out, host_keep = bench_block(args)
    if not args.no_cpu_baseline and host_keep is not None:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        F = np.stack(host_keep) if isinstance(host_keep, list) else host_keep
        m, r = mr if mr is not None else (M, R)
        wins = {"modal": 32, "waves": 1}.get(args.mode, args.cpu_windows)
        frames = min(F.shape[0] - m - 1, {"modal": 31, "waves": 2}.get(args.mode, args.cpu_windows))
        out["cpu_baseline"] = cpu_baseline(F, min(wins, F.shape[0] - m), m, r)
        out["cpu_baseline_streaming"] = cpu_baseline_streaming(F, frames, m, r)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
