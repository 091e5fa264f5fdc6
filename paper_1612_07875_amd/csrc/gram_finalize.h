// Finalize of the one-frame Gram pass, shared by its own kernel and by the
// fused finalize + tridiagonal solve of single pushes.
#pragma once

#include "dmd_internal.h"

namespace dmd {

// Sums the per-workgroup partials in a fixed order (lane-strided partial sums,
// then a fixed butterfly), rejects a snapshot whose inner products are not
// finite, otherwise writes the new Gram row and column and advances the
// window: the oldest snapshot leaves a full window (the shift of Algorithm 1).
// 1024 threads; every lane issues its loads independently so that the
// reduction is bound by memory-level parallelism, not latency.
constexpr int kFinThreads = 1024;
constexpr int kFinLanes = 16;  // lanes per column

__device__ inline void gram_finalize_body(double* __restrict__ G, const double* __restrict__ partials, int nblk, int m,
                                   int slots, DevState* __restrict__ st) {
    const int count = st->count;
    const int oldest = st->oldest;
    const int spare = slot_of(oldest, count, slots);
    const int keep0 = (count == m + 1) ? 1 : 0;
    const int nkept = count - keep0;

    __shared__ double g[kMaxM + 2];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    const int sub = threadIdx.x % kFinLanes;
    const int grp = threadIdx.x / kFinLanes;
    constexpr int kGroups = kFinThreads / kFinLanes;
    for (int j = grp; j <= nkept; j += kGroups) {
        const double* pj = partials + (int64_t)j * nblk;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = sub;
        for (; b + 3 * kFinLanes < nblk; b += 4 * kFinLanes) {
            a0 += pj[b];
            a1 += pj[b + kFinLanes];
            a2 += pj[b + 2 * kFinLanes];
            a3 += pj[b + 3 * kFinLanes];
        }
        for (; b < nblk; b += kFinLanes) a0 += pj[b];
        double v = (a0 + a1) + (a2 + a3);
#pragma unroll
        for (int off = kFinLanes / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (sub == 0) g[j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= nkept; j += kFinThreads)
        if (!isfinite(g[j])) bad = 1;
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) st->rejected_nonfinite += 1;
        return;
    }
    for (int j = threadIdx.x; j < nkept; j += kFinThreads) {
        const int sj = slot_of(oldest, keep0 + j, slots);
        G[sj + (int64_t)spare * slots] = g[j];  // <x_j, x_new>
        G[spare + (int64_t)sj * slots] = g[j];  // real data: symmetric
    }
    if (threadIdx.x == 0) {
        G[spare + (int64_t)spare * slots] = g[nkept];
        if (count == m + 1) st->oldest = slot_of(oldest, 1, slots);
        else st->count = count + 1;
        st->pushes += 1;
    }
}

}  // namespace dmd
