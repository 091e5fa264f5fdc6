// Streaming Gram update for one dense snapshot (Sec. 3.1, Algorithm 1's
// non-first-step branch; Algorithm 2's new xty column).
//
// Only the new snapshot's inner products are computed: one pass reads the m
// kept window columns plus the new snapshot and writes the snapshot into the
// first spare ring slot (ingest fused with the dots), so HBM traffic per push is
// (m+2) * n * sizeof(T) bytes.  The shift of the Gram is a change of the
// ring's `oldest` index, not a copy.
//
// Data are FP32 or FP64; products and sums are FP64 (an FP32 product is exact
// in FP64), so the Gram keeps the accuracy that the method of snapshots needs
// after squaring the condition number (Sec. 2.1).
//
// Reduction order is fixed: per-thread serial sums, a fixed butterfly inside
// each 64-wide wavefront, waves summed in index order, then workgroup
// partials summed in a fixed order by a small finalize kernel.  No
// floating-point atomics are used, so every run is bitwise identical.
#include "dmd_internal.h"
#include "gram_finalize.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kGroup = 4;  // window columns reduced together

template <typename T> struct Vec16;
template <> struct Vec16<float>  { using type = float4;  static constexpr int N = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int N = 2; };

// 16-byte vectors for nontemporal loads (the builtin takes clang vectors)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct NtVec;
template <> struct NtVec<float>  { using type = f32x4; };
template <> struct NtVec<double> { using type = f64x2; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Loads the ITER x N elements of this thread from column `col` of a slab.
// `vec_ok`: the slab is entirely inside [0, n) and `col` is 16-byte aligned.
// The 16-byte loads are nontemporal: every element is read once per pass and
// a window (m columns of n values) is far larger than the caches, so caching
// it only evicts other data.  Measured on 64 columns of 2,073,600 floats: a
// plain read-only pass runs at 0.78 of the HBM peak with cached loads and
// 0.87 with nontemporal ones; this kernel goes from 92 us to 87-89 us.
template <typename T, int ITER>
__device__ __forceinline__ void load_slab(const T* __restrict__ col, int64_t base, int64_t n,
                                          bool vec_ok, T (&v)[ITER][Vec16<T>::N]) {
    using NV = typename NtVec<T>::type;
    constexpr int N = Vec16<T>::N;
    if (vec_ok) {
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const NV w = __builtin_nontemporal_load(
                reinterpret_cast<const NV*>(col + base + (int64_t)(it * kThreads + threadIdx.x) * N));
#pragma unroll
            for (int k = 0; k < N; ++k) v[it][k] = w[k];
        }
    } else {
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int64_t i = base + (int64_t)(it * kThreads + threadIdx.x) * N + k;
                v[it][k] = i < n ? col[i] : T(0);
            }
        }
    }
}

__global__ __launch_bounds__(kFinThreads)
void k_gram_finalize(double* __restrict__ G, const double* __restrict__ partials, int nblk, int m, int slots,
                     DevState* __restrict__ st) {
    gram_finalize_body(G, partials, nblk, m, slots, st);
}

__global__ __launch_bounds__(kFinThreads)
void k_gram_finalize_grouped(const GramItem* __restrict__ items) {
    const GramItem& g = items[blockIdx.x];
    gram_finalize_body(g.G, g.partials, g.nblk, g.m, g.slots, g.st);
}

// One workgroup per slab of kThreads * N * ITER consecutive elements.
// partials[j * nblk + block] receives the slab's share of <x_j, x_new> for
// kept column j (window order) and, at j = nkept, of <x_new, x_new>.
template <typename T, int ITER>
__device__ void gram_slab(const T* __restrict__ x, T* __restrict__ ring, int64_t ld, int64_t n, int m, int slots,
                          int x_aligned, double* __restrict__ partials, int nblk,
                          const DevState* __restrict__ st, int blk) {
    constexpr int N = Vec16<T>::N;
    constexpr int SLAB = kThreads * N * ITER;
    using VT = typename Vec16<T>::type;

    const int count = st->count;
    const int oldest = st->oldest;
    const int spare = slot_of(oldest, count, slots);
    const int keep0 = (count == m + 1) ? 1 : 0;  // a full window drops its oldest column
    const int nkept = count - keep0;

    const int64_t base = (int64_t)blk * SLAB;
    const bool in_range = base + SLAB <= n;

    T xv[ITER][N];
    load_slab<T, ITER>(x, base, n, in_range && x_aligned, xv);

    // ingest: the new snapshot goes to the spare slot
    T* dst = ring + (int64_t)spare * ld;
    if (in_range) {
#pragma unroll
        for (int it = 0; it < ITER; ++it)
            *reinterpret_cast<VT*>(dst + base + (int64_t)(it * kThreads + threadIdx.x) * N) =
                *reinterpret_cast<const VT*>(&xv[it][0]);
    } else {
#pragma unroll
        for (int it = 0; it < ITER; ++it)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int64_t i = base + (int64_t)(it * kThreads + threadIdx.x) * N + k;
                if (i < n) dst[i] = xv[it][k];
            }
    }

    // Column groups: the slabs of the next group are loaded before the
    // current group's products and wavefront sums, so loads stay in flight
    // while the wavefront reduces; each wavefront's sums wait in LDS and the
    // waves are summed once at the end (one barrier per slab).
    constexpr int G = ITER * N >= 16 ? 2 : kGroup;  // columns per group (registers: two groups in flight)
    __shared__ double red[kWaves][kMaxM + 2];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    auto load_group = [&](int j0, T (&cv)[G][ITER][N]) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int j = j0 + u;
            if (j < nkept) {
                const T* col = ring + (int64_t)slot_of(oldest, keep0 + j, slots) * ld;
                load_slab<T, ITER>(col, base, n, in_range, cv[u]);
            }
        }
    };
    T cv[2][G][ITER][N];
    load_group(0, cv[0]);
    for (int j0 = 0; j0 <= nkept; j0 += 2 * G) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jg = j0 + h * G;
            if (jg > nkept) break;
            if (jg + G <= nkept) load_group(jg + G, cv[h ^ 1]);
            double acc[G];
#pragma unroll
            for (int u = 0; u < G; ++u) acc[u] = 0.0;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int j = jg + u;
                if (j < nkept) {
#pragma unroll
                    for (int it = 0; it < ITER; ++it)
#pragma unroll
                        for (int k = 0; k < N; ++k)
                            acc[u] = fma((double)cv[h][u][it][k], (double)xv[it][k], acc[u]);
                } else if (j == nkept) {
#pragma unroll
                    for (int it = 0; it < ITER; ++it)
#pragma unroll
                        for (int k = 0; k < N; ++k)
                            acc[u] = fma((double)xv[it][k], (double)xv[it][k], acc[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const double v = wave_sum(acc[u]);
                if (lane == 0 && jg + u <= nkept) red[wave][jg + u] = v;
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= nkept; j += kThreads) {
        double s = red[0][j];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += red[w][j];
        partials[(int64_t)j * nblk + blk] = s;
    }
}

template <typename T, int ITER>
__global__ __launch_bounds__(kThreads)
void k_gram_columns(const T* __restrict__ x, T* __restrict__ ring, int64_t ld, int64_t n, int m, int slots,
                    int x_aligned, double* __restrict__ partials, int nblk, const DevState* __restrict__ st) {
    gram_slab<T, ITER>(x, ring, ld, n, m, slots, x_aligned, partials, nblk, st, blockIdx.x);
}

// Grouped form: one launch covers the new snapshots of many streams; block b
// belongs to the item i with blk_start[i] <= b < blk_start[i+1].
__device__ __forceinline__ int find_item(const int* __restrict__ blk_start, int nitems, int b) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Each item keeps the slab size its stream uses on its own, so a stream's
// inner products are summed in the same order alone and in a batch.
__global__ __launch_bounds__(kThreads)
void k_gram_columns_grouped(const GramItem* __restrict__ items, const int* __restrict__ blk_start, int nitems) {
    const int i = find_item(blk_start, nitems, blockIdx.x);
    const GramItem g = items[i];
    const int blk = blockIdx.x - blk_start[i];
    const float* x = static_cast<const float*>(g.x);
    float* ring = static_cast<float*>(g.ring);
    switch (g.iter) {
        case 4: gram_slab<float, 4>(x, ring, g.ld, g.n, g.m, g.slots, g.x_aligned, g.partials, g.nblk, g.st, blk); break;
        case 2: gram_slab<float, 2>(x, ring, g.ld, g.n, g.m, g.slots, g.x_aligned, g.partials, g.nblk, g.st, blk); break;
        default: gram_slab<float, 1>(x, ring, g.ld, g.n, g.m, g.slots, g.x_aligned, g.partials, g.nblk, g.st, blk); break;
    }
}

template <typename T> int blocks_for(int64_t n, int iter) {
    const int64_t slab = (int64_t)kThreads * Vec16<T>::N * iter;
    return (int)((n + slab - 1) / slab);
}

}  // namespace

int gram_push_blocks(int64_t n, int elem_bytes) {
    // capacity of the partials buffer: the smallest ITER gives the most blocks
    return elem_bytes == 8 ? blocks_for<double>(n, 1) : blocks_for<float>(n, 1);
}

int gram_iter_rule(int64_t n, int elem_bytes) {
    // The largest slab (up to 4 x 16-byte loads per thread and column) that
    // still gives at least 256 workgroups, one per CU: big slabs keep many
    // requests in flight and leave few partial sums for the finalize kernel.
    const int64_t per_iter = (int64_t)kThreads * (16 / elem_bytes);
    if (n >= per_iter * 4 * 256) return 4;
    if (n >= per_iter * 2 * 256) return 2;
    return 1;
}

int gram_blocks(int64_t n, int elem_bytes, int iter) {
    return elem_bytes == 8 ? blocks_for<double>(n, iter) : blocks_for<float>(n, iter);
}

template <typename T>
hipError_t launch_gram_columns(const T* x, T* ring, int64_t ld, int64_t n, int m, int slots, double* partials,
                               int nblk_cap, const DevState* st, int iter, int* nblk_used, hipStream_t s) {
    if (iter != 1 && iter != 2 && iter != 4) return hipErrorInvalidValue;
    const int nblk = blocks_for<T>(n, iter);
    if (nblk > nblk_cap) return hipErrorInvalidValue;
    *nblk_used = nblk;
    const int x_aligned = ((uintptr_t)x % 16) == 0;
    dim3 grid(nblk), block(kThreads);
    switch (iter) {
        case 4: hipLaunchKernelGGL((k_gram_columns<T, 4>), grid, block, 0, s, x, ring, ld, n, m, slots, x_aligned, partials, nblk, st); break;
        case 2: hipLaunchKernelGGL((k_gram_columns<T, 2>), grid, block, 0, s, x, ring, ld, n, m, slots, x_aligned, partials, nblk, st); break;
        default: hipLaunchKernelGGL((k_gram_columns<T, 1>), grid, block, 0, s, x, ring, ld, n, m, slots, x_aligned, partials, nblk, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_gram_finalize(double* G, const double* partials, int nblk, int m, int slots, DevState* st,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_gram_finalize, dim3(1), dim3(kFinThreads), 0, s, G, partials, nblk, m, slots, st);
    return hipGetLastError();
}

hipError_t launch_gram_grouped(const GramItem* items, const int* blk_start, int nitems, int total_blocks,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_gram_columns_grouped, dim3(total_blocks), dim3(kThreads), 0, s, items, blk_start,
                       nitems);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_finalize_grouped, dim3(nitems), dim3(kFinThreads), 0, s, items);
    return hipGetLastError();
}

template hipError_t launch_gram_columns<float>(const float*, float*, int64_t, int64_t, int, int, double*, int,
                                               const DevState*, int, int*, hipStream_t);
template hipError_t launch_gram_columns<double>(const double*, double*, int64_t, int64_t, int, int, double*, int,
                                                const DevState*, int, int*, hipStream_t);

}  // namespace dmd
