// Whole Gram of a window, G = X^* X for its k <= m+1 columns (Algorithm 1's
// first step; Sec. 2.1 step 1), on the matrix cores.
//
// The k x k result is cut into 64 x 64 tiles; only tiles on or above the
// diagonal are computed (G is symmetric) and mirrored.  The n rows are split
// into `nsplit` ranges so that tiles x splits workgroups fill the chip (the
// tiles of one split on one XCD, sharing its L2); each workgroup stages 64
// (FP32 data) or 32 (FP64 data) rows of its two 64-column panels at a time
// in one of two LDS buffers (16-byte coalesced loads into registers during
// the previous stage's products) and accumulates its tile with MFMAs,
// skipping 16-column blocks past the window's last column; per-split tiles
// are summed in FP64 in a fixed order by a second kernel, which also writes
// the Gram (physical slot indexing) and the window state.
//
// Precision of the products and of the in-tile accumulation:
//   FP64    v_mfma_f64_16x16x4f64, data widened exactly to FP64;
//   FP32    v_mfma_f32_16x16x4f32, FP32 accumulation;
//   BF16X3  v_mfma_f32_16x16x32_bf16 on x = hi + lo (hi = bf16(x),
//           lo = bf16(x - hi)): hi*hi + hi*lo + lo*hi, FP32 accumulation.
//
// Fragment layouts (checked on the device): 16x16x4 A[l%16][l/16],
// B[l/16][l%16]; 16x16x32 A[l%16][8(l/16)+e], B[8(l/16)+e][l%16];
// D f32 [4(l/16)+v][l%16], D f64 [(l/16)+4v][l%16].
#include <type_traits>

#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

enum Mode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16X3 = 2 };

template <int MODE> struct MAcc { using type = v4f; };
template <> struct MAcc<MODE_F64> { using type = v4d; };

struct GramFullArgs {
    const void* ring;
    int64_t ld, n;
    int m, slots, oldest_override;  // oldest_override >= 0: use it instead of the state's
    int kcols;                      // columns of the window (<= m+1)
    int ntile, nsplit;
    int64_t rows_per_split;
    double* partial;                // [nsplit][ntiles_tri][64 * 64]
    const DevState* st;
};

__device__ __forceinline__ void tri_of(int t, int ntile, int& ti, int& tj) {
    // t-th pair (ti <= tj) in row-major order of the upper triangle
    ti = 0;
    int rem = t;
    while (rem >= ntile - ti) {
        rem -= ntile - ti;
        ++ti;
    }
    tj = ti + rem;
}

template <typename TX, int MODE>
__global__ __launch_bounds__(kThreads)
void k_gram_tiles(GramFullArgs a) {
    // Rows are staged 64 (FP32) or 32 (FP64) at a time, column-major with an
    // odd stride, in two LDS buffers: the next full stage is loaded into
    // registers while the current one is multiplied, then stored to the
    // other buffer (one barrier per stage).
    constexpr int PER = 16 / sizeof(TX);  // elements per 16-byte load
    constexpr int R = 16 * PER;           // rows per stage
    constexpr int LDR = R + 1;
    constexpr int TPC = R / PER;          // loads per column and stage
    using T = typename std::conditional<MODE == MODE_F64, double, float>::type;
    using AccT = typename MAcc<MODE>::type;
    using V = typename std::conditional<PER == 4, float4, double2>::type;
    __shared__ TX Lb[2][2 * kTile * LDR];

    // Workgroup b goes to XCD b % 8 (dispatch order).  With nsplit a
    // multiple of 8, the tiles of one row split share b % 8, so they run on
    // one XCD and read their common column panels through its L2.
    const int ntri = a.ntile * (a.ntile + 1) / 2;
    int tile, split;
    if (a.nsplit % 8 == 0) {
        const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
        split = slot / ntri * 8 + x;
        tile = slot % ntri;
    } else {
        tile = blockIdx.x % ntri;
        split = blockIdx.x / ntri;
    }
    int ti, tj;
    tri_of(tile, a.ntile, ti, tj);
    const bool diag = ti == tj;
    const int oldest = a.oldest_override >= 0 ? a.oldest_override : a.st->oldest;
    const int kcols = a.oldest_override >= 0 ? a.kcols : min(a.kcols, a.st->count);
    if (kcols <= 0) return;  // (no entry is written back)
    const TX* ring = reinterpret_cast<const TX*>(a.ring);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lk = lane >> 4;

    AccT acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = AccT{0, 0, 0, 0};

    const int64_t r_begin = (int64_t)split * a.rows_per_split;
    const int64_t r_end = min(a.n, r_begin + a.rows_per_split);
    const int npanel = diag ? 1 : 2;
    // global column of staged column c (past the window: the last column;
    // its products land only in entries that are not written back)
    auto gcol = [&](int c) {
        const int g = c < kTile ? ti * kTile + c : tj * kTile + c - kTile;
        return g < kcols ? g : kcols - 1;
    };
    // loads per thread and stage: both panels' columns (a diagonal tile
    // reads its one panel twice, so that no load sits under a branch)
    constexpr int NLD = 2 * kTile * TPC / kThreads;
    // the stage's loads of this thread: column t / TPC, rows q PER .. of the stage
    const TX* src[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int t = threadIdx.x + u * kThreads, c = t / TPC, q = t % TPC;
        src[u] = ring + (int64_t)slot_of(oldest, gcol(c < npanel * kTile ? c : c - kTile), a.slots) * a.ld + q * PER;
    }
    auto put = [&](TX* L, int u, const V& v) {
        const int t = threadIdx.x + u * kThreads, c = t / TPC, q = t % TPC;
        TX* d = L + c * LDR + q * PER;
        if constexpr (PER == 4) {
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        } else {
            d[0] = v.x; d[1] = v.y;
        }
    };
    // products of one staged buffer, NC 16-column blocks of the panel
    // (blocks past the window's last column are skipped)
    const int cj0 = diag ? 0 : kTile;
    auto products = [&](const TX* L, auto ncb) __attribute__((always_inline)) {
        constexpr int NC = decltype(ncb)::value;
        if constexpr (MODE == MODE_BF16X3) {
#pragma unroll
            for (int k0 = 0; k0 < R; k0 += 32) {
                v8bf ahi, alo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = (float)L[(16 * wave + li) * LDR + k0 + 8 * lk + e];
                    const __bf16 h = (__bf16)x;
                    ahi[e] = h;
                    alo[e] = (__bf16)(x - (float)h);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    v8bf bhi, blo;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float x = (float)L[(cj0 + 16 * c + li) * LDR + k0 + 8 * lk + e];
                        const __bf16 h = (__bf16)x;
                        bhi[e] = h;
                        blo[e] = (__bf16)(x - (float)h);
                    }
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[c], 0, 0, 0);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[c], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 4
            for (int k0 = 0; k0 < R; k0 += 4) {
                const T av = (T)L[(16 * wave + li) * LDR + k0 + lk];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const T bv = (T)L[(cj0 + 16 * c + li) * LDR + k0 + lk];
                    if constexpr (MODE == MODE_F64) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[c], 0, 0, 0);
                    else acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[c], 0, 0, 0);
                }
            }
        }
    };
    // the wave's 16 rows of the tile and the panel's 16-column blocks that
    // hold window columns
    const bool rows_live = ti * kTile + 16 * wave < kcols;
    const int cblk = rows_live ? max(0, min(4, (kcols - tj * kTile + 15) / 16)) : 0;
    auto compute = [&](const TX* L) __attribute__((always_inline)) {
        switch (cblk) {
            case 4: products(L, std::integral_constant<int, 4>{}); break;
            case 3: products(L, std::integral_constant<int, 3>{}); break;
            case 2: products(L, std::integral_constant<int, 2>{}); break;
            case 1: products(L, std::integral_constant<int, 1>{}); break;
            default: break;
        }
    };
    // full stages (r0 + R <= r_end) pipelined; the ragged last one after
    const int nfull = (int)((r_end - r_begin) / R);
    if (nfull > 0) {
#pragma unroll
        for (int u = 0; u < NLD; ++u) put(Lb[0], u, *reinterpret_cast<const V*>(src[u] + r_begin));
        __syncthreads();
    }
    for (int st = 0; st < nfull; ++st) {
        const int b = st & 1;
        const int64_t rn = r_begin + (int64_t)(st + 1) * R;
        V nx[NLD];
        if (st + 1 < nfull) {
#pragma unroll
            for (int u = 0; u < NLD; ++u) nx[u] = *reinterpret_cast<const V*>(src[u] + rn);
        }
        compute(Lb[b]);
        if (st + 1 < nfull) {
#pragma unroll
            for (int u = 0; u < NLD; ++u) put(Lb[b ^ 1], u, nx[u]);
        }
        __syncthreads();
    }
    {
        const int64_t r0 = r_begin + (int64_t)nfull * R;
        if (r0 < r_end) {
            TX* L = Lb[nfull & 1];
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                const int t = threadIdx.x + u * kThreads, q = t % TPC;
                TX e[PER];
#pragma unroll
                for (int i2 = 0; i2 < PER; ++i2) e[i2] = r0 + q * PER + i2 < r_end ? src[u][r0 + i2] : TX(0);
                if constexpr (PER == 4) put(L, u, V{e[0], e[1], e[2], e[3]});
                else put(L, u, V{e[0], e[1]});
            }
            __syncthreads();
            compute(L);
        }
    }

    double* out = a.partial + ((int64_t)split * ntri + tile) * (kTile * kTile);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * wave + (MODE == MODE_F64 ? lk + 4 * v : 4 * lk + v);
            const int j = 16 * c + li;
            out[i * kTile + j] = (double)acc[c][v];
        }
}

// Sum the per-split tiles in split order and write G (both triangles).
// set_window = 1: the Gram came with a new window (slots 0 .. kcols-1), so the
// window state is set; 2: the Gram of the current window was recomputed.  In
// both cases the previous eigenvectors no longer describe the Gram.
__global__ __launch_bounds__(kThreads)
void k_gram_reduce(GramFullArgs a, double* __restrict__ G, DevState* __restrict__ st, int set_window) {
    const int ntri = gridDim.x;
    const int tile = blockIdx.x;
    int ti, tj;
    tri_of(tile, a.ntile, ti, tj);
    const int oldest = a.oldest_override >= 0 ? a.oldest_override : st->oldest;
    const int kcols = a.oldest_override >= 0 ? a.kcols : min(a.kcols, st->count);
    __syncthreads();
    for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) {
        const int i = ti * kTile + e / kTile, j = tj * kTile + e % kTile;
        if (i >= kcols || j >= kcols || (ti == tj && j < i)) continue;
        double s = 0.0;
        for (int p = 0; p < a.nsplit; ++p) s += a.partial[((int64_t)p * ntri + tile) * (kTile * kTile) + e];
        const int si = slot_of(oldest, i, a.slots), sj = slot_of(oldest, j, a.slots);
        G[si + (int64_t)sj * a.slots] = s;
        G[sj + (int64_t)si * a.slots] = s;
    }
    __syncthreads();
    if (set_window && tile == 0 && threadIdx.x == 0) {
        if (set_window == 1) {
            st->oldest = a.oldest_override;
            st->count = a.kcols;
        }
        st->pushes += 1;
        st->vprev_valid = 0;
    }
}

// Copy k columns of X (n x k, leading dimension ldx) into ring slots 0 .. k-1.
template <typename TX>
__global__ __launch_bounds__(kThreads)
void k_copy_columns(const TX* __restrict__ X, int64_t ldx, TX* __restrict__ ring, int64_t ld, int64_t n, int k) {
    const int c = blockIdx.y;
    if (c >= k) return;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        ring[(int64_t)c * ld + i] = X[(int64_t)c * ldx + i];
}

}  // namespace

int gram_full_tiles(int m) {
    const int t = (m + 1 + kTile - 1) / kTile;
    return t * (t + 1) / 2;
}

int gram_full_splits(int m) {
    // about 512 workgroups; a multiple of 8 row splits where there are 8 or
    // more (one XCD per split, see k_gram_tiles)
    const int ntri = gram_full_tiles(m);
    int s = (512 + ntri - 1) / ntri;
    s = s > 128 ? 128 : s;
    return s >= 8 ? s / 8 * 8 : (s < 1 ? 1 : s);
}

hipError_t launch_gram_full(const void* ring, int64_t ld, int64_t n, int m, int slots, int elem_f64,
                            int precision, int kcols, int oldest_override, double* partial, double* G,
                            DevState* st, int set_window, hipStream_t s) {
    GramFullArgs a{};
    a.ring = ring;
    a.ld = ld;
    a.n = n;
    a.m = m;
    a.slots = slots;
    a.oldest_override = oldest_override;
    a.kcols = kcols;
    a.ntile = (kcols + kTile - 1) / kTile;
    const int ntri = a.ntile * (a.ntile + 1) / 2;
    a.nsplit = gram_full_splits(m);
    const int64_t granule = 64;
    a.rows_per_split = ((n + a.nsplit - 1) / a.nsplit + granule - 1) / granule * granule;
    a.partial = partial;
    a.st = st;
    dim3 grid(ntri * a.nsplit);
    // FP64 data always accumulates in FP64; FP32 data in the stream's precision
    int mode = MODE_F32;
    if (elem_f64 || precision == 3 /*FP64*/) mode = MODE_F64;
    else if (precision == 2 /*BF16X3*/) mode = MODE_BF16X3;
    if (elem_f64) {
        hipLaunchKernelGGL((k_gram_tiles<double, MODE_F64>), grid, dim3(kThreads), 0, s, a);
    } else if (mode == MODE_F64) {
        hipLaunchKernelGGL((k_gram_tiles<float, MODE_F64>), grid, dim3(kThreads), 0, s, a);
    } else if (mode == MODE_BF16X3) {
        hipLaunchKernelGGL((k_gram_tiles<float, MODE_BF16X3>), grid, dim3(kThreads), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_gram_tiles<float, MODE_F32>), grid, dim3(kThreads), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce, dim3(ntri), dim3(kThreads), 0, s, a, G, st, set_window);
    return hipGetLastError();
}

hipError_t launch_copy_columns(const void* X, int64_t ldx, void* ring, int64_t ld, int64_t n, int k, int elem_f64,
                               hipStream_t s) {
    const int64_t per = (int64_t)kThreads * 8;
    const unsigned gx = (unsigned)((n + per - 1) / per);
    dim3 grid(gx < 4096 ? gx : 4096, k);
    if (elem_f64)
        hipLaunchKernelGGL(k_copy_columns<double>, grid, dim3(kThreads), 0, s, static_cast<const double*>(X), ldx,
                           static_cast<double*>(ring), ld, n, k);
    else
        hipLaunchKernelGGL(k_copy_columns<float>, grid, dim3(kThreads), 0, s, static_cast<const float*>(X), ldx,
                           static_cast<float*>(ring), ld, n, k);
    return hipGetLastError();
}

}  // namespace dmd
