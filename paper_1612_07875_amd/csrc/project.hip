// Tall-skinny projections of the window: DMD modes Phi = X' (V Sigma^-1 W)
// (Eq. Phi) and POD modes U = X (V Sigma^-1) (Sec. 2.1, step 2).
//
// out (n x kcols) = X_sub (n x m, ring columns in window order) * B (m x kcols),
// B row-major.  For the modes B holds the complex m x r_eff matrix
// C = V Sigma^-1 W as 2 r_eff interleaved real columns, so a real window gives
// interleaved complex output directly.
//
// Dense contraction on the matrix cores: v_mfma_f32_16x16x4f32 (FP32) or
// v_mfma_f64_16x16x4f64 (FP64).  A wavefront owns 64 rows (four 16-row
// tiles) and all output columns (up to four 16-column tiles); per step of
// four window columns it loads its A fragments straight from the ring (each
// lane one element, 16 consecutive rows per column) and the B fragments from
// the (L2-resident) coefficient matrix.
//
// Fragment layouts of the 16x16x4 instructions (checked on the device):
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D (f32): lane l holds D[4 (l / 16) + v][l % 16], v = 0..3;
//   D (f64): lane l holds D[(l / 16) + 4 v][l % 16], v = 0..3.
#include <type_traits>

#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;   // 4 wavefronts
constexpr int kRowsPerWave = 64;
constexpr int kRowsPerBlock = kThreads / 64 * kRowsPerWave;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
struct Frag {  // one lane's 8 coefficient values of a B fragment (k_pack_coef)
    uint4 x, y;
};

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi): the BF16x3 split.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}
// The value of the neighbouring lane (lane ^ 1): DPP quad permutation 1,0,3,2.
__device__ __forceinline__ float swap_pair(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
// The split as one word: hi in the low half, lo in the high half.
__device__ __forceinline__ unsigned split_word(float x) {
    __bf16 h, l;
    split_bf16(x, h, l);
    return (unsigned)__builtin_bit_cast(unsigned short, h) | ((unsigned)__builtin_bit_cast(unsigned short, l) << 16);
}
// acc += a b in three BF16 products (hi*hi + hi*lo + lo*hi), FP32 accumulation;
// the small terms first.
__device__ __forceinline__ v4f mma_bf16x3(const v8bf& ahi, const v8bf& alo, const v8bf& bhi, const v8bf& blo, v4f acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<float> {
    using type = v4f;
    static __device__ __forceinline__ v4f mma(float a, float b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <> struct Acc<double> {
    using type = v4d;
    static __device__ __forceinline__ v4d mma(double a, double b, v4d c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// TX: ring element type; T: coefficient, accumulation and output type.
// NT: number of 16-column output tiles (kcols <= 16 NT).
// The A and B fragments of the next group of four k-steps are loaded while
// the current group's MFMAs run; output tiles go through LDS so that every
// store instruction writes 64 consecutive rows of one output column.
constexpr int kOLD = 17;  // padded row length of the output stage
constexpr int kStage = kThreads / 64 * 64 * kOLD;

template <typename TX, typename T, int NT>
__device__ void project_body(const ProjectArgs& a, int blk, T* stage) {
    using AccT = typename Acc<T>::type;
    constexpr int KG = sizeof(T) == 8 ? 2 : 4;  // k-steps (of 4 columns) per group
    constexpr int OLD = kOLD;
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY) return;
    if (a.block_only && st->block_rejected) return;
    const int k_eff = st->r_eff;
    const int kcols = a.cplx_out ? 2 * k_eff : k_eff;
    if (kcols == 0) return;
    const int m = window_cols(a.m, a.buildup, st);  // columns of X_sub (fewer during a build-up start)
    const int rowstride = a.cplx_out ? 2 * a.kmax : a.kmax;
    const T* B = reinterpret_cast<const T*>(a.B);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blk * kRowsPerBlock + wave * kRowsPerWave;
    const int oldest = st->oldest;
    const TX* ring = reinterpret_cast<const TX*>(a.ring);

    AccT acc[4][NT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = AccT{0, 0, 0, 0};

    bool rin[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) rin[rt] = row0 + 16 * rt + li < a.n;

    T av[2][KG][4], bv[2][KG][NT];
    auto load_group = [&](int buf, int k0) {
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const int col = k0 + 4 * g + lk;
            const bool cin = col < m;
            const TX* cp = ring + (int64_t)slot_of(oldest, a.first + (cin ? col : 0), a.slots) * a.ld;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                av[buf][g][rt] = (cin && rin[rt]) ? (T)__builtin_nontemporal_load(&cp[row0 + 16 * rt + li]) : T(0);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = 16 * nt + li;
                bv[buf][g][nt] = (cin && c < kcols) ? B[(int64_t)col * rowstride + c] : T(0);
            }
        }
    };
    auto mma_group = [&](int buf) {
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[rt][nt] = Acc<T>::mma(av[buf][g][rt], bv[buf][g][nt], acc[rt][nt]);
    };
    // two groups per iteration so that both register buffers have static indices
    const int ngroups = (m + 4 * KG - 1) / (4 * KG);
    load_group(0, 0);
    for (int gi = 0; gi < ngroups; gi += 2) {
        if (gi + 1 < ngroups) load_group(1, (gi + 1) * 4 * KG);
        mma_group(0);
        if (gi + 1 >= ngroups) break;
        if (gi + 2 < ngroups) load_group(0, (gi + 2) * 4 * KG);
        mma_group(1);
    }

    // window columns are read and modes written nontemporally: each is
    // touched once per call, and the solves of the next push, which may run
    // beside this kernel, keep their data cached
    T* out = reinterpret_cast<T*>(a.out);
    T* sw = stage + wave * 64 * OLD;
    const int64_t row = row0 + lane;  // the row this lane stores
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        if (16 * nt >= kcols) break;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) sw[(16 * rt + Acc<T>::row(lk, v)) * OLD + li] = acc[rt][nt][v];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row < a.n) {
            if (a.cplx_out) {
#pragma unroll
                for (int cc = 0; cc < 16; cc += 2) {
                    const int c = 16 * nt + cc;
                    if (c < kcols) {
                        const int64_t o = 2 * (row + (int64_t)(c >> 1) * a.ldo);
                        __builtin_nontemporal_store(sw[lane * OLD + cc], &out[o]);
                        __builtin_nontemporal_store(sw[lane * OLD + cc + 1], &out[o + 1]);
                    }
                }
            } else {
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) {
                    const int c = 16 * nt + cc;
                    if (c < kcols) out[row + (int64_t)c * a.ldo] = sw[lane * OLD + cc];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// BF16x3 form (FP32 ring and coefficients, DMD_PREC_BF16X3): per chunk of 32
// window columns each lane holds 8 consecutive columns of one row (A) and 8
// consecutive rows of one coefficient column (B) of the 16x16x32 fragments
// (A[l%16][8(l/16)+e], B[8(l/16)+e][l%16]; D as the f32 16x16x4 layout).
template <int NT>
__device__ void project_body_bf3(const ProjectArgs& a, int blk, float* stage) {
    constexpr int OLD = kOLD;
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY) return;
    if (a.block_only && st->block_rejected) return;
    const int k_eff = st->r_eff;
    const int kcols = a.cplx_out ? 2 * k_eff : k_eff;
    if (kcols == 0) return;
    const int m = window_cols(a.m, a.buildup, st);  // columns of X_sub (fewer during a build-up start)
    const int rowstride = a.cplx_out ? 2 * a.kmax : a.kmax;
    const float* B = reinterpret_cast<const float*>(a.B);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)blk * kRowsPerBlock + wave * kRowsPerWave;
    const int oldest = st->oldest;
    const float* ring = reinterpret_cast<const float*>(a.ring);

    v4f acc[4][NT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = v4f{0, 0, 0, 0};
    for (int c0 = 0; c0 < m; c0 += 32) {
        v8bf ahi[4], alo[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int col = c0 + 8 * lq + e;
            const bool cin = col < m;
            const float* cp = ring + (int64_t)slot_of(oldest, a.first + (cin ? col : 0), a.slots) * a.ld;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int64_t r = row0 + 16 * rt + li;
                const float x = (cin && r < a.n) ? cp[r] : 0.0f;
                __bf16 h, l;
                split_bf16(x, h, l);
                ahi[rt][e] = h;
                alo[rt][e] = l;
            }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            v8bf bhi, blo;
            const int c = 16 * nt + li;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int col = c0 + 8 * lq + e;
                const float y = (col < m && c < kcols) ? B[(int64_t)col * rowstride + c] : 0.0f;
                __bf16 h, l;
                split_bf16(y, h, l);
                bhi[e] = h;
                blo[e] = l;
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) acc[rt][nt] = mma_bf16x3(ahi[rt], alo[rt], bhi, blo, acc[rt][nt]);
        }
    }

    float* out = reinterpret_cast<float*>(a.out);
    float* sw = stage + wave * 64 * OLD;
    const int64_t row = row0 + lane;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        if (16 * nt >= kcols) break;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) sw[(16 * rt + 4 * lq + v) * OLD + li] = acc[rt][nt][v];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row < a.n) {
            if (a.cplx_out) {
#pragma unroll
                for (int cc = 0; cc < 16; cc += 2) {
                    const int c = 16 * nt + cc;
                    if (c < kcols) {
                        const int64_t o = 2 * (row + (int64_t)(c >> 1) * a.ldo);
                        __builtin_nontemporal_store(sw[lane * OLD + cc], &out[o]);
                        __builtin_nontemporal_store(sw[lane * OLD + cc + 1], &out[o + 1]);
                    }
                }
            } else {
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) {
                    const int c = 16 * nt + cc;
                    if (c < kcols) out[row + (int64_t)c * a.ldo] = sw[lane * OLD + cc];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <typename TX, typename T, int NT>
__global__ __launch_bounds__(kThreads)
void k_project_mfma(ProjectArgs a) {
    __shared__ T stage[kStage];
    project_body<TX, T, NT>(a, blockIdx.x, stage);
}

template <int NT>
__global__ __launch_bounds__(kThreads)
void k_project_bf3(ProjectArgs a) {
    __shared__ float stage[kStage];
    project_body_bf3<NT>(a, blockIdx.x, stage);
}

// Grouped form over many streams (FP32 ring and coefficients; each item in
// FP32 or BF16x3 by its precision): block b belongs to item i with
// blk_start[i] <= b < blk_start[i+1].
template <int NT>
__global__ __launch_bounds__(kThreads)
void k_project_grouped(const ProjectArgs* __restrict__ items, const int* __restrict__ blk_start, int nitems) {
    int lo = 0, hi = nitems - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const ProjectArgs a = items[lo];
    __shared__ float stage[kStage];
    if (a.precision == 2 /* DMD_PREC_BF16X3 */) project_body_bf3<NT>(a, b - blk_start[lo], stage);
    else project_body<float, float, NT>(a, b - blk_start[lo], stage);
}

template <typename TX, typename T, int NT>
hipError_t launch_nt(const ProjectArgs& a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.n + kRowsPerBlock - 1) / kRowsPerBlock);
    hipLaunchKernelGGL((k_project_mfma<TX, T, NT>), dim3(gx), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <int NT>
hipError_t launch_bf3_nt(const ProjectArgs& a, hipStream_t s) {
    const unsigned gx = (unsigned)((a.n + kRowsPerBlock - 1) / kRowsPerBlock);
    hipLaunchKernelGGL(k_project_bf3<NT>, dim3(gx), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// Stage rows row0 .. row0 + ROWS - 1 of `ncols` ring columns, the first in
// slot `base` (wrapping at `slots`), as LDS columns 0 .. ntot - 1: put(c, r4,
// x) stores the four rows from r4 of column c.  Columns from ncols on and
// rows at or past ld read as zero.  Each thread issues kStageBatch 16-byte
// loads before it writes any of them, so a workgroup's staging costs a few
// memory round trips instead of one per load.
constexpr int kStageBatch = 16;
template <int ROWS, typename Put>
__device__ __forceinline__ void stage_columns(const float* __restrict__ ring, int64_t ld, int slots, int base,
                                              int ncols, int ntot, int64_t row0, Put put) {
    constexpr int Q = ROWS / 4;
    const int total = ntot * Q;
    for (int t0 = threadIdx.x; t0 < total; t0 += kThreads * kStageBatch) {
        float4 x[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int t = t0 + u * kThreads;
            const int c = t / Q, q = t % Q;
            x[u] = float4{0.0f, 0.0f, 0.0f, 0.0f};
            if (t < total && c < ncols && row0 + 4 * q < ld)
                x[u] = *reinterpret_cast<const float4*>(ring + (int64_t)((base + c) % slots) * ld + row0 + 4 * q);
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int t = t0 + u * kThreads;
            if (t < total) put(t / Q, 4 * (t % Q), x[u]);
        }
    }
}

template <typename TX, typename T>
hipError_t launch_tiles(const ProjectArgs& a, hipStream_t s, int kc_max) {
    if (kc_max <= 16) return launch_nt<TX, T, 1>(a, s);
    if (kc_max <= 32) return launch_nt<TX, T, 2>(a, s);
    if (kc_max <= 48) return launch_nt<TX, T, 3>(a, s);
    return launch_nt<TX, T, 4>(a, s);
}

// ---------------------------------------------------------------------------
// Modes of every window of a block push (multi-column update, Sec. 5, with
// Eq. Phi per window).  The k windows' X' are m consecutive ring columns each,
// shifted by one column per window, so together they span m+k-1 columns.  A
// workgroup stages 64 rows of those columns in LDS once (16-byte loads; ring
// rows between n and the padded length are zero) and each wavefront
// multiplies them by the coefficient matrices of windows wave, wave+4, ...:
// the ring is read once for all k windows instead of k times.  Requires k <= 64.
// BF3: each chunk of 32 window columns as three BF16 16x16x32 products
// (hi*hi + hi*lo + lo*hi) instead of eight FP32 16x16x4 steps; element e of
// a lane's 8-wide fragment is window column 4e + lane/16 of the chunk, the
// same columns the FP32 form's k-step e reads, so both stage reads hit the
// same banks.  The staged columns are split once, as (hi, lo) pairs in one
// 32-bit word, and a fragment is put together from 8 words with 8 byte
// permutes.  The coefficients of all k windows come packed in fragment order
// (k_pack_coef: FP32, or BF16 hi and lo), two 16-byte loads per fragment.
constexpr int kBlkRows = 64;
constexpr int kBlkLDR = kBlkRows + 16;  // column stride: the four k-slots of a fragment hit distinct banks
constexpr size_t kBlockLdsMax = 150 * 1024;  // dynamic LDS of the one-pass block projection

// Windows ahead whose coefficient fragments a wavefront holds (see below):
// two for the FP32 form with two or more column tiles, one otherwise.
template <int NT, bool BF3>
constexpr int kBlockAhead = (!BF3 && NT >= 2) ? 2 : 1;
// Waves per SIMD: two for the BF16x3 form with three or more column tiles
// (whose A-fragment assembly needs the registers to prefetch two chunks) and
// for the FP32 form holding two windows' fragments, three otherwise.  Two
// waves also leave a CU room for a small solve when one of its projection
// workgroups retires, so the solves of the next block push run beside the
// projection instead of after it.
template <int NT, bool BF3>
__global__ __launch_bounds__(kThreads, ((BF3 && NT >= 3) || kBlockAhead<NT, BF3> == 2) ? 2 : 3)
void k_project_block(BlockProjectArgs a) {
    extern __shared__ float dynp[];
    const BlockDesc* desc = a.desc;
    if (!desc->valid) return;
    const int m = a.m, k = a.k;
    const int ncols = m + k - 1;
    const int ncols_pad = k - 1 + 32 * ((m + 31) / 32);  // whole chunks for every window
    float* U = dynp;
    const int64_t row0 = (int64_t)blockIdx.x * kBlkRows;
    const int base = desc->base;  // slot of staged column 0, before the wrap
    const float* ring = static_cast<const float*>(a.ring);
    stage_columns<kBlkRows>(ring, a.ld, a.slots, base, ncols, ncols_pad, row0, [&](int c, int r4, float4 x) {
        if constexpr (BF3) {
            *reinterpret_cast<uint4*>(&U[c * kBlkLDR + r4]) =
                uint4{split_word(x.x), split_word(x.y), split_word(x.z), split_word(x.w)};
        } else {
            *reinterpret_cast<float4*>(&U[c * kBlkLDR + r4]) = x;
        }
    });
    __syncthreads();
    const unsigned* U32 = reinterpret_cast<const unsigned*>(U);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nq = (m + 31) / 32;

    // The coefficient fragments of a window's first PF chunks (as many as the
    // registers allow: two, one or none) are loaded before the previous
    // window's output stores: vector-memory completions are counted in issue
    // order, so a load issued after those stores could not be waited for
    // without waiting for the stores as well.
    constexpr int PF = (NT <= 3 || BF3) ? 2 : 1;
    constexpr int PA = kBlockAhead<NT, BF3>;
    auto load_frag = [&](int w, int q, Frag (&f)[NT]) {
        const uint4* fb = a.cfrag + ((size_t)(w * nq + q) * NT * 64 + lane) * 2;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            f[nt].x = fb[nt * 128];
            f[nt].y = fb[nt * 128 + 1];
        }
    };
    // acc += (window w's columns cb .. cb+31) x (their coefficient fragments).
    // Columns past m read the zero padding of the stage (and meet zero
    // coefficients), so no chunk needs masks.
    auto chunk = [&](int w, int cb, const Frag (&f)[NT], v4f (&acc)[4][NT]) {
        if constexpr (BF3) {
            v8bf bhi[NT], blo[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                bhi[nt] = __builtin_bit_cast(v8bf, f[nt].x);
                blo[nt] = __builtin_bit_cast(v8bf, f[nt].y);
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                unsigned d[8];
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) d[ks] = U32[(w + cb + 4 * ks + lk) * kBlkLDR + 16 * rt + li];
                uint4 h, l;
                h.x = __builtin_amdgcn_perm(d[1], d[0], 0x05040100u);
                h.y = __builtin_amdgcn_perm(d[3], d[2], 0x05040100u);
                h.z = __builtin_amdgcn_perm(d[5], d[4], 0x05040100u);
                h.w = __builtin_amdgcn_perm(d[7], d[6], 0x05040100u);
                l.x = __builtin_amdgcn_perm(d[1], d[0], 0x07060302u);
                l.y = __builtin_amdgcn_perm(d[3], d[2], 0x07060302u);
                l.z = __builtin_amdgcn_perm(d[5], d[4], 0x07060302u);
                l.w = __builtin_amdgcn_perm(d[7], d[6], 0x07060302u);
                const v8bf ahi = __builtin_bit_cast(v8bf, h), alo = __builtin_bit_cast(v8bf, l);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mma_bf16x3(ahi, alo, bhi[nt], blo[nt], acc[rt][nt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const float* ucol = U + (w + cb + 4 * ks + lk) * kBlkLDR;
                float bv[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const uint4& u = ks < 4 ? f[nt].x : f[nt].y;
                    const unsigned e = (ks & 3) == 0 ? u.x : (ks & 3) == 1 ? u.y : (ks & 3) == 2 ? u.z : u.w;
                    bv[nt] = __builtin_bit_cast(float, e);
                }
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const float av = ucol[16 * rt + li];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[nt], acc[rt][nt], 0, 0, 0);
                }
            }
        }
    };


    // Fragments are loaded PA windows ahead: with PA = 2 a window's stores
    // have two windows of products to complete before a wait for fragments
    // (which in issue order follows them) has to see them done.  The window
    // loop is unrolled by PA so that every fragment array is indexed
    // statically (kept in registers).
    Frag fr[PA][PF == 2 ? 2 : 1][NT];
#pragma unroll
    for (int s = 0; s < PA; ++s) {
        const int w = wave + (kThreads / 64) * s;
        if (w < k) {
            if constexpr (PF >= 1) load_frag(w, 0, fr[s][0]);
            if constexpr (PF == 2)
                if (nq > 1) load_frag(w, 1, fr[s][1]);
        }
    }
    for (int w0 = wave; w0 < k; w0 += (kThreads / 64) * PA) {
#pragma unroll
    for (int s = 0; s < PA; ++s) {
        const int w = w0 + (kThreads / 64) * s;
        if (w >= k) break;
        const int kc = desc->kc[w];
        v4f acc[4][NT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = v4f{0, 0, 0, 0};
        if (kc > 0) {
            if constexpr (PF >= 1) chunk(w, 0, fr[s][0], acc);
            if constexpr (PF == 2)
                if (nq > 1) chunk(w, 32, fr[s][1], acc);
            for (int q = PF; q < nq; ++q) {
                Frag g[NT];
                load_frag(w, q, g);
                chunk(w, 32 * q, g, acc);
            }
        }
        const int wn = w + (kThreads / 64) * PA;
        if (wn < k) {
            if constexpr (PF >= 1) load_frag(wn, 0, fr[s][0]);
            if constexpr (PF == 2)
                if (nq > 1) load_frag(wn, 1, fr[s][1]);
        }
        if (kc == 0) continue;  // unsolved window: its output is left untouched
        // Output straight from the accumulators: lane (li, lq) of tile (rt, nt)
        // holds rows 16 rt + 4 lq + v (v = 0..3) of real column 16 nt + li,
        // i.e. the real (li even) or imaginary (li odd) part of complex column
        // 8 nt + li/2.  One swap with the neighbouring lane gives the even lane
        // rows v = 0, 1 and the odd lane rows v = 2, 3 as whole complex values:
        // two consecutive rows, one 16-byte store.  The stores are
        // nontemporal: the modes are not read again here, and streaming them
        // past the caches keeps the window columns and the solves' data of
        // the next block, which run beside this kernel, cached.
        float2* out = a.out + (int64_t)w * a.ldw;
        const bool odd = li & 1;
        const int r_eff = kc >> 1;
        // 16-byte stores where the layout allows and all 64 rows exist (uniform)
        auto store = [&](auto fast) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int j = 8 * nt + (li >> 1);
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const v4f d = acc[rt][nt];
                    const float x = odd ? d[0] : d[2], y = odd ? d[1] : d[3];
                    const float xs = swap_pair(x), ys = swap_pair(y);
                    const float4 val = odd ? float4{xs, d[2], ys, d[3]} : float4{d[0], xs, d[1], ys};
                    const int64_t row = row0 + 16 * rt + 4 * lk + (odd ? 2 : 0);
                    float2* o = out + row + (int64_t)j * a.ldo;
                    if constexpr (decltype(fast)::value) {
                        if (j < r_eff)
                            __builtin_nontemporal_store(v4f{val.x, val.y, val.z, val.w}, reinterpret_cast<v4f*>(o));
                    } else if (j < r_eff && row < a.n) {
                        o[0] = float2{val.x, val.y};
                        if (row + 1 < a.n) o[1] = float2{val.z, val.w};
                    }
                }
            }
        };
        if (a.out16 && row0 + kBlkRows <= a.n) store(std::true_type{});
        else store(std::false_type{});
    }
    }
}

// Coefficients of the k windows of a block push in the B-fragment order of
// k_project_block: entry ((w nq + q) NT + nt) 64 + lane holds the 8 values
// C[32 q + 4 e + lane/16][16 nt + lane%16], e = 0..7, of window w (zero
// outside m x 2 r_eff and for unsolved windows), as 8 floats, or for BF3 as
// their 8 BF16 hi parts followed by their 8 BF16 lo parts.
template <int NT, bool BF3>
__global__ __launch_bounds__(64)
void k_pack_coef(BlockProjectArgs a) {
    const int lane = threadIdx.x;
    const int nt = blockIdx.x % NT, q = blockIdx.x / NT, w = blockIdx.y;
    const int nq = (a.m + 31) / 32;
    const int k = a.k;
    const int set = a.kmax - k + w;
    const DevState* st =
        w == k - 1 ? a.st : reinterpret_cast<const DevState*>(a.shadow + (size_t)set * a.shadow_stride);
    const int kc = (st->solve_status == ST_OK || st->solve_status == ST_W_RANK) ? 2 * st->r_eff : 0;
    const float* B = w == k - 1 ? a.Bphi : a.Bphi_sets + (int64_t)set * a.bphi_stride;
    const int li = lane & 15, lk = lane >> 4;
    const int c = 16 * nt + li;
    if (blockIdx.x == 0 && lane == 0) {
        a.desc->kc[w] = kc;
        if (w == k - 1) {
            a.desc->valid = a.st->count >= a.m + 1 && !a.st->block_rejected;
            a.desc->base = a.st->oldest + 2 - k + a.slots;
        }
    }
    float y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int col = 32 * q + 4 * e + lk;
        y[e] = (col < a.m && c < kc) ? B[(int64_t)col * (2 * a.r) + c] : 0.0f;
    }
    uint4* out = a.cfrag + ((size_t)(w * nq + q) * NT * 64 + nt * 64 + lane) * 2;
    if constexpr (BF3) {
        v8bf hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 h, l;
            split_bf16(y[e], h, l);
            hi[e] = h;
            lo[e] = l;
        }
        out[0] = __builtin_bit_cast(uint4, hi);
        out[1] = __builtin_bit_cast(uint4, lo);
    } else {
        out[0] = uint4{__builtin_bit_cast(unsigned, y[0]), __builtin_bit_cast(unsigned, y[1]),
                       __builtin_bit_cast(unsigned, y[2]), __builtin_bit_cast(unsigned, y[3])};
        out[1] = uint4{__builtin_bit_cast(unsigned, y[4]), __builtin_bit_cast(unsigned, y[5]),
                       __builtin_bit_cast(unsigned, y[6]), __builtin_bit_cast(unsigned, y[7])};
    }
}

// ---------------------------------------------------------------------------
// FP32 block projection over window pairs.  When 2 r = 8 (mod 16) the real
// columns of one window fill NT tiles of 16 only partly (r = 20: 40 of 48),
// but two windows fill 4r/16 tiles exactly.  Windows 2p and 2p+1 read stage
// columns one apart, so as one product they read the m + 1 columns 2p ..
// 2p + m against a pair matrix P (rows i = 0 .. m, columns 0 .. 4r - 1):
// P[i][c] = C_2p[i][c] (c < 2r, i < m) and C_2p+1[i - 1][c - 2r] (c >= 2r,
// i >= 1), zero elsewhere.  The pair costs ceil((m + 1) / 4) k-steps of 4r/16
// tiles instead of 2 (m / 4) steps of ceil(2r / 16) tiles (r = 12, m = 32:
// 4 x 27 MFMAs per 64 rows instead of 4 x 32).  k-steps come as chunks of
// eight (two 16-byte loads per lane and tile) plus at most one single step.
// Up to three tiles (r = 4, 12): with five (r = 20) the pair's accumulators
// and fragments take all 256 registers of two waves per SIMD, and although
// the product itself is faster, the next block's solves then find no room on
// the CUs and run after it instead of beside it (measured: the per-window
// form with two windows of fragments in flight wins there).
constexpr int kPairMaxTiles = 3;
// With the pair form asked for by the stream's tuned shape (measured in the
// pipeline by dmd_tune), up to five tiles (r = 20).
constexpr int kPairMaxTilesTuned = 5;

struct PairShape {
    int nfull;  // whole 8-step chunks
    int tail;   // single steps after them (0 or 1)
};
__host__ __device__ inline PairShape pair_shape(int m) {
    const int nsteps = (m + 1 + 3) / 4;
    return PairShape{nsteps / 8, nsteps % 8};
}
// Whether the pair form applies: FP32, 2r = 8 mod 16, at least one whole
// chunk and at most one tail step, and at most kPairMaxTiles tiles (the rule,
// form 0) or kPairMaxTilesTuned (form 2); never for form 1.
bool use_pairs(const BlockProjectArgs& a) {
    if (a.bf16x3 || a.form == 1) return false;
    const int tiles = 4 * a.r / 16;
    const PairShape ps = pair_shape(a.m);
    if ((2 * a.r) % 16 != 8 || ps.nfull < 1 || ps.tail > 1) return false;
    return tiles <= (a.form == 2 ? kPairMaxTilesTuned : kPairMaxTiles);
}
size_t pair_lds(int m, int k) {
    const PairShape ps = pair_shape(m);
    return sizeof(float) * (size_t)(k + 1 + 4 * (8 * ps.nfull + ps.tail)) * kBlkLDR;
}

// Coefficients of window w of the block (m x 2 r row-major) and 2 r_eff, 0 if
// the window has no solve.
__device__ inline const float* window_coef(const BlockProjectArgs& a, int w, int& kc) {
    const int set = a.kmax - a.k + w;
    const DevState* st =
        w == a.k - 1 ? a.st : reinterpret_cast<const DevState*>(a.shadow + (size_t)set * a.shadow_stride);
    kc = (st->solve_status == ST_OK || st->solve_status == ST_W_RANK) ? 2 * st->r_eff : 0;
    return w == a.k - 1 ? a.Bphi : a.Bphi_sets + (int64_t)set * a.bphi_stride;
}

// Packs P of pair p = blockIdx.y, tile t = blockIdx.x.  Pair p starts at
// float p (8 nfull + tail) NTG 64; in it, float ((q NTG + t) 64 + lane) 8 + e
// of chunk q holds P[32 q + 4 e + lane/16][16 t + lane%16] (e = 0..7: one
// lane's eight steps, two 16-byte loads), and after the chunks float
// t 64 + lane of the tail step holds P[32 nfull + lane/16][16 t + lane%16].
template <int NTG>
__global__ __launch_bounds__(64)
void k_pack_pair(BlockProjectArgs a) {
    const int lane = threadIdx.x, t = blockIdx.x, p = blockIdx.y;
    const int li = lane & 15, lk = lane >> 4;
    const int k = a.k, m = a.m, r2 = 2 * a.r;
    const PairShape ps = pair_shape(m);
    const int w0 = 2 * p, w1 = 2 * p + 1;
    int kc0 = 0, kc1 = 0;
    const float* B0 = window_coef(a, w0, kc0);
    const float* B1 = w1 < k ? window_coef(a, w1, kc1) : nullptr;
    if (t == 0 && lane == 0) {
        a.desc->kc[w0] = kc0;
        if (w1 < k) a.desc->kc[w1] = kc1;
        if (w0 == k - 1 || w1 == k - 1) {
            a.desc->valid = a.st->count >= a.m + 1 && !a.st->block_rejected;
            a.desc->base = a.st->oldest + 2 - k + a.slots;
        }
    }
    const int c = 16 * t + li;
    auto P = [&](int i) -> float {
        if (c < r2) return (i < m && c < kc0) ? B0[(int64_t)i * r2 + c] : 0.0f;
        const int cc = c - r2;
        return (w1 < k && i >= 1 && i <= m && cc < kc1) ? B1[(int64_t)(i - 1) * r2 + cc] : 0.0f;
    };
    const size_t pair_base = (size_t)p * (8 * ps.nfull + ps.tail) * NTG * 64;
    float* out = reinterpret_cast<float*>(a.cfrag) + pair_base;
    for (int q = 0; q < ps.nfull; ++q) {
        float* o = out + (((size_t)q * NTG + t) * 64 + lane) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = P(32 * q + 4 * e + lk);
    }
    if (ps.tail) out[((size_t)8 * ps.nfull * NTG + t) * 64 + lane] = P(32 * ps.nfull + lk);
}

template <int NTG>
__global__ __launch_bounds__(kThreads, 2)
void k_project_pair(BlockProjectArgs a) {
    extern __shared__ float dynp[];
    const BlockDesc* desc = a.desc;
    if (!desc->valid) return;
    const int m = a.m, k = a.k, r2 = 2 * a.r;
    const PairShape ps = pair_shape(m);
    const int nst = 8 * ps.nfull + ps.tail;
    const int ncols = m + k - 1;
    const int ncols_pad = k + 1 + 4 * nst;  // the last pair's steps read zero columns past the union
    float* U = dynp;
    const int64_t row0 = (int64_t)blockIdx.x * kBlkRows;
    const int base = desc->base;
    const float* ring = static_cast<const float*>(a.ring);
    stage_columns<kBlkRows>(ring, a.ld, a.slots, base, ncols, ncols_pad, row0,
                            [&](int c, int r4, float4 x) { *reinterpret_cast<float4*>(&U[c * kBlkLDR + r4]) = x; });
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int npairs = (k + 1) / 2;
    const float* cf = reinterpret_cast<const float*>(a.cfrag);
    const size_t pair_stride = (size_t)nst * NTG * 64;
    // Chunk 0 and the tail step of a pair are loaded one pair ahead (before
    // the previous pair's stores, so waiting for them does not wait for
    // those); every later chunk at the top of the pair's iteration, a chunk
    // of products ahead of its use.
    Frag f0[NTG];
    float ft[NTG];
    auto load_chunk = [&](int p, int q, Frag (&f)[NTG]) {
        const float* pb = cf + (size_t)p * pair_stride;
#pragma unroll
        for (int t = 0; t < NTG; ++t) {
            const uint4* g = reinterpret_cast<const uint4*>(pb + (((size_t)q * NTG + t) * 64 + lane) * 8);
            f[t].x = g[0];
            f[t].y = g[1];
        }
    };
    auto load = [&](int p) {
        load_chunk(p, 0, f0);
        const float* pb = cf + (size_t)p * pair_stride;
#pragma unroll
        for (int t = 0; t < NTG; ++t) ft[t] = ps.tail ? pb[((size_t)8 * ps.nfull * NTG + t) * 64 + lane] : 0.0f;
    };
    // acc += stage columns c0 + 4 s + lk (s = 0..7) x the chunk's coefficients
    auto chunk = [&](int c0, const Frag (&f)[NTG], v4f (&acc)[4][NTG]) {
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const float* ucol = U + (c0 + 4 * ks + lk) * kBlkLDR;
            float bv[NTG];
#pragma unroll
            for (int t = 0; t < NTG; ++t) {
                const uint4& u = ks < 4 ? f[t].x : f[t].y;
                const unsigned e = (ks & 3) == 0 ? u.x : (ks & 3) == 1 ? u.y : (ks & 3) == 2 ? u.z : u.w;
                bv[t] = __builtin_bit_cast(float, e);
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const float av = ucol[16 * rt + li];
#pragma unroll
                for (int t = 0; t < NTG; ++t)
                    acc[rt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[t], acc[rt][t], 0, 0, 0);
            }
        }
    };
    if (wave < npairs) load(wave);
    for (int p = wave; p < npairs; p += kThreads / 64) {
        const int w0 = 2 * p, w1 = 2 * p + 1;
        const int kc0 = desc->kc[w0], kc1 = w1 < k ? desc->kc[w1] : 0;
        v4f acc[4][NTG];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int t = 0; t < NTG; ++t) acc[rt][t] = v4f{0, 0, 0, 0};
        if (kc0 + kc1 > 0) {
            Frag g[NTG];
            if (ps.nfull > 1) load_chunk(p, 1, g);
            chunk(w0, f0, acc);
            for (int q = 1; q < ps.nfull; ++q) {
                chunk(w0 + 32 * q, g, acc);
                if (q + 1 < ps.nfull) load_chunk(p, q + 1, g);
            }
            if (ps.tail) {
                const float* ucol = U + (w0 + 32 * ps.nfull + lk) * kBlkLDR;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const float av = ucol[16 * rt + li];
#pragma unroll
                    for (int t = 0; t < NTG; ++t)
                        acc[rt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ft[t], acc[rt][t], 0, 0, 0);
                }
            }
        }
        if (p + kThreads / 64 < npairs) load(p + kThreads / 64);
        if (kc0 + kc1 == 0) continue;
        // Stores as in k_project_block: one swap with the neighbouring lane
        // gives whole complex values of two consecutive rows; real column
        // 16 t + li of the pair is column (16 t + li) of window 2p below 2 r,
        // of window 2p + 1 above (r is even here, so a tile's lane pairs never
        // straddle the two).
        const bool odd = li & 1;
        auto store = [&](auto full) {
#pragma unroll
            for (int t = 0; t < NTG; ++t) {
                const int c = 16 * t + li;
                const bool second = c >= r2;
                const int w = second ? w1 : w0;
                const int j = (second ? c - r2 : c) >> 1;
                const int r_eff = (second ? kc1 : kc0) >> 1;
                float2* out = a.out + (int64_t)w * a.ldw;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const v4f d = acc[rt][t];
                    const float x = odd ? d[0] : d[2], y = odd ? d[1] : d[3];
                    const float xs = swap_pair(x), ys = swap_pair(y);
                    const float4 val = odd ? float4{xs, d[2], ys, d[3]} : float4{d[0], xs, d[1], ys};
                    const int64_t row = row0 + 16 * rt + 4 * lk + (odd ? 2 : 0);
                    float2* o = out + row + (int64_t)j * a.ldo;
                    if constexpr (decltype(full)::value) {
                        if (j < r_eff)
                            __builtin_nontemporal_store(v4f{val.x, val.y, val.z, val.w}, reinterpret_cast<v4f*>(o));
                    } else if (j < r_eff && row < a.n) {
                        o[0] = float2{val.x, val.y};
                        if (row + 1 < a.n) o[1] = float2{val.z, val.w};
                    }
                }
            }
        };
        if (a.out16 && row0 + kBlkRows <= a.n) store(std::true_type{});
        else store(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// FP32 block projection as one banded product.  The real output columns of
// the k windows, 2r per window, side by side form K = 2 r k columns; column
// g = 2 r w + c (window w, real column c) is the product of stage columns
// w .. w + m - 1 with C_w[.][c].  So all k windows are one product of the
// staged columns by a band matrix B[i][g] = C_w[i - w][c] (0 <= i - w < m,
// zero elsewhere), and a 32-column tile t of B, touching windows
// w_lo .. w_hi, is nonzero only in rows w_lo .. w_hi + m - 1: it costs
// ceil((m + w_hi - w_lo) / 2) steps of the 32x32x2 FP32 matrix instruction.
// With 2r >= 32 a tile touches at most two windows, so the executed work is
// within one row per tile of the algorithmic work for any r (r = 20, m = 64:
// 33 or 32 steps a tile; one product per window in 16-column tiles executes
// 48/40 of it).
// A workgroup stages 128 rows of the m + k - 1 columns (and a zero column);
// wavefront v takes tiles v, v + 4, ...: per step one packed B value per
// lane and four A fragments (one per 32-row tile) from the stage.
// Fragment layouts of v_mfma_f32_32x32x2f32: A: lane l holds A[l % 32][l / 32];
// B: lane l holds B[l / 32][l % 32]; D: lane l holds
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32], v = 0..15.
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int kBandRows = 128;
constexpr int kBandLDR = kBandRows + 32;  // 640-byte column stride: the two half-waves' columns on distinct banks

__host__ __device__ inline int band_tiles(int r, int k) { return (2 * r * k + 31) / 32; }
// Packed 8-step chunks per tile (the bound on the steps of any tile).
__host__ __device__ inline int band_chunks(int m, int r) {
    const int r2 = 2 * r;
    const int smax = (m + 31 / r2 + 1 + 1) / 2;
    return (smax + 7) / 8;
}
// Staged columns: the m + k - 1 ring columns, one zero column that the last
// step of an odd-length tile reads, and two more for the one-step read ahead.
__host__ __device__ inline int band_stage_cols(int m, int k) { return m + k + 2; }
size_t band_lds(int m, int k) { return sizeof(float) * (size_t)band_stage_cols(m, k) * kBandLDR; }
// Steps of the longest tile, and the stage of the fixed-step kernel: a tile
// from window w_lo reads columns up to w_lo + 2 S + 1 (one step read ahead).
__host__ __device__ inline int band_max_steps(int m, int r, int k) {
    int smax = 0;
    const int r2 = 2 * r;
    for (int t = 0; t < band_tiles(r, k); ++t) {
        const int wl = 32 * t / r2, wh = min((32 * t + 31) / r2, k - 1);
        const int s = (m + wh - wl + 1) / 2;
        smax = s > smax ? s : smax;
    }
    return smax;
}
__host__ __device__ inline int band_s_stage_cols(int m, int k, int S) {
    const int need = k + 2 * S + 1;
    return need > band_stage_cols(m, k) ? need : band_stage_cols(m, k);
}

// Packs tile t = blockIdx.x, chunk q = blockIdx.y: float ((t nch + q) 64 +
// lane) 8 + e holds B[w_lo + 2 (8 q + e) + lane / 32][32 t + lane % 32].
__global__ __launch_bounds__(64)
void k_pack_band(BlockProjectArgs a) {
    const int lane = threadIdx.x, t = blockIdx.x, q = blockIdx.y;
    const int k = a.k, m = a.m, r2 = 2 * a.r;
    const int nch = band_chunks(m, a.r);
    if (t == 0 && q == 0) {
        for (int w = lane; w < k; w += 64) {
            int kc = 0;
            window_coef(a, w, kc);
            a.desc->kc[w] = kc;
        }
        if (lane == 0) {
            a.desc->valid = a.st->count >= a.m + 1 && !a.st->block_rejected;
            a.desc->base = a.st->oldest + 2 - k + a.slots;
        }
    }
    const int wlo = 32 * t / r2;
    const int g = 32 * t + (lane & 31);
    const int w = g / r2, c = g % r2;
    int kc = 0;
    const float* B = w < k ? window_coef(a, w, kc) : nullptr;
    float y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int i = wlo + 2 * (8 * q + e) + (lane >> 5) - w;  // row of C_w
        y[e] = (w < k && c < kc && i >= 0 && i < m) ? B[(int64_t)i * r2 + c] : 0.0f;
    }
    uint4* out = a.cfrag + ((size_t)(t * nch + q) * 64 + lane) * 2;
    out[0] = uint4{__builtin_bit_cast(unsigned, y[0]), __builtin_bit_cast(unsigned, y[1]),
                   __builtin_bit_cast(unsigned, y[2]), __builtin_bit_cast(unsigned, y[3])};
    out[1] = uint4{__builtin_bit_cast(unsigned, y[4]), __builtin_bit_cast(unsigned, y[5]),
                   __builtin_bit_cast(unsigned, y[6]), __builtin_bit_cast(unsigned, y[7])};
}

__global__ __launch_bounds__(kThreads, 2)
void k_project_band(BlockProjectArgs a) {
    extern __shared__ float dynp[];
    const BlockDesc* desc = a.desc;
    if (!desc->valid) return;
    const int m = a.m, k = a.k, r2 = 2 * a.r;
    const int ncols = m + k - 1, nstage = band_stage_cols(m, k);
    const int ntile = band_tiles(a.r, k), nch = band_chunks(m, a.r);
    float* U = dynp;
    const int64_t row0 = (int64_t)blockIdx.x * kBandRows;
    const int base = desc->base;
    const float* ring = static_cast<const float*>(a.ring);
    stage_columns<kBandRows>(ring, a.ld, a.slots, base, ncols, nstage, row0,
                             [&](int c, int r4, float4 x) { *reinterpret_cast<float4*>(&U[c * kBandLDR + r4]) = x; });
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const bool odd = li & 1;
    const uint4* cf = a.cfrag + (size_t)lane * 2;
    auto load = [&](int t, int q, uint4 (&f)[2]) {
        const uint4* p = cf + (size_t)(t * nch + q) * 128;
        f[0] = p[0];
        f[1] = p[1];
    };
    // A fragments of one step: stage column c + lh, rows 32 rt + li
    auto load_a = [&](int c, float (&av)[4]) {
        const float* u = U + (c + lh) * kBandLDR + li;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) av[rt] = u[32 * rt];
    };
    auto bval = [](const uint4 (&f)[2], int e) {
        const uint4& u = e < 4 ? f[0] : f[1];
        const unsigned bits = (e & 3) == 0 ? u.x : (e & 3) == 1 ? u.y : (e & 3) == 2 ? u.z : u.w;
        return __builtin_bit_cast(float, bits);
    };
    // One step: acc += (A of column c) x b, with the next step's A fragments
    // (column c + 2) read from the stage before the products are issued, so
    // that the LDS latency hides behind them.  The stage holds two zero
    // columns past the last one any tile reads, for the read ahead.
    auto step = [&](int& c, float (&av)[4], float bv, v16f (&acc)[4]) {
        float an[4];
        load_a(c + 2, an);
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rt], bv, acc[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) av[rt] = an[rt];
        c += 2;
    };
    // Coefficient chunks ping-pong between two register sets (no copies, so
    // no wait for a chunk before its turn): chunks 0 and 1 of a tile are
    // loaded before the previous tile's stores, chunk q + 2 into the set
    // chunk q has just left.
    uint4 fa[2], fb[2];
    auto prefetch = [&](int t) {
        const int g0 = 32 * t;
        const int wl = g0 / r2, wh = min((g0 + 31) / r2, k - 1);
        load(t, 0, fa);
        if ((m + wh - wl + 1) / 2 > 8) load(t, 1, fb);
    };
    // steps with the values of chunk set f, then refill it with chunk qn
    auto chunk8 = [&](int& c, float (&av)[4], uint4 (&f)[2], v16f (&acc)[4], int t, int qn, int nq) {
#pragma unroll
        for (int e = 0; e < 8; ++e) step(c, av, bval(f, e), acc);
        if (qn < nq) load(t, qn, f);
    };
    auto tail = [&](int& c, float (&av)[4], const uint4 (&f)[2], v16f (&acc)[4], int ntail) {
        for (int e = 0; e < ntail; ++e) {
            const float bv = e == 0 ? bval(f, 0) : e == 1 ? bval(f, 1) : e == 2 ? bval(f, 2) :
                             e == 3 ? bval(f, 3) : e == 4 ? bval(f, 4) : e == 5 ? bval(f, 5) : bval(f, 6);
            step(c, av, bv, acc);
        }
    };
    if (wave < ntile) prefetch(wave);
    for (int t = wave; t < ntile; t += kThreads / 64) {
        // tile quantities as scalars: every branch below is uniform
        const int g0 = 32 * t;
        const int wlo = __builtin_amdgcn_readfirstlane(g0 / r2);
        const int whi = __builtin_amdgcn_readfirstlane(min((g0 + 31) / r2, k - 1));
        int live = 0;
        for (int w = wlo; w <= whi; ++w) live |= desc->kc[w];
        live = __builtin_amdgcn_readfirstlane(live);
        const int nsteps = (m + whi - wlo + 1) / 2;
        const int nfull = nsteps >> 3, ntail = nsteps & 7;
        const int nq = nfull + (ntail ? 1 : 0);
        v16f acc[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[rt][v] = 0.0f;
        if (live) {
            int c = wlo;
            float av[4];
            load_a(c, av);
            int q = 0;
            for (; q + 1 < nfull; q += 2) {
                chunk8(c, av, fa, acc, t, q + 2, nq);
                chunk8(c, av, fb, acc, t, q + 3, nq);
            }
            if (q < nfull) {  // odd number of whole chunks: the last one is in fa, the tail in fb
                chunk8(c, av, fa, acc, t, nq, nq);
                tail(c, av, fb, acc, ntail);
            } else {
                tail(c, av, fa, acc, ntail);
            }
        }
        // the next tile's first chunks before this tile's stores
        if (t + kThreads / 64 < ntile) prefetch(t + kThreads / 64);
        if (!live) continue;
        // Lane (li, lh) holds rows 32 rt + 8 gq + 4 lh + v (v = 0..3) of real
        // column g0 + li; one swap with the neighbouring lane gives the even
        // lane rows v = 0, 1 and the odd lane rows v = 2, 3 as whole complex
        // values (2 r is even, so a lane pair never straddles two windows).
        const int g = g0 + li;
        const int w = g / r2, c = g % r2;
        const bool ok = w < k && c < desc->kc[w < k ? w : 0];
        float2* out = a.out + (int64_t)(w < k ? w : 0) * a.ldw + (int64_t)(c >> 1) * a.ldo;
        auto store = [&](auto full) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const float d0 = acc[rt][4 * gq], d1 = acc[rt][4 * gq + 1];
                    const float d2 = acc[rt][4 * gq + 2], d3 = acc[rt][4 * gq + 3];
                    const float x = odd ? d0 : d2, y = odd ? d1 : d3;
                    const float xs = swap_pair(x), ys = swap_pair(y);
                    const float4 val = odd ? float4{xs, d2, ys, d3} : float4{d0, xs, d1, ys};
                    const int64_t row = row0 + 32 * rt + 8 * gq + 4 * lh + (odd ? 2 : 0);
                    float2* o = out + row;
                    if constexpr (decltype(full)::value) {
                        if (ok) __builtin_nontemporal_store(v4f{val.x, val.y, val.z, val.w}, reinterpret_cast<v4f*>(o));
                    } else if (ok && row < a.n) {
                        o[0] = float2{val.x, val.y};
                        if (row + 1 < a.n) o[1] = float2{val.z, val.w};
                    }
                }
        };
        if (a.out16 && row0 + kBandRows <= a.n) store(std::true_type{});
        else store(std::false_type{});
    }
}

// The banded product with a fixed number S of steps per tile (S = the longest
// tile's steps rounded up to an instance, at most 36: m up to about 70).
// Every tile runs the same straight-line sequence of products (a shorter
// tile meets zero coefficients in its last steps), and a tile's S values per
// lane are held in registers, loaded one tile ahead (two register sets in
// turn, the tile loop unrolled by two, the first tile peeled), so no load or
// branch sits between the products.  Output in runs of 128 bytes per complex
// column: the two 8-row groups gq = 2p, 2p + 1 are exchanged between 16-lane
// rows (v_permlane16_swap: odd rows of the first operand with even rows of
// the second), so that one store writes rows 16 p .. 16 p + 15 of eight
// complex columns, whole 128-byte lines, instead of 8 rows of sixteen.  The
// waits for the loads ahead can only be counted exactly when no branch
// skips a vector memory instruction: hence the fixed step count, every tile
// computed, stores that always issue (masked lanes write a sink) and the
// window ranks read from LDS.
__device__ __forceinline__ float4 band_pair(const v16f& d, int gq, bool odd) {
    // lane (li, lh): rows 8 gq + 4 lh + v of real column li; after one swap
    // with the neighbouring lane, two whole complex rows (v = 0, 1 on the
    // even lane, v = 2, 3 on the odd one)
    const float d0 = d[4 * gq], d1 = d[4 * gq + 1], d2 = d[4 * gq + 2], d3 = d[4 * gq + 3];
    const float x = odd ? d0 : d2, y = odd ? d1 : d3;
    const float xs = swap_pair(x), ys = swap_pair(y);
    return odd ? float4{xs, d2, ys, d3} : float4{d0, xs, d1, ys};
}
__device__ __forceinline__ void swap16(float& x, float& y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                   false, false);
    x = __builtin_bit_cast(float, (unsigned)r[0]);
    y = __builtin_bit_cast(float, (unsigned)r[1]);
}

// FULL: every row slab of the launch is whole and the output allows 16-byte
// stores (one store instruction per row pair and column group, whatever the
// data: the waits for the loads ahead are then counted exactly); the last,
// partial slab runs as a launch of its own with FULL = false.
template <int S, bool FULL>
__global__ __launch_bounds__(kThreads, 2)
void k_project_band_s(BlockProjectArgs a, int64_t slab0) {
    constexpr int NQ = (S + 3) / 4;  // 16-byte coefficient loads per lane and tile
    extern __shared__ float dynp[];
    const BlockDesc* desc = a.desc;
    if (!desc->valid) return;
    const int m = a.m, k = a.k, r2 = 2 * a.r;
    const int ncols = m + k - 1, nstage = band_s_stage_cols(m, k, S);
    const int nch = band_chunks(m, a.r);
    const int ntile = band_tiles(a.r, k);
    float* U = dynp;
    const int64_t row0 = (slab0 + blockIdx.x) * kBandRows;
    const int base = desc->base;
    const float* ring = static_cast<const float*>(a.ring);
    // the windows' ranks in LDS: reading them never waits on vector memory
    __shared__ int s_kc[64];
    if (threadIdx.x < 64) s_kc[threadIdx.x] = threadIdx.x < k ? desc->kc[threadIdx.x] : 0;
    stage_columns<kBandRows>(ring, a.ld, a.slots, base, ncols, nstage, row0,
                             [&](int c, int r4, float4 x) { *reinterpret_cast<float4*>(&U[c * kBandLDR + r4]) = x; });
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const bool odd = li & 1;
    const uint4* cf = a.cfrag + (size_t)lane * 2;
    auto load_a = [&](int c, float (&av)[4]) {
        const float* u = U + (c + lh) * kBandLDR + li;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) av[rt] = u[32 * rt];
    };
    auto bval = [](const uint4 (&b)[NQ], int st) {
        const uint4& u = b[st / 4];
        const unsigned bits = (st & 3) == 0 ? u.x : (st & 3) == 1 ? u.y : (st & 3) == 2 ? u.z : u.w;
        return __builtin_bit_cast(float, bits);
    };
    struct Tile {
        int g0, wlo, nsteps;
    };
    auto tile_of = [&](int t) {
        Tile T;
        T.g0 = 32 * t;
        T.wlo = __builtin_amdgcn_readfirstlane(T.g0 / r2);
        const int whi = __builtin_amdgcn_readfirstlane(min((T.g0 + 31) / r2, k - 1));
        T.nsteps = S;
        (void)whi;
        return T;
    };
    // the tile's S steps of values, four per 16-byte load (chunk q of the
    // packed layout holds steps 8 q .. 8 q + 7 as two such loads); steps
    // past a tile's own count hold zeros
    auto load_b = [&](int t, uint4 (&b)[NQ]) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) b[i] = cf[(size_t)(t * nch + i / 2) * 128 + (i & 1)];
    };
    auto step = [&](int& c, float (&av)[4], float bv, v16f (&acc)[4]) {
        float an[4];
        load_a(c + 2, an);  // the next step's A fragments ahead of the products
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rt], bv, acc[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) av[rt] = an[rt];
        c += 2;
    };
    // Every tile is computed (a tile of unsolved windows has zero
    // coefficients and stores nothing), so that no branch skips vector
    // memory instructions and the waits for the loads ahead stay exact.
    auto tile = [&](int t, const uint4 (&b)[NQ]) {
        const Tile T = tile_of(t);
        v16f acc[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[rt][v] = 0.0f;
        int c = T.wlo;
        float av[4];
        load_a(c, av);
        // every tile takes S steps (straight-line code, no branch between the
        // products): a tile with fewer meets zero coefficients in the rest
#pragma unroll
        for (int st = 0; st < S; ++st) step(c, av, bval(b, st), acc);
        // the two complex columns of this lane's stores: jA = (lane % 16) / 2
        // and jA + 8 of the tile (real columns g0 + 2 j, g0 + 2 j + 1)
        const int jA = (lane & 15) >> 1;
        float2* o[2];
        bool ok[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int g = T.g0 + 2 * (jA + 8 * h);
            const int w = g / r2, cc = g % r2;
            const int ws = w < k ? w : 0;
            ok[h] = w < k && cc < s_kc[ws];
            o[h] = a.out + (int64_t)ws * a.ldw + (int64_t)(cc >> 1) * a.ldo;
        }
        const int rsub = 8 * ((lane >> 4) & 1) + 4 * lh + (odd ? 2 : 0);
        v4f* sink = reinterpret_cast<v4f*>(a.desc->sink) + lane;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                float4 x = band_pair(acc[rt], 2 * p, odd), y = band_pair(acc[rt], 2 * p + 1, odd);
                swap16(x.x, y.x);
                swap16(x.y, y.y);
                swap16(x.z, y.z);
                swap16(x.w, y.w);
                const int64_t row = row0 + 32 * rt + 16 * p + rsub;
                const float4 val[2] = {x, y};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float2* q = o[h] + row;
                    if constexpr (FULL) {
                        // unconditional: lanes whose column is past the
                        // window's rank (or past the last window) write the
                        // descriptor's sink, so no branch skips a store
                        v4f* dst = ok[h] ? reinterpret_cast<v4f*>(q) : sink;
                        __builtin_nontemporal_store(v4f{val[h].x, val[h].y, val[h].z, val[h].w}, dst);
                    } else if (ok[h] && row < a.n) {
                        q[0] = float2{val[h].x, val[h].y};
                        if (row + 1 < a.n) q[1] = float2{val[h].z, val[h].w};
                    }
                }
            }
    };
    constexpr int T4 = kThreads / 64;
    uint4 bA[NQ], bB[NQ];
    // the next tile's values (the last tile's again past the end: loads are
    // never skipped)
    auto ahead = [&](int t) { return t + T4 < ntile ? t + T4 : ntile - 1; };
    int t = wave;
    if (t >= ntile) return;
    load_b(t, bA);
    // (the scheduling barriers keep the loads ahead where they are issued;
    // the first tile is peeled so that every tile in the loop follows the
    // same pattern of stores and loads, and its waits are counted exactly)
    load_b(ahead(t), bB);
    __builtin_amdgcn_sched_barrier(0);
    tile(t, bA);
    t += T4;
    while (t < ntile) {
        load_b(ahead(t), bA);
        __builtin_amdgcn_sched_barrier(0);
        tile(t, bB);
        t += T4;
        if (t >= ntile) break;
        load_b(ahead(t), bB);
        __builtin_amdgcn_sched_barrier(0);
        tile(t, bA);
        t += T4;
    }
}

// The banded product on v_mfma_f32_16x16x4f32 (the form run wherever one of
// its fixed-step instances applies).  Same 32-column tiles, windows and
// stores as above, but each step covers 4 staged columns with 16 products
// (8 row tiles of 16 x 2 column tiles of 16) instead of 2 columns with 4
// products of 32 x 32: the 16 x 16 products keep the matrix cores busier
// (a probe of the products alone sustains 155-157 TFLOP/s against 129 for
// 32 x 32 products rotating over four accumulators).  Lane l holds
// A[l % 16][l / 16] (row, staged column), B[l / 16][l % 16] (staged column,
// output column) and D[4 (l / 16) + v][l % 16]; one swap with the neighbouring
// lane gives each lane two whole complex rows, and one store instruction
// writes 16 rows of 8 complex columns (128-byte runs).
constexpr int kBand16LDR = kBandRows + 16;  // 576-byte stride: the 4 columns a step reads on distinct banks
// packed values per lane and tile: steps x 2 column tiles, in 16-byte groups
__host__ __device__ inline int band16_nq(int S4) { return (2 * S4 + 3) / 4; }
// a tile from window w_lo reads columns w_lo .. w_lo + 4 S4 - 1 and one step ahead
__host__ __device__ inline int band16_stage_cols(int m, int k, int S4) {
    const int need = k + 4 * S4 + 3;
    return need > m + k - 1 ? need : m + k - 1;
}
__host__ __device__ inline int band16_max_steps(int m, int r, int k) {
    int smax = 0;
    const int r2 = 2 * r;
    for (int t = 0; t < band_tiles(r, k); ++t) {
        const int wl = 32 * t / r2, wh = min((32 * t + 31) / r2, k - 1);
        const int st = (m + wh - wl + 3) / 4;
        smax = st > smax ? st : smax;
    }
    return smax;
}

// Packs tile t = blockIdx.x: lane l's values, in the order 2 s + ct, are
// B[w_lo + 4 s + l / 16][32 t + 16 ct + l % 16] (zero outside the window's
// rows and rank).  Also fills the block descriptor (ring position, ranks).
template <int S4>
__global__ __launch_bounds__(64)
void k_pack_band16(BlockProjectArgs a) {
    constexpr int NQ = (2 * S4 + 3) / 4;
    const int lane = threadIdx.x, t = blockIdx.x;
    const int k = a.k, m = a.m, r2 = 2 * a.r;
    if (t == 0) {
        for (int w = lane; w < k; w += 64) {
            int kc = 0;
            window_coef(a, w, kc);
            a.desc->kc[w] = kc;
        }
        if (lane == 0) {
            a.desc->valid = a.st->count >= a.m + 1 && !a.st->block_rejected;
            a.desc->base = a.st->oldest + 2 - k + a.slots;
        }
    }
    const int wlo = 32 * t / r2;
    const int lr = lane & 15, lk = lane >> 4;
    float y[4 * NQ];
#pragma unroll
    for (int j = 0; j < 4 * NQ; ++j) y[j] = 0.0f;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int g = 32 * t + 16 * ct + lr;
        const int w = g / r2, c = g % r2;
        int kc = 0;
        const float* B = w < k ? window_coef(a, w, kc) : nullptr;
#pragma unroll
        for (int st = 0; st < S4; ++st) {
            const int i = wlo + 4 * st + lk - w;  // row of C_w
            y[2 * st + ct] = (w < k && c < kc && i >= 0 && i < m) ? B[(int64_t)i * r2 + c] : 0.0f;
        }
    }
    uint4* out = a.cfrag + (size_t)t * NQ * 64 + lane;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        out[(size_t)q * 64] = uint4{__builtin_bit_cast(unsigned, y[4 * q]), __builtin_bit_cast(unsigned, y[4 * q + 1]),
                                    __builtin_bit_cast(unsigned, y[4 * q + 2]), __builtin_bit_cast(unsigned, y[4 * q + 3])};
}

// FULL as in k_project_band_s; S4 steps of 4 staged columns per tile (a
// shorter tile meets zero coefficients), every tile computed, stores that
// always issue.
template <int S4, bool FULL>
__global__ __launch_bounds__(kThreads, 2)
void k_project_band16_s(BlockProjectArgs a, int64_t slab0) {
    constexpr int NQ = (2 * S4 + 3) / 4;
    extern __shared__ float dynp[];
    const BlockDesc* desc = a.desc;
    if (!desc->valid) return;
    const int m = a.m, k = a.k, r2 = 2 * a.r;
    const int ncols = m + k - 1, nstage = band16_stage_cols(m, k, S4);
    const int ntile = band_tiles(a.r, k);
    float* U = dynp;
    const int64_t row0 = (slab0 + blockIdx.x) * kBandRows;
    const int base = desc->base;
    const float* ring = static_cast<const float*>(a.ring);
    __shared__ int s_kc[64];
    if (threadIdx.x < 64) s_kc[threadIdx.x] = threadIdx.x < k ? desc->kc[threadIdx.x] : 0;
    stage_columns<kBandRows>(ring, a.ld, a.slots, base, ncols, nstage, row0,
                             [&](int c, int r4, float4 x) { *reinterpret_cast<float4*>(&U[c * kBand16LDR + r4]) = x; });
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const bool odd = lr & 1;
    const uint4* cf = a.cfrag + lane;
    auto load_a = [&](int c, float (&av)[8]) {
        const float* u = U + (c + lk) * kBand16LDR + lr;
#pragma unroll
        for (int rt = 0; rt < 8; ++rt) av[rt] = u[16 * rt];
    };
    auto load_b = [&](int t, uint4 (&b)[NQ]) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) b[i] = cf[(size_t)(t * NQ + i) * 64];
    };
    auto bval = [](const uint4 (&b)[NQ], int j) {
        const uint4& u = b[j / 4];
        const unsigned bits = (j & 3) == 0 ? u.x : (j & 3) == 1 ? u.y : (j & 3) == 2 ? u.z : u.w;
        return __builtin_bit_cast(float, bits);
    };
    auto tile = [&](int t, const uint4 (&b)[NQ]) {
        const int g0 = 32 * t;
        const int wlo = __builtin_amdgcn_readfirstlane(g0 / r2);
        v4f acc[2][8];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) acc[ct][rt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        int c = wlo;
        float av[8];
        load_a(c, av);
#pragma unroll
        for (int st = 0; st < S4; ++st) {
            float an[8];
            load_a(c + 4, an);  // the next step's A fragments ahead of the products
            __builtin_amdgcn_sched_barrier(0);
            const float b0 = bval(b, 2 * st), b1 = bval(b, 2 * st + 1);
#pragma unroll
            for (int rt = 0; rt < 8; ++rt)
                acc[0][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt], b0, acc[0][rt], 0, 0, 0);
#pragma unroll
            for (int rt = 0; rt < 8; ++rt)
                acc[1][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt], b1, acc[1][rt], 0, 0, 0);
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) av[rt] = an[rt];
            c += 4;
        }
        v4f* sink = reinterpret_cast<v4f*>(a.desc->sink) + lane;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            // this lane pair's complex column: real column g, imaginary g + 1
            const int g = g0 + 16 * ct + (lr & ~1);
            const int w = g / r2, cc = g % r2;
            const int ws = w < k ? w : 0;
            const bool ok = w < k && cc < s_kc[ws];
            float2* o = a.out + (int64_t)ws * a.ldw + (int64_t)(cc >> 1) * a.ldo;
#pragma unroll
            for (int rt = 0; rt < 8; ++rt) {
                const v4f d = acc[ct][rt];
                const float x = odd ? d[0] : d[2], y = odd ? d[1] : d[3];
                const float xs = swap_pair(x), ys = swap_pair(y);
                const float4 val = odd ? float4{xs, d[2], ys, d[3]} : float4{d[0], xs, d[1], ys};
                const int64_t row = row0 + 16 * rt + 4 * lk + (odd ? 2 : 0);
                float2* q = o + row;
                if constexpr (FULL) {
                    v4f* dst = ok ? reinterpret_cast<v4f*>(q) : sink;
                    __builtin_nontemporal_store(v4f{val.x, val.y, val.z, val.w}, dst);
                } else if (ok && row < a.n) {
                    q[0] = float2{val.x, val.y};
                    if (row + 1 < a.n) q[1] = float2{val.z, val.w};
                }
            }
        }
    };
    constexpr int T4 = kThreads / 64;
    uint4 bA[NQ], bB[NQ];
    auto ahead = [&](int t) { return t + T4 < ntile ? t + T4 : ntile - 1; };
    int t = wave;
    if (t >= ntile) return;
    load_b(t, bA);
    load_b(ahead(t), bB);
    __builtin_amdgcn_sched_barrier(0);
    tile(t, bA);
    t += T4;
    while (t < ntile) {
        load_b(ahead(t), bA);
        __builtin_amdgcn_sched_barrier(0);
        tile(t, bB);
        t += T4;
        if (t >= ntile) break;
        load_b(ahead(t), bB);
        __builtin_amdgcn_sched_barrier(0);
        tile(t, bA);
        t += T4;
    }
}

size_t block_lds(int m, int k) { return sizeof(float) * (size_t)(k - 1 + 32 * ((m + 31) / 32)) * kBlkLDR; }

template <int NT>
hipError_t launch_block_nt(const BlockProjectArgs& a, hipStream_t s) {
    const size_t lds = block_lds(a.m, a.k);
    if (lds > kBlockLdsMax) return hipErrorInvalidValue;
    if (!a.cfrag || !a.desc) return hipErrorInvalidValue;
    auto kern = a.bf16x3 ? k_project_block<NT, true> : k_project_block<NT, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)((a.n + kBlkRows - 1) / kBlkRows);
    hipLaunchKernelGGL(kern, dim3(gx), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

// Fixed-step instances of the 16 x 16 banded kernel (4 staged columns a
// step), and the instance for these sizes: the longest tile's steps rounded
// up by at most one, its stage within the LDS budget; 0 if none applies.
constexpr int kBand16Steps[] = {5, 9, 13, 17};
constexpr int kBand16NSteps = sizeof(kBand16Steps) / sizeof(kBand16Steps[0]);
int band16_fixed_steps(int m, int r, int k) {
    const int smax = band16_max_steps(m, r, k);
    for (int S4 : kBand16Steps)
        if (smax <= S4 && S4 - smax <= 1 &&
            sizeof(float) * (size_t)band16_stage_cols(m, k, S4) * kBand16LDR <= kBlockLdsMax)
            return S4;
    return 0;
}

size_t project_block_frag_bytes(int m, int r, int kmax) {
    const PairShape ps = pair_shape(m);
    const size_t per_window = (size_t)kmax * ((m + 31) / 32) * 4 * 64 * 32;
    const size_t pairs =
        (size_t)((kmax + 1) / 2) * (8 * ps.nfull + ps.tail) * kPairMaxTilesTuned * 64 * sizeof(float);
    const size_t band = (size_t)band_tiles(r, kmax) * band_chunks(m, r) * 64 * 32;
    const size_t band16 = (size_t)band_tiles(r, kmax) * band16_nq(kBand16Steps[kBand16NSteps - 1]) * 64 * 16;
    size_t b = per_window > pairs ? per_window : pairs;
    b = b > band ? b : band;
    return b > band16 ? b : band16;
}

bool project_block_fits(int m, int k, int r) {
    return 2 * r <= 64 && k <= 64 && block_lds(m, k) <= kBlockLdsMax && pair_lds(m, k) <= kBlockLdsMax;
}

bool pairs_apply(int m, int r, int k) {
    BlockProjectArgs a{};
    a.m = m;
    a.r = r;
    a.k = k;
    a.form = 2;
    return use_pairs(a);
}
bool band_applies(int m, int r, int k) { return r >= 1 && band_lds(m, k) <= kBlockLdsMax; }


// Fixed-step instances of the banded kernel: S steps per tile.
constexpr int kBandSteps[] = {9, 13, 17, 21, 25, 29, 33, 36};
// The instance for these sizes (the longest tile's steps rounded up by at most
// 3), or 0 if none applies (the chunk-loop kernel then runs).
int band_fixed_steps(int m, int r, int k) {
    const int smax = band_max_steps(m, r, k);
    for (int S : kBandSteps)
        if (smax <= S && S - smax <= 3 && (S + 7) / 8 <= band_chunks(m, r) &&
            sizeof(float) * (size_t)band_s_stage_cols(m, k, S) * kBandLDR <= kBlockLdsMax)
            return S;
    return 0;
}

// The banded form: FP32 products, and its stage fits; asked for (form 3, by
// the tuned shape of the stream), or by the rule (form 0) where a fixed-step
// instance applies: at the full-HD workload (m = 64, r = 20, k = 32) the step
// with it takes 4.17 ms against 4.68 with one product per window (the
// chunk-loop kernel, for other sizes, is slower than one product per window).
bool use_band(const BlockProjectArgs& a) {
    if (a.bf16x3 || a.form == 1 || a.form == 2) return false;
    if (band_lds(a.m, a.k) > kBlockLdsMax) return false;
    return a.form == 3 || band_fixed_steps(a.m, a.r, a.k) > 0;
}

int block_rule_form(int m, int r, int k) {
    BlockProjectArgs a{};
    a.m = m;
    a.r = r;
    a.k = k;
    return use_band(a) ? 3 : use_pairs(a) ? 2 : 1;
}

hipError_t launch_band16(const BlockProjectArgs& a, hipStream_t s, bool pack, int S4) {
    const int ntile = band_tiles(a.r, a.k);
    const void* pk = nullptr;
    const void* full = nullptr;
    const void* part = nullptr;
#define DMD_BAND16_S(N)                                                                          \
    if (S4 == N) {                                                                               \
        pk = reinterpret_cast<const void*>(k_pack_band16<N>);                                    \
        full = reinterpret_cast<const void*>(k_project_band16_s<N, true>);                       \
        part = reinterpret_cast<const void*>(k_project_band16_s<N, false>);                      \
    }
    DMD_BAND16_S(5)
    DMD_BAND16_S(9)
    DMD_BAND16_S(13)
    DMD_BAND16_S(17)
#undef DMD_BAND16_S
    if (!pk) return hipErrorInvalidValue;
    if (pack) {
        void* args[] = {const_cast<BlockProjectArgs*>(&a)};
        return hipLaunchKernel(pk, dim3((unsigned)ntile), dim3(64), args, 0, s);
    }
    const size_t lds = sizeof(float) * (size_t)band16_stage_cols(a.m, a.k, S4) * kBand16LDR;
    const int64_t nslab = (a.n + kBandRows - 1) / kBandRows;
    // whole slabs with 16-byte stores in one launch, the rest in another
    const int64_t nfull = a.out16 ? a.n / kBandRows : 0;
    int64_t slab0 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const void* kern = pass == 0 ? full : part;
        const int64_t cnt = pass == 0 ? nfull : nslab - nfull;
        if (cnt <= 0) continue;
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        void* args[] = {const_cast<BlockProjectArgs*>(&a), &slab0};
        e = hipLaunchKernel(kern, dim3((unsigned)cnt), dim3(kThreads), args, lds, s);
        if (e != hipSuccess) return e;
        slab0 += cnt;
    }
    return hipSuccess;
}

hipError_t launch_band(const BlockProjectArgs& a, hipStream_t s, bool pack) {
    if (!a.cfrag || !a.desc) return hipErrorInvalidValue;
    // the 16 x 16 form wherever one of its instances applies (the pack and
    // the projection of a block take the same decision from the same sizes)
    if (const int S4 = band16_fixed_steps(a.m, a.r, a.k)) return launch_band16(a, s, pack, S4);
    const int ntile = band_tiles(a.r, a.k);
    if (pack) {
        hipLaunchKernelGGL(k_pack_band, dim3((unsigned)ntile, (unsigned)band_chunks(a.m, a.r)), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    size_t lds = band_lds(a.m, a.k);
    if (lds > kBlockLdsMax) return hipErrorInvalidValue;
    // fixed-step kernels for the longest tile's step count rounded up to the
    // next instance (at most 3 steps of zeros per tile), else the chunk loop
    // fixed-step kernels for the longest tile's step count rounded up to the
    // next instance (at most 3 steps of zeros per tile), else the chunk loop
    const void* full = nullptr;
    const void* part = nullptr;
    const int Sfix = band_fixed_steps(a.m, a.r, a.k);
    auto pick = [&](int S, const void* f_full, const void* f_part) {
        if (S == Sfix) {
            full = f_full;
            part = f_part;
            lds = sizeof(float) * (size_t)band_s_stage_cols(a.m, a.k, S) * kBandLDR;
        }
    };
#define DMD_BAND_S(S) \
    pick(S, reinterpret_cast<const void*>(k_project_band_s<S, true>), \
         reinterpret_cast<const void*>(k_project_band_s<S, false>))
    DMD_BAND_S(9);
    DMD_BAND_S(13);
    DMD_BAND_S(17);
    DMD_BAND_S(21);
    DMD_BAND_S(25);
    DMD_BAND_S(29);
    DMD_BAND_S(33);
    DMD_BAND_S(36);
#undef DMD_BAND_S
    const int64_t nslab = (a.n + kBandRows - 1) / kBandRows;
    if (!full) {
        const void* kern = reinterpret_cast<const void*>(k_project_band);
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_project_band, dim3((unsigned)nslab), dim3(kThreads), lds, s, a);
        return hipGetLastError();
    }
    // whole slabs with 16-byte stores in one launch, the rest (or all of it,
    // where the output does not allow 16-byte stores) in another
    const int64_t nfull = a.out16 ? a.n / kBandRows : 0;
    int64_t slab0 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const void* kern = pass == 0 ? full : part;
        const int64_t cnt = pass == 0 ? nfull : nslab - nfull;
        if (cnt <= 0) continue;
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        void* args[] = {const_cast<BlockProjectArgs*>(&a), &slab0};
        e = hipLaunchKernel(kern, dim3((unsigned)cnt), dim3(kThreads), args, lds, s);
        if (e != hipSuccess) return e;
        slab0 += cnt;
    }
    return hipSuccess;
}

template <int NT>
hipError_t launch_pack_nt(const BlockProjectArgs& a, hipStream_t s) {
    if (!a.cfrag || !a.desc) return hipErrorInvalidValue;
    const dim3 pgrid((unsigned)(((a.m + 31) / 32) * NT), (unsigned)a.k);
    if (a.bf16x3) hipLaunchKernelGGL((k_pack_coef<NT, true>), pgrid, dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_pack_coef<NT, false>), pgrid, dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int NTG>
hipError_t launch_pair_ntg(const BlockProjectArgs& a, hipStream_t s, bool pack) {
    if (!a.cfrag || !a.desc) return hipErrorInvalidValue;
    if (pack) {
        hipLaunchKernelGGL(k_pack_pair<NTG>, dim3(NTG, (unsigned)((a.k + 1) / 2)), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    const size_t lds = pair_lds(a.m, a.k);
    if (lds > kBlockLdsMax) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_project_pair<NTG>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)((a.n + kBlkRows - 1) / kBlkRows);
    hipLaunchKernelGGL(k_project_pair<NTG>, dim3(gx), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_pair(const BlockProjectArgs& a, hipStream_t s, bool pack) {
    switch (4 * a.r / 16) {
        case 1: return launch_pair_ntg<1>(a, s, pack);
        case 3: return launch_pair_ntg<3>(a, s, pack);
        case 5: return launch_pair_ntg<5>(a, s, pack);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_block(const BlockProjectArgs& a, hipStream_t s) {
    const int kc_max = 2 * a.r;
    if (kc_max > 64 || a.k < 1 || a.k > a.kmax) return hipErrorInvalidValue;
    if (use_band(a)) return launch_band(a, s, true);
    if (use_pairs(a)) return launch_pair(a, s, true);
    if (kc_max <= 16) return launch_pack_nt<1>(a, s);
    if (kc_max <= 32) return launch_pack_nt<2>(a, s);
    if (kc_max <= 48) return launch_pack_nt<3>(a, s);
    return launch_pack_nt<4>(a, s);
}

hipError_t launch_project_block(const BlockProjectArgs& a, hipStream_t s) {
    const int kc_max = 2 * a.r;
    if (kc_max > 64 || a.k < 1 || a.k > a.kmax || a.ld % kBlkRows) return hipErrorInvalidValue;
    if (use_band(a)) return launch_band(a, s, false);
    if (use_pairs(a)) return launch_pair(a, s, false);
    if (kc_max <= 16) return launch_block_nt<1>(a, s);
    if (kc_max <= 32) return launch_block_nt<2>(a, s);
    if (kc_max <= 48) return launch_block_nt<3>(a, s);
    return launch_block_nt<4>(a, s);
}

int project_item_blocks(int64_t n) { return (int)((n + kRowsPerBlock - 1) / kRowsPerBlock); }

hipError_t launch_project_grouped(const ProjectArgs* items, const int* blk_start, int nitems, int total_blocks,
                                  hipStream_t s) {
    // four 16-column tiles cover every r <= 32
    hipLaunchKernelGGL(k_project_grouped<4>, dim3(total_blocks), dim3(kThreads), 0, s, items, blk_start, nitems);
    return hipGetLastError();
}

hipError_t launch_project(const ProjectArgs& a, hipStream_t s) {
    const int kc_max = a.cplx_out ? 2 * a.kmax : a.kmax;
    if (kc_max > 64) return hipErrorInvalidValue;
    if (a.elem_f64) return launch_tiles<double, double>(a, s, kc_max);
    if (a.coef_f64) return launch_tiles<float, double>(a, s, kc_max);
    if (a.precision == 2 /* DMD_PREC_BF16X3 */) {
        if (kc_max <= 16) return launch_bf3_nt<1>(a, s);
        if (kc_max <= 32) return launch_bf3_nt<2>(a, s);
        if (kc_max <= 48) return launch_bf3_nt<3>(a, s);
        return launch_bf3_nt<4>(a, s);
    }
    return launch_tiles<float, float>(a, s, kc_max);
}

}  // namespace dmd
