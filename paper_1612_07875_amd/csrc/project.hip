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
    for (int t = threadIdx.x; t < ncols_pad * (kBlkRows / 4); t += kThreads) {
        const int c = t / (kBlkRows / 4), q = t % (kBlkRows / 4);
        float4 x = float4{0.0f, 0.0f, 0.0f, 0.0f};
        if (c < ncols) x = *reinterpret_cast<const float4*>(ring + (int64_t)((base + c) % a.slots) * a.ld + row0 + 4 * q);
        if constexpr (BF3) {
            *reinterpret_cast<uint4*>(&U[c * kBlkLDR + 4 * q]) =
                uint4{split_word(x.x), split_word(x.y), split_word(x.z), split_word(x.w)};
        } else {
            *reinterpret_cast<float4*>(&U[c * kBlkLDR + 4 * q]) = x;
        }
    }
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
    for (int t = threadIdx.x; t < ncols_pad * (kBlkRows / 4); t += kThreads) {
        const int c = t / (kBlkRows / 4), q = t % (kBlkRows / 4);
        float4 x = float4{0.0f, 0.0f, 0.0f, 0.0f};
        if (c < ncols) x = *reinterpret_cast<const float4*>(ring + (int64_t)((base + c) % a.slots) * a.ld + row0 + 4 * q);
        *reinterpret_cast<float4*>(&U[c * kBlkLDR + 4 * q]) = x;
    }
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

size_t project_block_frag_bytes(int m, int kmax) {
    const PairShape ps = pair_shape(m);
    const size_t per_window = (size_t)kmax * ((m + 31) / 32) * 4 * 64 * 32;
    const size_t pairs =
        (size_t)((kmax + 1) / 2) * (8 * ps.nfull + ps.tail) * kPairMaxTilesTuned * 64 * sizeof(float);
    return per_window > pairs ? per_window : pairs;
}

bool project_block_fits(int m, int k, int r) {
    return 2 * r <= 64 && k <= 64 && block_lds(m, k) <= kBlockLdsMax && pair_lds(m, k) <= kBlockLdsMax;
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
    if (use_pairs(a)) return launch_pair(a, s, true);
    if (kc_max <= 16) return launch_pack_nt<1>(a, s);
    if (kc_max <= 32) return launch_pack_nt<2>(a, s);
    if (kc_max <= 48) return launch_pack_nt<3>(a, s);
    return launch_pack_nt<4>(a, s);
}

hipError_t launch_project_block(const BlockProjectArgs& a, hipStream_t s) {
    const int kc_max = 2 * a.r;
    if (kc_max > 64 || a.k < 1 || a.k > a.kmax || a.ld % kBlkRows) return hipErrorInvalidValue;
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

namespace {
__global__ __launch_bounds__(256)
void k_snapshot(const DevState* __restrict__ st, DevState* __restrict__ st_out, const uint4* __restrict__ B,
                uint4* __restrict__ B_out, int n16) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += gridDim.x * blockDim.x) B_out[i] = B[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) *st_out = *st;
}
}  // namespace

hipError_t launch_snapshot(const DevState* st, DevState* st_out, const void* B, void* B_out, size_t bytes,
                           hipStream_t s) {
    if (bytes % 16) return hipErrorInvalidValue;
    const int n16 = (int)(bytes / 16);
    const int blocks = n16 / 256 + 1 < 64 ? n16 / 256 + 1 : 64;
    hipLaunchKernelGGL(k_snapshot, dim3(blocks), dim3(256), 0, s, st, st_out, static_cast<const uint4*>(B),
                       static_cast<uint4*>(B_out), n16);
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
