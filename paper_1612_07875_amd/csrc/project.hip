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
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;   // 4 wavefronts
constexpr int kRowsPerWave = 64;
constexpr int kRowsPerBlock = kThreads / 64 * kRowsPerWave;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi): the BF16x3 split.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
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
    const int m = a.m;
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
            for (int rt = 0; rt < 4; ++rt) av[buf][g][rt] = (cin && rin[rt]) ? (T)cp[row0 + 16 * rt + li] : T(0);
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
                        out[o] = sw[lane * OLD + cc];
                        out[o + 1] = sw[lane * OLD + cc + 1];
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
    const int m = a.m;
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
                        out[o] = sw[lane * OLD + cc];
                        out[o + 1] = sw[lane * OLD + cc + 1];
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
// same banks.
constexpr int kBlkRows = 64;
constexpr int kBlkLDR = kBlkRows + 16;  // column stride: the four k-slots of a fragment hit distinct banks
constexpr size_t kBlockLdsMax = 150 * 1024;  // dynamic LDS of the one-pass block projection
constexpr int kBlkOLD = 17;             // padded row length of the output stage

template <int NT, bool BF3>
__global__ __launch_bounds__(kThreads, 3)
void k_project_block(BlockProjectArgs a) {
    extern __shared__ float dynp[];
    const DevState* stf = a.st;
    if (stf->count < a.m + 1 || stf->block_rejected) return;
    const int m = a.m, k = a.k;
    const int ncols = m + k - 1;
    float* U = dynp;
    float* stage = dynp + (size_t)ncols * kBlkLDR;
    const int64_t row0 = (int64_t)blockIdx.x * kBlkRows;
    const int base = stf->oldest + 2 - k + a.slots;  // slot of staged column 0, before the wrap
    const float* ring = static_cast<const float*>(a.ring);
    for (int t = threadIdx.x; t < ncols * (kBlkRows / 4); t += kThreads) {
        const int c = t / (kBlkRows / 4), q = t % (kBlkRows / 4);
        const float* src = ring + (int64_t)((base + c) % a.slots) * a.ld + row0 + 4 * q;
        *reinterpret_cast<float4*>(&U[c * kBlkLDR + 4 * q]) = *reinterpret_cast<const float4*>(src);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    float* sw = stage + wave * 64 * kBlkOLD;
    const int rs = 2 * a.r;
    for (int w = wave; w < k; w += kThreads / 64) {
        const int set = a.kmax - k + w;
        const DevState* st =
            w == k - 1 ? stf : reinterpret_cast<const DevState*>(a.shadow + (size_t)set * a.shadow_stride);
        if (st->solve_status != ST_OK && st->solve_status != ST_W_RANK) continue;
        const int kc = 2 * st->r_eff;
        if (kc == 0) continue;
        const float* B = w == k - 1 ? a.Bphi : a.Bphi_sets + (int64_t)set * a.bphi_stride;
        v4f acc[4][NT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = v4f{0, 0, 0, 0};
        // coefficients of 8 k-steps (32 window columns) are loaded together
        // before their MFMAs, so the L2 latency is paid once per chunk
        for (int cb = 0; cb < m; cb += 32) {
            if constexpr (BF3) {
                v8bf bhi[NT], blo[NT];
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const int col = cb + 4 * ks + lk;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int c = 16 * nt + li;
                        __bf16 h, l;
                        split_bf16((col < m && c < kc) ? B[(int64_t)col * rs + c] : 0.0f, h, l);
                        bhi[nt][ks] = h;
                        blo[nt][ks] = l;
                    }
                }
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    v8bf ahi, alo;
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks) {
                        const int col = cb + 4 * ks + lk;
                        const bool cin = col < m;
                        const float av = cin ? U[(w + col) * kBlkLDR + 16 * rt + li] : 0.0f;
                        __bf16 h, l;
                        split_bf16(av, h, l);
                        ahi[ks] = h;
                        alo[ks] = l;
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = mma_bf16x3(ahi, alo, bhi[nt], blo[nt], acc[rt][nt]);
                }
            } else {
                float bv[8][NT];
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const int col = cb + 4 * ks + lk;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int c = 16 * nt + li;
                        bv[ks][nt] = (col < m && c < kc) ? B[(int64_t)col * rs + c] : 0.0f;
                    }
                }
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const int col = cb + 4 * ks + lk;
                    const bool cin = col < m;
                    const float* ucol = U + (w + (cin ? col : 0)) * kBlkLDR;
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt) {
                        const float av = cin ? ucol[16 * rt + li] : 0.0f;
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[ks][nt], acc[rt][nt], 0, 0, 0);
                    }
                }
            }
        }
        float2* out = a.out + (int64_t)w * a.ldw;
        const int64_t row = row0 + lane;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (16 * nt >= kc) break;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) sw[(16 * rt + 4 * lk + v) * kBlkOLD + li] = acc[rt][nt][v];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (row < a.n) {
#pragma unroll
                for (int cc = 0; cc < 16; cc += 2) {
                    const int c = 16 * nt + cc;
                    if (c < kc)
                        out[row + (int64_t)(c >> 1) * a.ldo] = float2{sw[lane * kBlkOLD + cc], sw[lane * kBlkOLD + cc + 1]};
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

size_t block_lds(int m, int k) {
    return sizeof(float) * ((size_t)(m + k - 1) * kBlkLDR + (kThreads / 64) * 64 * kBlkOLD);
}

template <int NT>
hipError_t launch_block_nt(const BlockProjectArgs& a, hipStream_t s) {
    const size_t lds = block_lds(a.m, a.k);
    if (lds > kBlockLdsMax) return hipErrorInvalidValue;
    auto kern = a.bf16x3 ? k_project_block<NT, true> : k_project_block<NT, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const unsigned gx = (unsigned)((a.n + kBlkRows - 1) / kBlkRows);
    hipLaunchKernelGGL(kern, dim3(gx), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

bool project_block_fits(int m, int k, int r) { return 2 * r <= 64 && k <= 64 && block_lds(m, k) <= kBlockLdsMax; }

hipError_t launch_project_block(const BlockProjectArgs& a, hipStream_t s) {
    const int kc_max = 2 * a.r;
    if (kc_max > 64 || a.k < 1 || a.k > a.kmax || a.ld % kBlkRows) return hipErrorInvalidValue;
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
