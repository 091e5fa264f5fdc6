// Multi-column streaming update (Sec. 5: updating the decomposition with more
// than one new column at a time).
//
// k new snapshots arrive together.  Every window that the k single pushes
// would pass through is a principal submatrix of the Gram of the union
// U = [window | new snapshots] (count + k columns), and of that Gram only the
// block U^* Y, Y = the k new columns, is new.  One pass over the union
// computes that (count + k) x k block as a tall-skinny product on the matrix
// cores: the union's columns are cut into tiles of 128, the rows into splits,
// and each workgroup stages 64 (FP32 data) or 32 (FP64 data) rows of its tile
// and of Y in LDS per step and accumulates with v_mfma_f64_16x16x4f64.  FP32
// data are widened exactly, so products are exact and sums are FP64 -- the
// accuracy class of the one-column update.  The workgroups of the first tile
// also copy Y into the ring's spare slots in the same pass (ingest fused).
//
// Reduction order is fixed (per-lane k order within an MFMA, then splits in
// index order), so results are bitwise reproducible run to run; they differ
// from k one-column updates only by summation order.
//
// Fragment layouts (checked on the device): 16x16x4 f64 A[l%16][l/16],
// B[l/16][l%16], D[(l/16)+4v][l%16].  Rows of the product (the k index of the
// MFMA) may be assigned to lanes in any order as long as A and B agree: lane
// (i, q) takes rows 4q .. 4q+3 of each 16-row group, one per MFMA, so that it
// reads them with one vector LDS load.
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kTI = 128;               // union columns per tile
constexpr int kTJ = 64;                // new columns: k <= 64
constexpr int kThreads = 512;          // 8 waves x 16 union columns
constexpr int kRedElems = 32;          // reduction: elements per workgroup
constexpr int kRedChunks = 32;         // reduction: split chunks per element
// tiles x splits: one workgroup per CU.  A block push usually runs beside the
// previous block's projection; two of these workgroups fill a CU's registers
// and keep the projection off it, one leaves room for a projection
// workgroup (the pass alone takes 430 us instead of 372, the block step
// 8130 -> 8230-8290 window updates/s at full HD, k = 32).
constexpr int kTargetGroups = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename TX> struct Stage;
template <> struct Stage<float>  { static constexpr int R = 64, PER = 4; using V = float4; };
template <> struct Stage<double> { static constexpr int R = 32, PER = 2; using V = double2; };

// Entry (i, j) of the block (union column i, new column j) is read by some
// window the k pushes pass through iff the two columns fit in one window of
// m + 1 columns (i >= cb + j - m), and, for a pair of new columns, it is the
// upper entry (i - cb <= j), from which the pair is written.  Entries outside
// are neither summed nor written: no window ever reads them (a slot that
// leaves the window has all its Gram entries rewritten when it is reused).
__device__ __forceinline__ bool block_needed(int i, int j, int cb, int m) {
    return i >= cb + j - m && (i < cb || i - cb <= j);
}

template <typename TX>
__global__ __launch_bounds__(kThreads, 4)
void k_block_tiles(BlockArgs a) {
    constexpr int R = Stage<TX>::R, PER = Stage<TX>::PER;
    constexpr int LDR = R + 4;                              // 16-byte rows, spread over the banks
    constexpr int TPC = R / PER;                            // 16-byte loads per column and step
    constexpr int MAXT = (kTI + kTJ) * TPC / kThreads;      // loads per thread and step
    using V = typename Stage<TX>::V;
    __shared__ __align__(16) TX Ls[(kTI + kTJ) * LDR];

    const int ti = blockIdx.x, split = blockIdx.y;
    const int cb = a.st->count, ob = a.st->oldest;
    const int U = cb + a.k;
    const int i0 = ti * kTI;
    if (i0 >= U) return;                                    // never read by the reduction
    const int ni = min(kTI, U - i0), nj = a.k;
    const int ni16 = (ni + 15) & ~15, nj16 = (nj + 15) & ~15;
    const int ntask = (ni16 + nj16) * TPC;
    const bool ingest = ti == 0;
    const TX* ring = static_cast<const TX*>(a.ring);
    TX* ring_w = static_cast<TX*>(const_cast<void*>(a.ring));
    const TX* xnew = static_cast<const TX*>(a.xnew);

    const int64_t r_begin = (int64_t)split * a.rows_per_split;
    const int64_t r_end = min(a.n, r_begin + a.rows_per_split);

    // staged column p: p < ni16 -> union column i0 + p; else new column p - ni16
    auto source = [&](int p, bool& valid, bool& aligned) -> const TX* {
        if (p < ni16) {
            const int c = i0 + p;
            valid = p < ni;
            if (c < cb) {
                aligned = true;
                return ring + (int64_t)slot_of(ob, c, a.slots) * a.ld;
            }
            aligned = a.x_aligned;
            return xnew + (int64_t)(c - cb) * a.ldx;
        }
        const int j = p - ni16;
        valid = j < nj;
        aligned = a.x_aligned;
        return xnew + (int64_t)j * a.ldx;
    };

    V regs[MAXT];
    auto load = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < MAXT; ++u) {
            const int t = threadIdx.x + u * kThreads;
            TX v[PER];
#pragma unroll
            for (int e = 0; e < PER; ++e) v[e] = TX(0);
            if (t < ntask) {
                const int p = t / TPC, q = t % TPC;
                const int64_t r = r0 + (int64_t)q * PER;
                bool valid, aligned;
                const TX* src = source(p, valid, aligned);
                if (valid && r < r_end) {
                    if (aligned && r + PER <= r_end) {
                        const V w = *reinterpret_cast<const V*>(src + r);
                        const TX* pw = reinterpret_cast<const TX*>(&w);
#pragma unroll
                        for (int e = 0; e < PER; ++e) v[e] = pw[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < PER; ++e) v[e] = (r + e < r_end) ? src[r + e] : TX(0);
                    }
                }
            }
            regs[u] = *reinterpret_cast<const V*>(v);
        }
    };
    auto store = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < MAXT; ++u) {
            const int t = threadIdx.x + u * kThreads;
            if (t < ntask) {
                const int p = t / TPC, q = t % TPC;
                *reinterpret_cast<V*>(&Ls[p * LDR + q * PER]) = regs[u];
                const int j = p - ni16;
                const int64_t r = r0 + (int64_t)q * PER;
                if (ingest && j >= 0 && j < nj && r < r_end) {
                    TX* dst = ring_w + (int64_t)slot_of(ob, cb + j, a.slots) * a.ld + r;
                    if (r + PER <= r_end) {
                        *reinterpret_cast<V*>(dst) = regs[u];
                    } else {
                        const TX* pw = reinterpret_cast<const TX*>(&regs[u]);
                        for (int e = 0; e < PER && r + e < r_end; ++e) dst[e] = pw[e];
                    }
                }
            }
        }
    };

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int nsub = nj16 / 16, n16 = ni16 / 16;
    // Work units: the 16 x 16 tiles (union tile iu of this workgroup's
    // columns, new subtile c) that hold an entry some window reads.  Unit u
    // goes to wave u % 8, i.e. to SIMD u % 4, so the four SIMDs' matrix cores
    // get equal shares; a wave holds at most four (n16 <= 8, nsub <= 4).
    // Every wave derives the same list (lane l < 16 tests row l of a tile).
    int my_iu[4] = {0, 0, 0, 0}, my_c[4] = {0, 0, 0, 0}, nmine = 0;
    {
        int u = 0;
        for (int c = 0; c < nsub; ++c)
            for (int iu = 0; iu < n16; ++iu) {
                const int ja = 16 * c, jb = min(ja + 15, nj - 1), i = i0 + 16 * iu + lane;
                bool ok = false;
                if (lane < 16 && i < U) {
                    const int jlo = i < cb ? ja : max(ja, i - cb);
                    const int jhi = min(jb, i - cb + a.m);
                    ok = jlo <= jhi;
                }
                if (__ballot(ok) == 0) continue;
                if ((u & 7) == wave && nmine < 4) {
                    my_iu[nmine] = iu;
                    my_c[nmine] = c;
                    ++nmine;
                }
                ++u;
            }
    }
    v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = v4d{0, 0, 0, 0};

    if (r_begin < r_end) load(r_begin);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += R) {
        __syncthreads();                     // the previous step's LDS reads are done
        store(r0);
        __syncthreads();
        if (r0 + R < r_end) load(r0 + R);    // in flight during this step's MFMAs
#pragma unroll 1
        for (int k0 = 0; k0 < R; k0 += 16) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t < nmine) {
                    const TX* pa = Ls + (16 * my_iu[t] + li) * LDR + 4 * lq + k0;
                    const TX* pb = Ls + (ni16 + 16 * my_c[t] + li) * LDR + 4 * lq + k0;
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)pa[s], (double)pb[s], acc[t], 0, 0, 0);
                }
            }
        }
    }

    // partial[split][i * kmax + j] for union column i, new column j
    double* out = a.partial + (int64_t)split * (a.slots * a.kmax);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= nmine) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * my_iu[t] + lq + 4 * v;
            const int j = 16 * my_c[t] + li;
            if (i < ni && j < nj) out[(int64_t)(i0 + i) * a.kmax + j] = acc[t][v];
        }
    }
}

// Sum the splits of every entry in a fixed order (chunk c takes splits c,
// c + 32, ...; chunks in index order), write the block, flag non-finite sums.
__global__ __launch_bounds__(kRedElems * kRedChunks)
void k_block_reduce(BlockArgs a) {
    const int cb = a.st->count, U = cb + a.k;
    const int el = threadIdx.x % kRedElems, ch = threadIdx.x / kRedElems;
    const int e = blockIdx.x * kRedElems + el;
    const int i = e / a.kmax, j = e % a.kmax;
    const bool valid = i < U && j < a.k && block_needed(i, j, cb, a.m);
    const int64_t estride = (int64_t)a.slots * a.kmax;
    double s = 0.0;
    if (valid)
        for (int p = ch; p < a.nsplit; p += kRedChunks) s += a.partial[(int64_t)p * estride + e];
    __shared__ double red[kRedChunks][kRedElems + 1];
    red[ch][el] = s;
    __syncthreads();
    if (ch == 0 && valid) {
        double t = red[0][el];
        for (int c = 1; c < kRedChunks; ++c) t += red[c][el];
        a.gblock[e] = t;
        if (!isfinite(t)) atomicOr(a.flag, 1);
    }
}

// Accept or reject the whole block; on acceptance write the new Gram rows and
// columns (physical slot indexing, each entry from exactly one block element)
// and advance the window by k.  Also set the state of every intermediate
// window so that their solves can run side by side with the final one.
__global__ __launch_bounds__(256)
void k_block_commit(BlockArgs a) {
    DevState* st = a.st;
    const int cb = st->count, ob = st->oldest, pushes0 = st->pushes;
    const int k = a.k, U = cb + k, m = a.m, slots = a.slots;
    const int bad = *a.flag;
    __syncthreads();
    for (int w = threadIdx.x; w < k - 1; w += blockDim.x) {
        DevState* sw = reinterpret_cast<DevState*>(a.shadow + (size_t)(a.kmax - k + w) * a.shadow_stride);
        const int cw = bad ? 0 : min(m + 1, cb + w + 1);
        sw->oldest = bad ? 0 : slot_of(ob, cb + w + 1 - cw, slots);
        sw->count = cw;
        sw->rejected_nonfinite = 0;
        sw->rejected_index = 0;
        sw->solve_status = ST_E_NOT_READY;
        sw->r_eff = 0;
        sw->sweeps = 0;
        sw->qr_iters = 0;
        sw->pushes = pushes0 + w + 1;
        sw->vprev_valid = 0;
        sw->vprev_push = -1;
        sw->warm = 0;
        sw->skipped = 0;
        sw->block_rejected = bad ? 1 : 0;
    }
    if (bad) {
        if (threadIdx.x == 0) {
            st->rejected_nonfinite += 1;
            st->block_rejected = 1;
            *a.flag = 0;
        }
        return;
    }
    for (int e = threadIdx.x; e < U * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        if (!block_needed(i, j, cb, m)) continue;  // never read (a pair of new columns: from its upper entry)
        const double v = a.gblock[i * a.kmax + j];
        const int si = slot_of(ob, i, slots), sj = slot_of(ob, cb + j, slots);
        a.G[si + (int64_t)sj * slots] = v;
        a.G[sj + (int64_t)si * slots] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int cnt = min(m + 1, U);
        st->oldest = slot_of(ob, U - cnt, slots);
        st->count = cnt;
        st->pushes = pushes0 + k;
        st->block_rejected = 0;
    }
}

int tiles_for(int m, int kmax) { return (m + 1 + kmax + kTI - 1) / kTI; }

}  // namespace

int gram_block_tiles(int m, int kmax) { return tiles_for(m, kmax); }

int gram_block_splits(int m, int kmax) {
    const int t = tiles_for(m, kmax);
    return (kTargetGroups + t - 1) / t;
}

hipError_t launch_gram_block(BlockArgs a, int elem_f64, hipStream_t s) {
    if (a.k < 1 || a.k > a.kmax || a.kmax > kTJ || a.slots < a.m + 1 + a.kmax) return hipErrorInvalidValue;
    a.ntile_i = tiles_for(a.m, a.kmax);
    a.ntile_j = 1;
    // row splits: at most the capacity, at least 64 rows each
    const int cap = gram_block_splits(a.m, a.kmax);
    const int64_t granule = 64;
    const int64_t max_by_rows = (a.n + granule - 1) / granule;
    a.nsplit = (int)(max_by_rows < cap ? max_by_rows : cap);
    a.rows_per_split = ((a.n + a.nsplit - 1) / a.nsplit + granule - 1) / granule * granule;
    dim3 grid(a.ntile_i, a.nsplit);
    if (elem_f64) hipLaunchKernelGGL(k_block_tiles<double>, grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL(k_block_tiles<float>, grid, dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int elems = a.slots * a.kmax;
    hipLaunchKernelGGL(k_block_reduce, dim3((elems + kRedElems - 1) / kRedElems), dim3(kRedElems * kRedChunks), 0, s,
                       a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_block_commit, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace dmd
