// Sparse complex snapshots (Sec. 3.5): SVD and DMD are invariant under a
// unitary transform, so a stream of Fourier coefficients can be decomposed
// directly; most coefficients are zero, so inner products and projections run
// over the stored entries only.
//
// A snapshot is (idx[nnz] strictly increasing in [0, n), val[nnz] complex64).
// The window ring holds m+2 such snapshots (capacity max_nnz each).  Inner
// products <x_j, x_new> = sum conj(x_j[k]) x_new[k] are formed by scattering
// the new snapshot into a dense scratch vector (kept all-zero between pushes)
// and gathering it at every window column's indices: O(nnz) per column, no
// index intersection.  Products of complex64 values are accumulated in FP64;
// every reduction has a fixed order (bitwise reproducible).
#include "cplx.h"
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;
constexpr int kChunks = 8;  // workgroups per window column in the inner-product kernel

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Copy the snapshot into the spare ring slot, scatter it into the dense
// scratch vector, and flag indices that are out of range or not increasing.
__global__ __launch_bounds__(kThreads)
void k_csr_ingest(const int32_t* __restrict__ idx, const float2* __restrict__ val, int nnz, int64_t n,
                  int32_t* __restrict__ ring_idx, float2* __restrict__ ring_val, int32_t* __restrict__ ring_nnz,
                  int max_nnz, int m, float2* __restrict__ scatter, int* __restrict__ flag,
                  const DevState* __restrict__ st) {
    const int slots = m + 2;
    const int spare = slot_of(st->oldest, st->count, slots);
    const int64_t base = (int64_t)spare * max_nnz;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < nnz; e += gridDim.x * kThreads) {
        const int32_t i = idx[e];
        const float2 v = val[e];
        const bool in_range = i >= 0 && (int64_t)i < n;
        const bool increasing = e == 0 || idx[e - 1] < i;
        if (!(in_range && increasing)) atomicOr(flag, 1);
        ring_idx[base + e] = i;
        ring_val[base + e] = v;
        if (in_range) scatter[i] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ring_nnz[spare] = nnz;
}

// partials[(j * kChunks + c) * 2 + {0,1}] = share c of <x_j, x_new> for kept
// window column j (window order) and, at j = nkept, of <x_new, x_new>.
__global__ __launch_bounds__(kThreads)
void k_csr_gram(const int32_t* __restrict__ ring_idx, const float2* __restrict__ ring_val,
                const int32_t* __restrict__ ring_nnz, int max_nnz, int m, const float2* __restrict__ scatter,
                double* __restrict__ partials, const DevState* __restrict__ st) {
    const int slots = m + 2;
    const int count = st->count, oldest = st->oldest;
    const int keep0 = (count == m + 1) ? 1 : 0;
    const int nkept = count - keep0;
    const int j = blockIdx.y;
    if (j > nkept) return;
    const int slot = j < nkept ? slot_of(oldest, keep0 + j, slots) : slot_of(oldest, count, slots);
    const int nz = ring_nnz[slot];
    const int c = blockIdx.x;
    const int e0 = (int)((int64_t)nz * c / kChunks), e1 = (int)((int64_t)nz * (c + 1) / kChunks);
    const int64_t base = (int64_t)slot * max_nnz;
    // The new snapshot's own product reads its values directly: its indices
    // are checked only by the finalize kernel, so they may still be out of
    // range here.  With valid indices the scatter vector holds exactly these
    // values, so the sum is the same either way.  The kept columns' indices
    // were checked when they were pushed or restored.
    const bool self = j == nkept;
    double re = 0.0, im = 0.0;
    for (int e = e0 + threadIdx.x; e < e1; e += kThreads) {
        const float2 a = ring_val[base + e];
        const float2 b = self ? a : scatter[ring_idx[base + e]];
        // conj(a) * b in FP64 (products of FP32 values are exact)
        re = fma((double)a.x, (double)b.x, re);
        re = fma((double)a.y, (double)b.y, re);
        im = fma((double)a.x, (double)b.y, im);
        im = fma(-(double)a.y, (double)b.x, im);
    }
    __shared__ double red[2][kThreads / 64];
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = re;
        red[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            sr += red[0][w];
            si += red[1][w];
        }
        partials[2 * ((int64_t)j * kChunks + c)] = sr;
        partials[2 * ((int64_t)j * kChunks + c) + 1] = si;
    }
}

// Fixed-order sum of the partials; reject the snapshot on bad indices or
// non-finite products, else write the new Hermitian Gram row and column and
// advance the window.
__global__ __launch_bounds__(kThreads)
void k_csr_finalize(double* __restrict__ G, const double* __restrict__ partials, int m, int* __restrict__ flag,
                    DevState* __restrict__ st) {
    const int slots = m + 2;
    const int count = st->count, oldest = st->oldest;
    const int spare = slot_of(oldest, count, slots);
    const int keep0 = (count == m + 1) ? 1 : 0;
    const int nkept = count - keep0;
    __shared__ double g[2 * (kMaxM + 2)];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = threadIdx.x; j <= nkept; j += kThreads) {
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < kChunks; ++c) {
            sr += partials[2 * ((int64_t)j * kChunks + c)];
            si += partials[2 * ((int64_t)j * kChunks + c) + 1];
        }
        g[2 * j] = sr;
        g[2 * j + 1] = si;
        if (!isfinite(sr) || !isfinite(si)) bad = 1;
    }
    __syncthreads();
    const int idx_bad = *flag;
    if (idx_bad || bad) {
        if (threadIdx.x == 0) {
            if (idx_bad) st->rejected_index += 1;
            else st->rejected_nonfinite += 1;
            *flag = 0;
        }
        return;
    }
    for (int j = threadIdx.x; j < nkept; j += kThreads) {
        const int sj = slot_of(oldest, keep0 + j, slots);
        double* col = G + 2 * (sj + (int64_t)spare * slots);  // <x_j, x_new>
        double* row = G + 2 * (spare + (int64_t)sj * slots);  // <x_new, x_j> = conj
        col[0] = g[2 * j];
        col[1] = g[2 * j + 1];
        row[0] = g[2 * j];
        row[1] = -g[2 * j + 1];
    }
    if (threadIdx.x == 0) {
        double* d = G + 2 * (spare + (int64_t)spare * slots);
        d[0] = g[2 * nkept];
        d[1] = 0.0;
        if (count == m + 1) st->oldest = slot_of(oldest, 1, slots);
        else st->count = count + 1;
        st->pushes += 1;
        *flag = 0;
    }
}

// Restore the scratch vector to zero at the pushed snapshot's indices.
__global__ __launch_bounds__(kThreads)
void k_csr_clear(const int32_t* __restrict__ idx, int nnz, int64_t n, float2* __restrict__ scatter) {
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < nnz; e += gridDim.x * kThreads) {
        const int32_t i = idx[e];
        if (i >= 0 && (int64_t)i < n) scatter[i] = make_float2(0.f, 0.f);
    }
}

// out[:, q] = sum_j X_sub[:, j] B[j][q] for sparse complex columns, one
// workgroup per output column: the column is zeroed, then window columns are
// added in window order (entries of one column have distinct rows, so the
// read-modify-writes of one step never collide; steps are separated by
// barriers): deterministic.
__global__ __launch_bounds__(kThreads)
void k_csr_project(const DevState* __restrict__ st, const int32_t* __restrict__ ring_idx,
                   const float2* __restrict__ ring_val, const int32_t* __restrict__ ring_nnz, int max_nnz, int m,
                   int first, const float2* __restrict__ B, int kmax, float2* __restrict__ out, int64_t ldo,
                   int64_t n, const int* __restrict__ overflow) {
    // fallback, used only when the window's union of supports exceeds the
    // dense block's capacity: one workgroup per output column
    if (st->solve_status == ST_E_NOT_READY || !*overflow) return;
    const int q = blockIdx.x;
    if (q >= st->r_eff) return;
    const int slots = m + 2;
    const int oldest = st->oldest;
    float2* col = out + (int64_t)q * ldo;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) col[i] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        const int slot = slot_of(oldest, first + j, slots);
        const int nz = ring_nnz[slot];
        const float2 c = B[(int64_t)j * kmax + q];
        const int64_t base = (int64_t)slot * max_nnz;
        for (int e = threadIdx.x; e < nz; e += kThreads) {
            const int32_t i = ring_idx[base + e];
            const float2 v = ring_val[base + e];
            float2 o = col[i];
            o.x = fmaf(v.x, c.x, fmaf(-v.y, c.y, o.x));
            o.y = fmaf(v.x, c.y, fmaf(v.y, c.x, o.y));
            col[i] = o;
        }
        __syncthreads();
    }
}

// ---- projection through the union of the window's supports
//
// Every index that occurs in a window column gets a row u of a dense block
// D (u x m, complex64; row order is immaterial, so the rows are handed out by
// an atomic counter); D holds the window on its union U, zero elsewhere, so
// out[U[u]][q] = sum_j D[u][j] B[j][q] is a small dense product, summed in
// column order j = 0 .. m-1 exactly as a column-by-column scatter would (a
// missing entry adds an exact zero).  Outside U the output is zero.
struct UnionArgs {
    const DevState* st;
    const int32_t* ring_idx;
    const float2* ring_val;
    const int32_t* ring_nnz;
    int max_nnz, m, first;
    int32_t* pos;     // n entries, -1 outside U (restored after use)
    int32_t* U;       // cap entries
    int* ucount;      // |U|
    int* overflow;    // |U| > cap: the fallback kernel runs instead
    int cap;
    float2* D;        // cap x m
};

__global__ __launch_bounds__(64)
void k_union_reset(UnionArgs a) {
    if (threadIdx.x == 0) {
        *a.ucount = 0;
        *a.overflow = 0;
    }
}

// one pass over the window's entries: first occurrence of an index claims a row
__global__ __launch_bounds__(kThreads)
void k_union_mark(UnionArgs a) {
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY) return;
    const int slots = a.m + 2;
    const int j = blockIdx.y;
    const int slot = slot_of(st->oldest, a.first + j, slots);
    const int nz = a.ring_nnz[slot];
    const int64_t base = (int64_t)slot * a.max_nnz;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < nz; e += gridDim.x * kThreads) {
        const int32_t i = a.ring_idx[base + e];
        if (atomicCAS(&a.pos[i], -1, INT32_MAX) == -1) {
            const int u = atomicAdd(a.ucount, 1);
            if (u < a.cap) a.U[u] = i;
            else atomicOr(a.overflow, 1);
            a.pos[i] = u;  // read only by later kernels
        }
    }
}

__global__ __launch_bounds__(kThreads)
void k_union_zero(UnionArgs a) {
    if (a.st->solve_status == ST_E_NOT_READY || *a.overflow) return;
    const int64_t total = (int64_t)*a.ucount * a.m;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < total; k += (int64_t)gridDim.x * kThreads)
        a.D[k] = float2{0.0f, 0.0f};
}

__global__ __launch_bounds__(kThreads)
void k_union_gather(UnionArgs a) {
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY || *a.overflow) return;
    const int slots = a.m + 2;
    const int j = blockIdx.y;
    const int slot = slot_of(st->oldest, a.first + j, slots);
    const int nz = a.ring_nnz[slot];
    const int64_t base = (int64_t)slot * a.max_nnz;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < nz; e += gridDim.x * kThreads)
        a.D[(int64_t)a.pos[a.ring_idx[base + e]] * a.m + j] = a.ring_val[base + e];
}

// zero the n x r_eff output (16-byte stores where aligned)
__global__ __launch_bounds__(kThreads)
void k_union_clear_out(UnionArgs a, float2* __restrict__ out, int64_t ldo, int64_t n) {
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY || *a.overflow) return;
    const int q = blockIdx.y;
    if (q >= st->r_eff) return;
    float2* col = out + (int64_t)q * ldo;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        col[i] = float2{0.0f, 0.0f};
}

__global__ __launch_bounds__(kThreads)
void k_union_product(UnionArgs a, const float2* __restrict__ B, int kmax, float2* __restrict__ out, int64_t ldo) {
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY || *a.overflow) return;
    const int q = blockIdx.y;
    if (q >= st->r_eff) return;
    const int nu = *a.ucount;
    for (int u = blockIdx.x * kThreads + threadIdx.x; u < nu; u += gridDim.x * kThreads) {
        const float2* d = a.D + (int64_t)u * a.m;
        float2 o{0.0f, 0.0f};
        for (int j = 0; j < a.m; ++j) {
            const float2 v = d[j];
            const float2 c = B[(int64_t)j * kmax + q];
            o.x = fmaf(v.x, c.x, fmaf(-v.y, c.y, o.x));
            o.y = fmaf(v.x, c.y, fmaf(v.y, c.x, o.y));
        }
        out[a.U[u] + (int64_t)q * ldo] = o;
    }
}

// give the index map back its -1s (the whole map after an overflow, when
// rows past the capacity were not recorded in U)
__global__ __launch_bounds__(kThreads)
void k_union_restore(UnionArgs a, int64_t n) {
    if (a.st->solve_status == ST_E_NOT_READY) return;
    if (*a.overflow) {
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
            a.pos[i] = -1;
        return;
    }
    const int nu = *a.ucount;
    for (int u = blockIdx.x * kThreads + threadIdx.x; u < nu; u += gridDim.x * kThreads) a.pos[a.U[u]] = -1;
}

}  // namespace

hipError_t launch_csr_push(const int32_t* idx, const float2* val, int nnz, int64_t n, int32_t* ring_idx,
                           float2* ring_val, int32_t* ring_nnz, int max_nnz, int m, float2* scatter, int* flag,
                           double* G, double* partials, DevState* st, hipStream_t s) {
    const int gx = nnz > 0 ? (nnz + kThreads - 1) / kThreads : 1;
    const int gi = gx < 1024 ? gx : 1024;
    hipLaunchKernelGGL(k_csr_ingest, dim3(gi), dim3(kThreads), 0, s, idx, val, nnz, n, ring_idx, ring_val, ring_nnz,
                       max_nnz, m, scatter, flag, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_gram, dim3(kChunks, m + 1), dim3(kThreads), 0, s, ring_idx, ring_val, ring_nnz, max_nnz,
                       m, scatter, partials, st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_finalize, dim3(1), dim3(kThreads), 0, s, G, partials, m, flag, st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_clear, dim3(gi), dim3(kThreads), 0, s, idx, nnz, n, scatter);
    return hipGetLastError();
}

int csr_partials_per_column() { return kChunks; }

int csr_union_cap(int64_t n, int max_nnz) {
    const int64_t c = 4 * (int64_t)max_nnz;
    return (int)(c < n ? c : n);
}

hipError_t launch_csr_project(const DevState* st, const int32_t* ring_idx, const float2* ring_val,
                              const int32_t* ring_nnz, int max_nnz, int m, int first, const float2* B, int kmax,
                              float2* out, int64_t ldo, int64_t n, const CsrUnionScratch& u, hipStream_t s) {
    UnionArgs a{st, ring_idx, ring_val, ring_nnz, max_nnz, m, first, u.pos, u.U, u.ucount, u.overflow, u.cap, u.D};
    const unsigned ge = (unsigned)((max_nnz + kThreads - 1) / kThreads);
    const unsigned gz = (unsigned)(((int64_t)u.cap * m + kThreads - 1) / kThreads);
    const unsigned gu = (unsigned)((u.cap + kThreads - 1) / kThreads);
    const int64_t gn = (n + kThreads - 1) / kThreads;
    const unsigned go = (unsigned)(gn < 4096 ? gn : 4096);
    hipLaunchKernelGGL(k_union_reset, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_union_mark, dim3(ge, m), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_union_zero, dim3(gz < 4096 ? gz : 4096), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_union_gather, dim3(ge, m), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_union_clear_out, dim3(go, kmax), dim3(kThreads), 0, s, a, out, ldo, n);
    hipLaunchKernelGGL(k_union_product, dim3(gu, kmax), dim3(kThreads), 0, s, a, B, kmax, out, ldo);
    hipLaunchKernelGGL(k_csr_project, dim3(kmax), dim3(kThreads), 0, s, st, ring_idx, ring_val, ring_nnz, max_nnz, m,
                       first, B, kmax, out, ldo, n, u.overflow);
    hipLaunchKernelGGL(k_union_restore, dim3(go), dim3(kThreads), 0, s, a, n);
    return hipGetLastError();
}

}  // namespace dmd
