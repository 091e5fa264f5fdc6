// FP64 small solves of streaming DMD, run on the GPU after each Gram update.
//
// k_solve_sym (one workgroup):
//   * gathers xtx = X^* X (the first m window columns) from the physical Gram;
//   * eigendecomposition xtx V = V diag(d) by cyclic two-sided Jacobi with
//     parallel (round-robin) ordering: every round applies m/2 disjoint
//     rotations at once;  real symmetric or complex Hermitian;
//   * sigma = sqrt(|d|) sorted descending with V's columns permuted alike
//     (Algorithm 1), truncation to r_eff <= r resolvable values;
//   * A~ = Sigma^-1 V^* (X^* X') V Sigma^-1 from the Gram block xty without
//     forming U (Eq. Atilde; Algorithm 2; Sec. 3.4);
//   * POD coefficients V Sigma^-1 (Sec. 2.1, step 2).
// k_solve_eig (one wavefront):
//   * A~ W = W Lambda: Householder reduction to Hessenberg form, single-shift
//     complex QR iteration with Wilkinson shifts and deflation to Schur form
//     A~ = Z T Z^*, eigenvectors of T by back substitution, W = Z Y;
//   * eigenpairs sorted (|lambda| descending, arg ascending), W's columns
//     scaled to unit norm with the largest-modulus entry real positive;
//   * mode amplitudes b = (W Lambda)^-1 alpha_1 (Sec. 3.3) and the background
//     mode argmin |log lambda| (Algorithm 3);
//   * DMD coefficients C = V Sigma^-1 W for the projection Phi = X' C (Eq. Phi)
//     and the background coefficients C[:, bg] b_bg lambda_bg^m.
#include <cfloat>

#include "cplx.h"
#include "dmd_internal.h"
#include "gram_finalize.h"

namespace dmd {
namespace {

constexpr int kRMax = 32;         // largest truncation rank handled by k_solve_eig
constexpr double kEps = DBL_EPSILON;

// acc + sum of fa(k) * fb(k) over k = k0, k0 + step, ... < L, added in that
// order.  The operands of U consecutive terms are read before their
// products, so that their memory latencies overlap: a loop that reads,
// waits and multiplies one term at a time pays a full round trip per term,
// which the workspace forms of the solves (matrix and coefficients in
// global memory) cannot afford.  The sum is the plain loop's, bit for bit.
// U = 1 is the plain loop (the LDS forms: their register count decides
// whether a solve fits beside a running projection).
template <int U, typename S, typename FA, typename FB>
__device__ __forceinline__ S ordered_dot(S acc, int k0, int step, int L, FA fa, FB fb) {
    int k = k0;
    if constexpr (U > 1) {
        for (; k + (U - 1) * step < L; k += U * step) {
            S x[U], y[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[u] = fa(k + u * step);
                y[u] = fb(k + u * step);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = acc + mulr(x[u], y[u]);
        }
    }
    for (; k < L; k += step) acc = acc + mulr(fa(k), fb(k));
    return acc;
}
// terms read ahead by the workspace forms: 8 real or 4 complex values
template <typename S, bool LDS> constexpr int kAhead = LDS ? 1 : (sizeof(S) == sizeof(double) ? 8 : 4);

template <typename S> __device__ __forceinline__ S gram_at(const double* G, int a, int b, int slots);
template <> __device__ __forceinline__ double gram_at<double>(const double* G, int a, int b, int slots) {
    return G[a + (int64_t)b * slots];
}
template <> __device__ __forceinline__ cplx gram_at<cplx>(const double* G, int a, int b, int slots) {
    const double* p = G + 2 * (a + (int64_t)b * slots);
    return cplx{p[0], p[1]};
}

template <typename S> __device__ __forceinline__ void store_s(double* out, int64_t i, S v);
template <> __device__ __forceinline__ void store_s<double>(double* out, int64_t i, double v) { out[i] = v; }
template <> __device__ __forceinline__ void store_s<cplx>(double* out, int64_t i, cplx v) {
    out[2 * i] = v.re;
    out[2 * i + 1] = v.im;
}

// Round-robin tournament: in round `rd` (0 .. M-2) pair i (0 .. M/2-1) is (p, q);
// every index appears in exactly one pair per round and every pair of indices
// meets once per sweep.
__device__ __forceinline__ void rr_pair(int rd, int i, int M, int& p, int& q) {
    const int n1 = M - 1;
    if (i == 0) {
        p = n1;
        q = rd;
    } else {
        p = rd + i;
        if (p >= n1) p -= n1;
        q = rd - i;
        if (q < 0) q += n1;
    }
}

// 1/sqrt(x) to full FP64 accuracy: hardware estimate plus two Newton steps
// (the estimate carries ~23 correct bits).  Dependent FP64 operations cost
// ~32 cycles each here, so this replaces the longer correctly-rounded
// sqrt/division sequences on the latency-bound paths.
__device__ __forceinline__ double rsqrt_acc(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}
// 1/x to ~46 bits (estimate plus one Newton step).
__device__ __forceinline__ double rcp_fast(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
// 1/x to full FP64 accuracy (estimate plus two Newton steps).
__device__ __forceinline__ double rcp_acc(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// A double from another lane of the same 16-lane row, by a DPP lane pattern
// (a register move, no trip through the LDS crossbar as __shfl_xor takes).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over each aligned group of G lanes (G = 1, 2, 4, .., 64; every lane of
// the group active), the same value in every lane of the group: neighbour
// pairs, then pairs of pairs (quad permutations 1,0,3,2 and 2,3,0,1); then
// the mirror of each 8-lane half-row and of each 16-lane row, which read a
// lane of the other half whose partial sum equals its own by then; then the
// 16- and 32-lane halves through __shfl_xor.  Each step adds a value to its
// partner's in either order, so all lanes end bitwise equal.
__device__ __forceinline__ double group_sum(double x, int G) {
    if (G >= 2) x += dpp_f64<0xB1>(x);
    if (G >= 4) x += dpp_f64<0x4E>(x);
    if (G >= 8) x += dpp_f64<0x141>(x);
    if (G >= 16) x += dpp_f64<0x140>(x);
    if (G >= 32) x += __shfl_xor(x, 16, 64);
    if (G >= 64) x += __shfl_xor(x, 32, 64);
    return x;
}
__device__ __forceinline__ cplx group_sum(cplx x, int G) { return cplx{group_sum(x.re, G), group_sum(x.im, G)}; }
__device__ __forceinline__ double wave_sum(double x) { return group_sum(x, 64); }
__device__ __forceinline__ double wave_max(double x) {
    x = fmax(x, dpp_f64<0xB1>(x));
    x = fmax(x, dpp_f64<0x4E>(x));
    x = fmax(x, dpp_f64<0x141>(x));
    x = fmax(x, dpp_f64<0x140>(x));
    x = fmax(x, __shfl_xor(x, 16, 64));
    return fmax(x, __shfl_xor(x, 32, 64));
}
// Ordering of LDS accesses among the lanes of one wavefront: LDS executes a
// wavefront's instructions in issue order, so a compiler-level fence at
// wavefront scope is all that a one-wavefront workgroup needs between a
// write and another lane's read (no wait for outstanding LDS work).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// x of lane src (src the same in every lane), read from the register file.
__device__ __forceinline__ double lane_f64(double x, int src) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Rotation (c, s) with c^2 + s^2 = 1 to working precision that annihilates
// the off-diagonal of the real 2x2 [[a, g], [g, b]] (g > 0): t = tan(phi) is
// the root of t^2 + 2 theta t - 1 = 0 of smaller modulus, theta = (b-a)/(2g).
__device__ __forceinline__ void jacobi_cs(double a, double b, double g, double& c, double& s) {
    const double theta = 0.5 * (b - a) * rcp_fast(g);
    double t;
    if (fabs(theta) > 1e100) {
        t = 0.5 * rcp_fast(theta);
    } else {
        const double q = fma(theta, theta, 1.0);
        const double den = fabs(theta) + q * rsqrt_acc(q);
        t = copysign(rcp_fast(den), theta);
        if (theta == 0.0) t = 1.0;
    }
    c = rsqrt_acc(fma(t, t, 1.0));
    s = t * c;
}

// Copies the results block (state, sigma, lambda) to its pinned host mirror so
// that the host reads a consistent snapshot of this solve after one event wait.
__device__ void publish(const SolveArgs& a) {
    __syncthreads();
    const int n4 = a.res_bytes / 4;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.res_block);
    volatile uint32_t* dst = reinterpret_cast<volatile uint32_t*>(a.res_host);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) dst[i] = src[i];
    __threadfence_system();
}

// --------------------------------------------------------------------------
// k_solve_sym
// --------------------------------------------------------------------------

// C = op(A) B for M x M matrices with leading dimension ld (op = identity or
// conjugate transpose).  LDS path: each thread owns a 4 x 4 block with rows
// strided by 16 so that a wavefront reads 16 consecutive rows per access.
template <typename S, int NT, bool CONJ_A>
__device__ void gemm_sq(S* __restrict__ C, const S* __restrict__ A, const S* __restrict__ B, int M, int ld) {
    using SC = Scal<S>;
    const int nrg = (M + 63) / 64;  // row/column super-groups of 64
    for (int t = threadIdx.x; t < 256 * nrg * nrg; t += NT) {
        const int g = t / 256, w = t % 256;
        const int i0 = (g % nrg) * 64 + (w % 16), j0 = (g / nrg) * 64 + (w / 16);
        S acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = SC::zero();
        for (int k = 0; k < M; ++k) {
            S av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * r;
                av[r] = i < M ? (CONJ_A ? SC::cj(A[k + (size_t)i * ld]) : A[i + (size_t)k * ld]) : SC::zero();
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int j = j0 + 16 * c;
                bv[c] = j < M ? B[k + (size_t)j * ld] : SC::zero();
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = acc[r][c] + mulr(av[r], bv[c]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = i0 + 16 * r, j = j0 + 16 * c;
                if (i < M && j < M) C[i + (size_t)j * ld] = acc[r][c];
            }
    }
}

template <typename S> __device__ __forceinline__ S load_s(const double* p, int64_t i);
template <> __device__ __forceinline__ double load_s<double>(const double* p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ cplx load_s<cplx>(const double* p, int64_t i) { return cplx{p[2 * i], p[2 * i + 1]}; }

// Common end of the symmetric solves: sigma sorted descending (stable in the
// index) with V permuted alike (Algorithm 1), the rank r_eff, canonical V_r,
// A~ = Sigma^-1 V_r^* xty V_r Sigma^-1 (Eq. Atilde, Algorithm 2), the POD
// coefficients V_r Sigma^-1 and the status.
// s_sig[i]: sigma of eigenvector i (i < m); Vc: eigenvectors by column
// (leading dimension ld), the first nvec of them valid (nvec >= r_eff);
// spare1, spare2: M x ld scratch.
template <typename S, int NT, int AHEAD = 1>
__device__ void sym_tail(const SolveArgs& a, int ld, S* Vc, S* spare1, S* spare2, double* s_sig, int* s_perm,
                         int nvec, int sweeps, bool converged, int warm) {
    using SC = Scal<S>;
    const int tid = threadIdx.x;
    const int slots = a.slots;
    DevState* st = a.st;
    const int m = window_cols(a.m, a.buildup, st);  // columns of X (fewer during a build-up start)
    const int ldv = a.m;                            // storage stride of V and V_full
    const int oldest = st->oldest;
    const int nw = NT / 64, lane = tid & 63, wv = tid >> 6;
    __shared__ int s_reff;
    for (int i = m + tid; i < a.m; i += NT) a.sigma[i] = 0.0;
    // sigma = sqrt(|d|), sorted descending (stable in the index)
    for (int i = tid; i < m; i += NT) {
        const double si = s_sig[i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double sj = s_sig[j];
            rank += (sj > si) || (sj == si && j < i);
        }
        s_perm[rank] = i;
        a.sigma[rank] = si;
    }
    __syncthreads();
    if (tid == 0) {
        const double s0 = s_sig[s_perm[0]];
        int k = 0;
        if (s0 > 0.0) {
            const double thr = a.rcond * s0;
            const int lim = a.r < m ? a.r : m;
            while (k < lim && s_sig[s_perm[k]] > thr) ++k;
        }
        s_reff = k;
    }
    // the eigenvectors in sigma order, kept for the next solve's warm start
    // (only when all m are known and the window is full)
    const bool keep_full = nvec >= m && m == ldv;
    if (keep_full) {
        for (int idx = tid; idx < m * m; idx += NT) {
            const int i = idx % m, k = idx / m;
            store_s<S>(a.Vfull, i + (int64_t)k * ldv, Vc[i + (size_t)s_perm[k] * ld]);
        }
    }
    __syncthreads();
    const int k_eff = s_reff;

    // canonical V_r: column perm[k] of V, phase so that its largest-modulus
    // entry (lowest index on ties) is real positive
    S* Vr = spare1;  // m x k_eff, leading dimension ld
    for (int k = wv; k < k_eff; k += nw) {
        const int col = s_perm[k];
        double best = -1.0;
        int bi = 0;
        for (int i = lane; i < m; i += 64) {
            const double v = SC::absv(Vc[i + (size_t)col * ld]);
            if (v > best) { best = v; bi = i; }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const S ph = SC::cj(SC::phase(Vc[bi + (size_t)col * ld]));
        for (int i = lane; i < m; i += 64) {
            const S v = mulr(Vc[i + (size_t)col * ld], ph);
            Vr[i + (size_t)k * ld] = v;
            store_s<S>(a.V, i + (int64_t)k * ldv, v);
        }
        for (int i = m + lane; i < ldv; i += 64) store_s<S>(a.V, i + (int64_t)k * ldv, SC::zero());
    }
    __syncthreads();

    // T = xty V_r (m x k_eff) with xty[i][j] = <x_i, x_{j+1}>
    S* T = spare2;
    for (int idx = tid; idx < m * k_eff; idx += NT) {
        const int i = idx % m, b = idx / m;
        const int si = slot_of(oldest, i, slots);
        const S acc = ordered_dot<AHEAD>(SC::zero(), 0, 1, m,
                                     [&](int j) { return gram_at<S>(a.G, si, slot_of(oldest, j + 1, slots), slots); },
                                     [&](int j) { return Vr[j + (size_t)b * ld]; });
        T[i + (size_t)b * ld] = acc;
    }
    __syncthreads();

    // A~[p][q] = (V_r^* T)[p][q] / (sigma_p sigma_q)
    for (int idx = tid; idx < k_eff * k_eff; idx += NT) {
        const int p = idx % k_eff, q = idx / k_eff;
        const S acc = ordered_dot<AHEAD>(SC::zero(), 0, 1, m, [&](int i) { return SC::cj(Vr[i + (size_t)p * ld]); },
                                     [&](int i) { return T[i + (size_t)q * ld]; });
        const double sp = s_sig[s_perm[p]], sq = s_sig[s_perm[q]];
        store_s<S>(a.At, p + (int64_t)q * k_eff, acc * (1.0 / (sp * sq)));
    }
    // POD coefficients V_r Sigma^-1 (row-major m x r, real or interleaved complex)
    const int cw = (sizeof(S) == sizeof(cplx)) ? 2 : 1;
    for (int idx = tid; idx < m * k_eff; idx += NT) {
        const int i = idx / k_eff, q = idx % k_eff;
        const S v = Vr[i + (size_t)q * ld] * (1.0 / s_sig[s_perm[q]]);
        const cplx cv = SC::toc(v);
        const int64_t o = (int64_t)i * cw * a.r + (int64_t)cw * q;
        if (a.coef_f64) {
            double* B = reinterpret_cast<double*>(a.Bpod);
            B[o] = cv.re;
            if (cw == 2) B[o + 1] = cv.im;
        } else {
            float* B = reinterpret_cast<float*>(a.Bpod);
            B[o] = (float)cv.re;
            if (cw == 2) B[o + 1] = (float)cv.im;
        }
    }
    if (tid == 0) {
        const int lim = a.r < m ? a.r : m;
        st->skipped = 0;
        st->r_eff = k_eff;
        st->sweeps = sweeps;
        st->solve_status = converged ? (k_eff < lim ? ST_W_RANK : ST_OK) : ST_E_CONVERGENCE;
        if (k_eff == 0) st->solve_status = ST_W_RANK;
        st->vprev_valid = (converged && keep_full) ? 1 : 0;
        st->vprev_push = st->pushes;
        st->warm = warm;
    }
}

// LDS: matrices in dynamic LDS (real, M <= 64); else in the global workspace.
// PMAX: largest number of rotation pairs per round (M / 2).
template <typename S, int NT, bool LDS, int PMAX>
__device__ void solve_sym_body(const SolveArgs& a, int M) {
    using SC = Scal<S>;
    extern __shared__ double dyn[];
    const int tid = threadIdx.x;
    const int slots = a.slots;
    DevState* st = a.st;
    // the columns of X; a partial window (build-up) is the leading block of
    // the zero-padded M x M matrix, whose padding no rotation touches
    const int m = window_cols(a.m, a.buildup, st);
    if (m == 0) {
        if (tid == 0) {
            st->solve_status = ST_E_NOT_READY;
            st->r_eff = 0;
        }
        return;
    }
    if (st->vprev_valid && st->pushes == st->vprev_push) {
        // no snapshot was accepted since the last converged solve: its results stand
        if (tid == 0) st->skipped = 1;
        return;
    }
    const int oldest = st->oldest;
    const int ld = M + 1;  // odd leading dimension: column accesses spread over LDS banks
    const size_t MM = (size_t)M * ld;
    S* bufA;
    if constexpr (LDS) bufA = reinterpret_cast<S*>(dyn);
    else bufA = reinterpret_cast<S*>(a.work);
    S* bufV = bufA + MM;
    S* bufQ = bufV + MM;
    const int P = M / 2;

    __shared__ double s_c[PMAX], s_s[PMAX];
    __shared__ S s_e[PMAX];
    __shared__ int s_p[PMAX], s_q[PMAX];
    __shared__ int s_rot, s_warm;
    __shared__ double s_red[NT / 64];
    __shared__ double s_sig[2 * PMAX];
    __shared__ int s_perm[2 * PMAX];

    if (tid == 0) {
        // warm start from the previous solve's eigenvectors when the window
        // moved by exactly one snapshot (or not at all) since then
        int w = 0;
        if (a.warm_start && st->vprev_valid) {
            if (st->pushes == st->vprev_push + 1) w = 1;
            else if (st->pushes == st->vprev_push) w = 2;
        }
        s_warm = w;
    }
    // xtx = Gram of the first m window columns; padded to even M with a decoupled zero
    for (int idx = tid; idx < M * M; idx += NT) {
        const int i = idx % M, j = idx / M;
        S v = SC::zero();
        if (i < m && j < m) v = gram_at<S>(a.G, slot_of(oldest, i, slots), slot_of(oldest, j, slots), slots);
        bufA[i + (size_t)j * ld] = v;
    }
    __syncthreads();
    const int warm = s_warm;
    if (warm) {
        // Q = previous eigenvectors with rows shifted by one window position:
        // row i of Q is row i+1 of the previous V and the last row is the
        // previous first row (the departed snapshot), so Q stays unitary and
        // Q^* xtx Q is close to diagonal.
        const int shift = warm == 1 ? 1 : 0;
        for (int idx = tid; idx < M * M; idx += NT) {
            const int i = idx % M, j = idx / M;
            S v = (i == j) ? SC::one() : SC::zero();
            if (i < m && j < m) {
                int src = i + shift;
                if (src >= m) src -= m;
                v = load_s<S>(a.Vfull, src + (int64_t)j * a.m);
            }
            bufQ[i + (size_t)j * ld] = v;
        }
        __syncthreads();
        gemm_sq<S, NT, false>(bufV, bufA, bufQ, M, ld);  // T = xtx Q
        __syncthreads();
        gemm_sq<S, NT, true>(bufA, bufQ, bufV, M, ld);   // B = Q^* T
        __syncthreads();
        for (int idx = tid; idx < M * M; idx += NT) {    // exact Hermitian symmetry
            const int i = idx % M, j = idx / M;
            if (i < j) {
                const cplx u = SC::toc(bufA[i + (size_t)j * ld]), w = conj(SC::toc(bufA[j + (size_t)i * ld]));
                const S avg = SC::fromc(0.5 * (u + w));
                bufA[i + (size_t)j * ld] = avg;
                bufA[j + (size_t)i * ld] = SC::cj(avg);
            } else if (i == j) {
                bufA[i + (size_t)i * ld] = SC::fromc(mkc(SC::re(bufA[i + (size_t)i * ld])));
            }
        }
    }
    for (int idx = tid; idx < M * M; idx += NT) {
        const int i = idx % M, j = idx / M;
        bufV[i + (size_t)j * ld] = (i == j) ? SC::one() : SC::zero();
    }
    __syncthreads();

    // rotation floor: entries below 1e-18 * trace cannot move any eigenvalue
    // that a Gram accumulated in FP64 resolves
    double tr = 0.0;
    for (int i = tid; i < m; i += NT) tr += fabs(SC::re(bufA[i + (size_t)i * ld]));
    for (int off = 32; off >= 1; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = tr;
    __syncthreads();
    tr = 0.0;
    for (int w = 0; w < NT / 64; ++w) tr += s_red[w];
    const double floor_abs = 1e-18 * tr;
    const double tol = a.tol;
    S* A = bufA;
    S* V = bufV;
    const int nw = NT / 64, lane = tid & 63, wv = tid >> 6;

    int sweep = 0;
    bool converged = false;
    for (; sweep < a.max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int rd = 0; rd < M - 1; ++rd) {
            if (tid < P) {
                int p, q;
                rr_pair(rd, tid, M, p, q);
                const S apq = A[p + (size_t)q * ld];
                const double app = SC::re(A[p + (size_t)p * ld]);
                const double aqq = SC::re(A[q + (size_t)q * ld]);
                const double g = SC::absv(apq);
                double c = 1.0, s = 0.0;
                S e = SC::one();
                if (g > floor_abs && g * g > tol * tol * fabs(app * aqq)) {
                    jacobi_cs(app, aqq, g, c, s);
                    e = SC::phase(apq);
                    s_rot = 1;
                }
                s_c[tid] = c;
                s_s[tid] = s;
                s_e[tid] = e;
                s_p[tid] = p;
                s_q[tid] = q;
            }
            __syncthreads();
            // A <- J^* A J on 2x2 blocks (rows of pair k, columns of pair l), k <= l,
            // mirrored so that A stays exactly Hermitian.  Each half-wavefront
            // owns one row pair (its rotation is uniform) and its lanes walk l.
            for (int k = 2 * wv + (lane >> 5); k < P; k += 2 * nw) {
                const double sk = s_s[k], ck = s_c[k];
                const S ek = s_e[k];
                const int p = s_p[k], q = s_q[k];
                for (int l = k + (lane & 31); l < P; l += 32) {
                    const double sl = s_s[l];
                    if (sk == 0.0 && sl == 0.0) continue;
                    if (l == k) {
                        // the pair's own 2x2 block, rotated exactly as the others
                        // (in the basis where a_pq = g e is real): the new
                        // off-diagonal is zero up to rounding of (c, s)
                        const double aa = SC::re(A[p + (size_t)p * ld]), bb = SC::re(A[q + (size_t)q * ld]);
                        const double g = SC::absv(A[p + (size_t)q * ld]);
                        const double cs = ck * sk, c2 = ck * ck, s2 = sk * sk;
                        const double na = c2 * aa - 2.0 * cs * g + s2 * bb;
                        const double nb = s2 * aa + 2.0 * cs * g + c2 * bb;
                        const double nx = cs * (aa - bb) + (c2 - s2) * g;
                        A[p + (size_t)p * ld] = SC::fromc(mkc(na));
                        A[q + (size_t)q * ld] = SC::fromc(mkc(nb));
                        A[p + (size_t)q * ld] = nx * ek;
                        A[q + (size_t)p * ld] = SC::cj(nx * ek);
                        continue;
                    }
                    const int u = s_p[l], v = s_q[l];
                    const double cl = s_c[l];
                    const S el = s_e[l];
                    const S apu = A[p + (size_t)u * ld], apv = A[p + (size_t)v * ld];
                    const S aqu = A[q + (size_t)u * ld], aqv = A[q + (size_t)v * ld];
                    // rows: p' = c p - s e q ;  q' = s conj(e) p + c q
                    const S bpu = ck * apu - sk * mulr(ek, aqu);
                    const S bpv = ck * apv - sk * mulr(ek, aqv);
                    const S bqu = sk * mulr(SC::cj(ek), apu) + ck * aqu;
                    const S bqv = sk * mulr(SC::cj(ek), apv) + ck * aqv;
                    // columns: u' = c u - s conj(e) v ;  v' = s e u + c v
                    const S npu = cl * bpu - sl * mulr(SC::cj(el), bpv);
                    const S npv = sl * mulr(el, bpu) + cl * bpv;
                    const S nqu = cl * bqu - sl * mulr(SC::cj(el), bqv);
                    const S nqv = sl * mulr(el, bqu) + cl * bqv;
                    A[p + (size_t)u * ld] = npu;
                    A[p + (size_t)v * ld] = npv;
                    A[q + (size_t)u * ld] = nqu;
                    A[q + (size_t)v * ld] = nqv;
                    A[u + (size_t)p * ld] = SC::cj(npu);
                    A[v + (size_t)p * ld] = SC::cj(npv);
                    A[u + (size_t)q * ld] = SC::cj(nqu);
                    A[v + (size_t)q * ld] = SC::cj(nqv);
                }
            }
            // V <- V J: one wavefront per pair, lanes over rows
            for (int k = wv; k < P; k += nw) {
                const double sk = s_s[k];
                if (sk == 0.0) continue;
                const double ck = s_c[k];
                const S ek = s_e[k];
                const int p = s_p[k], q = s_q[k];
                for (int i = lane; i < M; i += 64) {
                    const S vp = V[i + (size_t)p * ld], vq = V[i + (size_t)q * ld];
                    V[i + (size_t)p * ld] = ck * vp - sk * mulr(SC::cj(ek), vq);
                    V[i + (size_t)q * ld] = sk * mulr(ek, vp) + ck * vq;
                }
            }
            __syncthreads();
        }
        if (s_rot == 0) {
            converged = true;
            break;
        }
        __syncthreads();
    }

    // eigenvalues d, then eigenvectors of xtx: V (cold) or Q V (warm)
    for (int i = tid; i < m; i += NT) s_sig[i] = sqrt(fabs(SC::re(A[i + (size_t)i * ld])));
    __syncthreads();
    S* Vc;
    S* spare1;
    S* spare2;
    if (warm) {
        gemm_sq<S, NT, false>(bufA, bufQ, bufV, M, ld);
        Vc = bufA;
        spare1 = bufV;
        spare2 = bufQ;
    } else {
        Vc = bufV;
        spare1 = bufA;
        spare2 = bufQ;
    }
    sym_tail<S, NT, kAhead<S, LDS>>(a, ld, Vc, spare1, spare2, s_sig, s_perm, m, sweep + (converged ? 1 : 0), converged, warm);
}

template <typename S, int NT, bool LDS, int PMAX>
__global__ __launch_bounds__(NT)
void k_solve_sym(SolveArgs a, int M) {
    solve_sym_body<S, NT, LDS, PMAX>(a, M);
}

// Grouped form: one workgroup per stream (independent solves run on separate CUs).
template <typename S, int NT, bool LDS, int PMAX>
__global__ __launch_bounds__(NT)
void k_solve_sym_grouped(const SolveArgs* __restrict__ items) {
    const SolveArgs a = items[blockIdx.x];
    solve_sym_body<S, NT, LDS, PMAX>(a, a.m + (a.m & 1));
}

// --------------------------------------------------------------------------
// k_solve_eig: one wavefront, A~ (k x k, k <= 32) in LDS
// --------------------------------------------------------------------------
// Column stride of the k x k (k <= kRMax) matrices in LDS: one more than
// kRMax, so that a row read across lanes (lane = column) spreads over the
// LDS banks instead of hitting the same one from every lane.
constexpr int LDH = kRMax + 1;


// Real Schur form of the real upper Hessenberg k x k matrix held in the real
// parts of H (imaginary parts zero), one wavefront: implicit double-shift
// (Francis) QR -- each sweep chases a 3 x 3 Householder bulge started from
// the first column of (H - mu1)(H - mu2), mu1,2 the eigenvalues of the
// trailing 2 x 2 block (an exceptional pair every 10th sweep), so that a
// complex-conjugate pair converges together in real arithmetic; Z (complex
// storage, real values) accumulates the transformations.  The 2 x 2 blocks
// left on the diagonal are then triangularized by one complex rotation each,
// so that H becomes the complex upper triangular T of the complex Schur form.
__device__ __forceinline__ void real_schur(cplx* H, cplx* Z, int k, int lane, int max_iter, double hmax, int& total, bool& failed) {
    auto h = [&](int i, int j) -> double& { return H[i + j * LDH].re; };
    int nn = k - 1, its = 0;
    while (nn >= 0) {
        // deflation: largest l in [1, nn] with a negligible subdiagonal
        bool small = false;
        if (lane >= 1 && lane <= nn) {
            const double sub = fabs(h(lane, lane - 1));
            double scale = fabs(h(lane, lane)) + fabs(h(lane - 1, lane - 1));
            if (scale == 0.0) scale = hmax;
            small = sub <= kEps * scale;
        }
        const unsigned long long mask = __ballot(small);
        const int l = mask ? 63 - __clzll(mask) : 0;
        wave_sync();
        if (l > 0 && lane == 0) h(l, l - 1) = 0.0;
        wave_sync();
        if (l >= nn - 1) {  // a 1 x 1 or 2 x 2 block splits off
            nn = l - 1;
            its = 0;
            continue;
        }
        if (its >= max_iter) {
            failed = true;
            break;
        }
        ++its;
        ++total;
        // shift pair by its sum s and product t
        double s, t;
        {
            const double a11 = h(nn - 1, nn - 1), a12 = h(nn - 1, nn), a21 = h(nn, nn - 1), a22 = h(nn, nn);
            if (its % 10 == 0) {
                const double e = fabs(a21) + fabs(h(nn - 1, nn - 2));
                const double mu = a22 + 0.75 * e;
                s = 2.0 * mu;
                t = mu * mu + 0.4375 * e * e;
            } else {
                s = a11 + a22;
                t = a11 * a22 - a12 * a21;
            }
        }
        // (x, y, z): the first column of (H - mu1)(H - mu2) to start the
        // sweep, then the bulge below the subdiagonal of column kk-1; the
        // latter were just written by the lanes that updated column kk-1,
        // and are read from their registers (the LDS copy only when that
        // step applied no reflector)
        double x, y, z;
        {
            const double h00 = h(l, l), h10 = h(l + 1, l);
            x = h00 * h00 + h(l, l + 1) * h10 - s * h00 + t;
            y = h10 * (h00 + h(l + 1, l + 1) - s);
            z = h10 * h(l + 2, l + 1);
        }
        // One bulge step is straight-line code: every lane reads its column
        // (rows kk .. kk+2) and its row of Z (columns kk .. kk+2) before the
        // reflector is known, and lanes outside a range write to a sink
        // entry past the matrix instead of branching, so that the updates
        // of H's rows and of Z interleave.
        const int lc = lane < LDH ? lane : LDH - 1;  // this lane's column / row, clamped
        const int sink = LDH * LDH + lane;
        for (int kk = l; kk < nn; ++kk) {
            const bool three = kk + 2 <= nn;
            const double r0 = h(kk, lc), r1 = h(kk + 1, lc), r2 = h(kk + 2, lc);
            const double zc0 = Z[lc + kk * LDH].re, zc1 = Z[lc + (kk + 1) * LDH].re, zc2 = Z[lc + (kk + 2) * LDH].re;
            // (the bulge chase is a chain of dependent FP64 steps: the norm and
            // 2 / v^T v come from the hardware estimates plus Newton steps,
            // shorter chains than the correctly rounded square root and division)
            const double s2 = x * x + y * y + z * z;
            const double nrm = s2 > 0.0 ? s2 * rsqrt_acc(s2) : 0.0;
            // reflector P = I - tau v v^T, v = (x - alpha, y, z), P (x, y, z) = (alpha, 0, 0)
            // (z = 0 exactly when the step has two rows)
            const double alpha = x > 0.0 ? -nrm : nrm;
            const double v0 = x - alpha;
            const double vtv = v0 * v0 + y * y + z * z;
            const double tau = vtv > 0.0 ? 2.0 * rcp_acc(vtv) : 0.0;
            double nc0 = 0.0;  // this lane's new H[lane][kk]
            if (tau != 0.0) {
                // rows kk .. kk+2 over columns jlo .. k-1 (lane = column); the
                // entries below the subdiagonal of column kk-1 become zero
                const int jlo = kk > l ? kk - 1 : l;
                const bool rok = lane >= jlo && lane < k;
                const double f = tau * (v0 * r0 + y * r1 + z * r2);
                const bool below = kk > l && lane == kk - 1;
                H[rok ? kk + lc * LDH : sink].re = r0 - f * v0;
                H[rok ? kk + 1 + lc * LDH : sink].re = below ? 0.0 : r1 - f * y;
                H[rok && three ? kk + 2 + lc * LDH : sink].re = below ? 0.0 : r2 - f * z;
                // Z over all rows (lane = row)
                const bool zok = lane < k;
                const double fz = tau * (zc0 * v0 + zc1 * y + zc2 * z);
                Z[zok ? lc + kk * LDH : sink].re = zc0 - fz * v0;
                Z[zok ? lc + (kk + 1) * LDH : sink].re = zc1 - fz * y;
                Z[zok && three ? lc + (kk + 2) * LDH : sink].re = zc2 - fz * z;
                wave_sync();
                // columns kk .. kk+2 over rows 0 .. min(kk+3, nn) (lane = row)
                const int ihi = kk + 3 < nn ? kk + 3 : nn;
                const bool cok = lane <= ihi;
                const double c0 = h(lc, kk), c1 = h(lc, kk + 1), c2 = h(lc, kk + 2);
                const double fc = tau * (c0 * v0 + c1 * y + c2 * z);
                nc0 = c0 - fc * v0;
                H[cok ? lc + kk * LDH : sink].re = nc0;
                H[cok ? lc + (kk + 1) * LDH : sink].re = c1 - fc * y;
                H[cok && three ? lc + (kk + 2) * LDH : sink].re = c2 - fc * z;
            }
            wave_sync();
            if (kk + 1 < nn) {
                // rows kk+1 .. kk+3 of column kk (rows 0 .. kk+3 were updated above)
                const bool z3 = kk + 3 <= nn;
                if (tau != 0.0) {
                    x = lane_f64(nc0, kk + 1);
                    y = lane_f64(nc0, kk + 2);
                    z = z3 ? lane_f64(nc0, kk + 3) : 0.0;
                } else {
                    x = h(kk + 1, kk);
                    y = h(kk + 2, kk);
                    z = z3 ? h(kk + 3, kk) : 0.0;
                }
            }
        }
    }
    wave_sync();
    // triangularize each 2 x 2 diagonal block [[a, b], [c, d]], c != 0: with
    // u = (lambda_1 - d, c) / ||.||, lambda_1 an eigenvalue of the block, the
    // rotation G = [[u0, -conj(u1)], [u1, conj(u0)]] gives G^* B G = [[lambda_1, .], [0, lambda_2]]
    for (int i = 0; i + 1 < k; ++i) {
        const double c = h(i + 1, i);
        if (c == 0.0) continue;
        const double a = h(i, i), b = h(i, i + 1), d = h(i + 1, i + 1);
        const double half = 0.5 * (a - d), disc = half * half + b * c;
        cplx l1;
        if (disc >= 0.0) l1 = mkc(0.5 * (a + d) + copysign(sqrt(disc), half));
        else l1 = cplx{0.5 * (a + d), sqrt(-disc)};
        cplx u0 = l1 - mkc(d), u1 = mkc(c);
        const double nu = sqrt(abs2(u0) + abs2(u1));
        u0 = (1.0 / nu) * u0;
        u1 = (1.0 / nu) * u1;
        wave_sync();
        {
            const int j = lane;  // rows i, i+1 over columns i .. k-1
            if (j >= i && j < k) {
                const cplx r0 = H[i + j * LDH], r1 = H[(i + 1) + j * LDH];
                H[i + j * LDH] = conj_mul(u0, r0) + conj_mul(u1, r1);
                H[(i + 1) + j * LDH] = u0 * r1 - u1 * r0;
            }
        }
        wave_sync();
        {
            const int r = lane;  // columns i, i+1 over rows 0 .. i+1; Z over all rows
            if (r <= i + 1) {
                const cplx c0 = H[r + i * LDH], c1 = H[r + (i + 1) * LDH];
                H[r + i * LDH] = c0 * u0 + c1 * u1;
                H[r + (i + 1) * LDH] = mul_conj(c1, u0) - mul_conj(c0, u1);
            }
            if (r < k) {
                const cplx c0 = Z[r + i * LDH], c1 = Z[r + (i + 1) * LDH];
                Z[r + i * LDH] = c0 * u0 + c1 * u1;
                Z[r + (i + 1) * LDH] = mul_conj(c1, u0) - mul_conj(c0, u1);
            }
        }
        wave_sync();
        if (lane == 0) H[(i + 1) + i * LDH] = mkc(0.0);
        wave_sync();
        ++i;  // the next row belongs to this block
    }
}

__device__ __forceinline__ void solve_eig_body(const SolveArgs& a) {
    const int lane = threadIdx.x;
    DevState* st = a.st;
    const int status0 = st->solve_status;
    const int k = st->r_eff;
    const int m = window_cols(a.m, a.buildup, st);  // columns of X
    const int ldv = a.m;                            // leading dimension of V
    if (st->skipped) {
        publish(a);
        return;
    }
    if (status0 == ST_E_NOT_READY || k == 0) {
        if (lane == 0 && status0 != ST_E_NOT_READY) st->solves += 1;
        publish(a);
        return;
    }

    __shared__ cplx H[LDH * LDH + 64];  // (64 sink entries past the matrix)
    __shared__ cplx Z[LDH * LDH + 64];
    __shared__ cplx Y[LDH * LDH];
    __shared__ cplx hv[LDH];
    __shared__ double s_sig[kRMax];
    __shared__ int s_rank[kRMax];

    for (int idx = lane; idx < LDH * LDH; idx += 64) {
        const int i = idx % LDH, j = idx / LDH;
        cplx h = mkc(0.0);
        if (i < k && j < k) {
            if (a.cplx) h = cplx{a.At[2 * (i + j * k)], a.At[2 * (i + j * k) + 1]};
            else h = mkc(a.At[i + j * k]);
        }
        H[idx] = h;
        Z[idx] = mkc(i == j ? 1.0 : 0.0);
        Y[idx] = mkc(0.0);
    }
    if (lane < k) s_sig[lane] = a.sigma[lane];
    wave_sync();

    // ---- Householder reduction to upper Hessenberg form, Z accumulates
    for (int c = 0; c + 2 < k; ++c) {
        const int len = k - c - 1;  // rows c+1 .. k-1
        double tail2 = 0.0;
        if (lane >= 1 && lane < len) tail2 = abs2(H[(c + 1 + lane) + c * LDH]);
        tail2 = wave_sum(tail2);
        const cplx x0 = H[(c + 1) + c * LDH];
        const double ax0 = cabs(x0);
        const double alpha = sqrt(ax0 * ax0 + tail2);
        if (tail2 == 0.0) {
            wave_sync();
            continue;
        }
        const cplx ph = ax0 > 0.0 ? cplx{x0.re / ax0, x0.im / ax0} : mkc(1.0);
        // v = x + ph*alpha e1 ; v^* v = 2 alpha (alpha + |x0|) ; P = I - tau v v^*
        if (lane < len) hv[lane] = (lane == 0) ? x0 + ph * alpha : H[(c + 1 + lane) + c * LDH];
        wave_sync();
        const double tau = 1.0 / (alpha * (alpha + ax0));
        // left: rows c+1.., columns c..k-1 (lane = column)
        {
            const int j = lane;
            if (j >= c && j < k) {
                cplx w = mkc(0.0);
                for (int i = 0; i < len; ++i) w = w + conj_mul(hv[i], H[(c + 1 + i) + j * LDH]);
                w = tau * w;
                for (int i = 0; i < len; ++i) H[(c + 1 + i) + j * LDH] = H[(c + 1 + i) + j * LDH] - hv[i] * w;
            }
        }
        wave_sync();
        // right: all rows, columns c+1.. (lane = row); also Z
        {
            const int i = lane;
            if (i < k) {
                cplx w = mkc(0.0), wz = mkc(0.0);
                for (int j = 0; j < len; ++j) {
                    w = w + H[i + (c + 1 + j) * LDH] * hv[j];
                    wz = wz + Z[i + (c + 1 + j) * LDH] * hv[j];
                }
                w = tau * w;
                wz = tau * wz;
                for (int j = 0; j < len; ++j) {
                    H[i + (c + 1 + j) * LDH] = H[i + (c + 1 + j) * LDH] - mul_conj(w, hv[j]);
                    Z[i + (c + 1 + j) * LDH] = Z[i + (c + 1 + j) * LDH] - mul_conj(wz, hv[j]);
                }
            }
        }
        wave_sync();
        if (lane < len) H[(c + 1 + lane) + c * LDH] = (lane == 0) ? -(ph * alpha) : mkc(0.0);
        wave_sync();
    }

    // ---- Schur form T = Z^* A~ Z (full T and Z): real A~ by the implicit
    // double-shift QR, each 2 x 2 block then triangularized by one complex
    // rotation; complex A~ by the single-shift complex QR
    double hmax = 0.0;
    for (int idx = lane; idx < k * k; idx += 64) hmax = fmax(hmax, cabs(H[(idx % k) + (idx / k) * LDH]));
    hmax = wave_max(hmax);
    const double smallnum = (hmax > 0.0 ? hmax : 1.0) * kEps;

    int total = 0;
    bool failed = false;
    const int max_iter = a.max_qr_iter;
    if (!a.cplx) {
        real_schur(H, Z, k, lane, max_iter, hmax, total, failed);
    } else {
    int hi = k - 1, iter = 0;
    while (hi > 0) {
        // deflation: largest l in [1, hi] with a negligible subdiagonal
        bool small = false;
        if (lane >= 1 && lane <= hi) {
            const double sub = cabs(H[lane + (lane - 1) * LDH]);
            double scale = cabs(H[lane + lane * LDH]) + cabs(H[(lane - 1) + (lane - 1) * LDH]);
            if (scale == 0.0) scale = hmax;
            small = sub <= kEps * scale;
        }
        const unsigned long long mask = __ballot(small);
        const int l = mask ? 63 - __clzll(mask) : 0;
        wave_sync();
        if (l > 0 && lane == 0) H[l + (l - 1) * LDH] = mkc(0.0);
        wave_sync();
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (iter >= max_iter) {
            failed = true;
            break;
        }
        ++iter;
        ++total;
        // Wilkinson shift: eigenvalue of the trailing 2x2 closer to H[hi][hi];
        // every 10th iteration an exceptional shift
        const cplx ta = H[(hi - 1) + (hi - 1) * LDH], tb = H[(hi - 1) + hi * LDH];
        const cplx tc = H[hi + (hi - 1) * LDH], td = H[hi + hi * LDH];
        cplx mu;
        if (iter % 10 == 0) {
            mu = td + mkc(0.75 * cabs(tc));
        } else {
            const cplx half = 0.5 * (ta - td);
            const cplx disc = csqrt(half * half + tb * tc);
            const cplx mu1 = td + half + disc, mu2 = td + half - disc;
            // (a+d)/2 +- disc == d + (a-d)/2 +- disc
            mu = (cabs(mu1 - td) <= cabs(mu2 - td)) ? mu1 : mu2;
        }
        // (x, y): the shifted first column to start the sweep, then the
        // bulge below the subdiagonal of column kk-1, read from the registers
        // of the lanes that just updated that column
        cplx x = H[l + l * LDH] - mu, y = H[(l + 1) + l * LDH];
        // straight-line steps as in the real sweep: loads first, lanes
        // outside a range write to a sink entry past the matrix
        const int lc = lane < LDH ? lane : LDH - 1;
        const int sink = LDH * LDH + lane;
        for (int kk = l; kk < hi; ++kk) {
            const cplx ru = H[kk + lc * LDH], rv = H[(kk + 1) + lc * LDH];
            const cplx zu = Z[lc + kk * LDH], zv = Z[lc + (kk + 1) * LDH];
            // G = [[c, s], [-conj(s), c]] with G [x; y] = [rho; 0]:
            // c = |x| / r, s = (x / |x|) conj(y) / r, r^2 = |x|^2 + |y|^2
            double c;
            cplx s;
            const double x2 = abs2(x), y2 = abs2(y);
            if (y2 == 0.0) {
                c = 1.0;
                s = mkc(0.0);
            } else if (x2 == 0.0) {
                c = 0.0;
                s = mkc(1.0);
            } else if (x2 > 1e-250 && y2 > 1e-250 && x2 < 1e250 && y2 < 1e250) {
                const double rx = rsqrt_acc(x2), rr = rsqrt_acc(x2 + y2);
                c = x2 * rx * rr;
                s = (rx * rr) * mul_conj(x, y);
            } else {
                const double ax = cabs(x), rr = hypot(ax, cabs(y));
                c = ax / rr;
                s = (1.0 / rr) * mul_conj(cplx{x.re / ax, x.im / ax}, y);
            }
            // rows kk, kk+1 over columns jlo .. k-1 (lane = column); the entry
            // below the subdiagonal of column kk-1 becomes zero.  Z over all
            // rows (lane = row).
            {
                const int jlo = kk > l ? kk - 1 : l;
                const bool rok = lane >= jlo && lane < k;
                const bool below = kk > l && lane == kk - 1;
                H[rok ? kk + lc * LDH : sink] = c * ru + s * rv;
                H[rok ? (kk + 1) + lc * LDH : sink] = below ? mkc(0.0) : c * rv - conj_mul(s, ru);
                const bool zok = lane < k;
                Z[zok ? lc + kk * LDH : sink] = c * zu + mul_conj(zv, s);
                Z[zok ? lc + (kk + 1) * LDH : sink] = c * zv - zu * s;
            }
            wave_sync();
            // columns kk, kk+1 over rows 0 .. min(kk+2, hi) (lane = row)
            cplx nc;  // this lane's new H[lane][kk]
            {
                const int ihi = kk + 2 < hi ? kk + 2 : hi;
                const bool cok = lane <= ihi;
                const cplx u = H[lc + kk * LDH], v = H[lc + (kk + 1) * LDH];
                nc = c * u + mul_conj(v, s);
                H[cok ? lc + kk * LDH : sink] = nc;
                H[cok ? lc + (kk + 1) * LDH : sink] = c * v - u * s;
            }
            wave_sync();
            if (kk + 1 < hi) {  // rows kk+1, kk+2 of column kk (both updated above)
                x = cplx{lane_f64(nc.re, kk + 1), lane_f64(nc.im, kk + 1)};
                y = cplx{lane_f64(nc.re, kk + 2), lane_f64(nc.im, kk + 2)};
            }
        }
    }
    }
    wave_sync();

    // ---- eigenvectors of the triangular T: (T - t_qq) y = 0, y_q = 1 (lane q)
    {
        const int q = lane;
        if (q < k) {
            const cplx lq = H[q + q * LDH];
            for (int i = k - 1; i > q; --i) Y[i + q * LDH] = mkc(0.0);
            Y[q + q * LDH] = mkc(1.0);
            for (int i = q - 1; i >= 0; --i) {
                cplx acc = mkc(0.0);
                for (int j = i + 1; j <= q; ++j) acc = acc + H[i + j * LDH] * Y[j + q * LDH];
                cplx d = H[i + i * LDH] - lq;
                if (cabs(d) < smallnum) d = mkc(smallnum);
                Y[i + q * LDH] = -cdiv(acc, d);
            }
        }
    }
    wave_sync();
    // W = Z Y (lane = row), written over T
    cplx lam_q = mkc(0.0);
    if (lane < k) lam_q = H[lane + lane * LDH];
    wave_sync();
    {
        const int i = lane;
        if (i < k) {
            for (int q = 0; q < k; ++q) {
                cplx acc = mkc(0.0);
                for (int j = 0; j <= q; ++j) acc = acc + Z[i + j * LDH] * Y[j + q * LDH];
                H[i + q * LDH] = acc;  // T is no longer needed
            }
        }
    }
    wave_sync();
    // normalise column q (lane q): unit norm, largest-modulus entry (lowest
    // index on ties) real positive; rank by |lambda| descending, arg ascending
    __shared__ cplx s_lam[kRMax];
    __shared__ int s_partner[kRMax];
    if (lane < k) s_lam[lane] = lam_q;
    wave_sync();
    if (!a.cplx) {
        // A real A~ has a spectrum closed under conjugation.  The complex QR
        // returns each conjugate pair with independent rounding; pair them
        // up and make the member with negative imaginary part the exact
        // conjugate of its partner (eigenvector too), and make numerically
        // real eigenvalues exactly real, so that the order of eigenpairs does
        // not depend on rounding.
        const double dl = 1e-10;
        int partner = -1;
        if (lane < k && lam_q.im < -dl * cabs(lam_q)) {
            double best = 1e300;
            for (int p = 0; p < k; ++p) {
                const cplx lp = s_lam[p];
                if (!(lp.im > dl * cabs(lp))) continue;
                const double d = cabs(conj(lp) - lam_q);
                if (d < best) { best = d; partner = p; }
            }
        }
        if (lane < k) s_partner[lane] = partner;
        wave_sync();
        // accept the pairing only if it is a bijection between the two halves
        int npos = 0, nneg = 0, ok = 1;
        for (int p = 0; p < k; ++p) {
            const cplx lp = s_lam[p];
            if (lp.im > dl * cabs(lp)) ++npos;
            if (lp.im < -dl * cabs(lp)) {
                ++nneg;
                if (s_partner[p] < 0) ok = 0;
                for (int q2 = 0; q2 < p; ++q2)
                    if (s_partner[q2] == s_partner[p] && s_partner[p] >= 0) ok = 0;
            }
        }
        ok = ok && (npos == nneg);
        wave_sync();
        if (ok && lane < k) {
            const int pr = s_partner[lane];
            if (pr >= 0) {
                lam_q = conj(s_lam[pr]);
                for (int i = 0; i < k; ++i) H[i + lane * LDH] = conj(H[i + pr * LDH]);
            } else if (!(lam_q.im > dl * cabs(lam_q))) {
                lam_q.im = 0.0;
            }
        }
        wave_sync();
        if (lane < k) s_lam[lane] = lam_q;
        wave_sync();
    }
    __shared__ double s_mod[kRMax], s_arg[kRMax];
    __shared__ cplx s_ls[kRMax];  // eigenvalues in sorted order
    if (lane < k) {
        s_mod[lane] = cabs(lam_q);
        s_arg[lane] = atan2(lam_q.im, lam_q.re);
    }
    wave_sync();
    if (lane < k) {
        const int q = lane;
        double nrm2 = 0.0, best = -1.0;
        int bi = 0;
        for (int i = 0; i < k; ++i) {
            const double v = abs2(H[i + q * LDH]);
            nrm2 += v;
            if (v > best) { best = v; bi = i; }
        }
        const cplx piv = H[bi + q * LDH];
        const double ap = cabs(piv);
        const cplx ph = ap > 0.0 ? cplx{piv.re / ap, -piv.im / ap} : mkc(1.0);
        const cplx scale_q = (nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 1.0) * ph;
        const double mq = s_mod[q], aq = s_arg[q];
        int rank = 0;
        for (int p = 0; p < k; ++p) {
            const double mp = s_mod[p], app = s_arg[p];
            rank += (mp > mq) || (mp == mq && app < aq) || (mp == mq && app == aq && p < q);
        }
        s_rank[q] = rank;
        s_ls[rank] = lam_q;
        a.lam[2 * rank] = lam_q.re;
        a.lam[2 * rank + 1] = lam_q.im;
        for (int i = 0; i < k; ++i) {
            const cplx w = H[i + q * LDH] * scale_q;
            Y[i + rank * LDH] = w;  // sorted, canonical W
            a.W[2 * (i + (int64_t)rank * k)] = w.re;
            a.W[2 * (i + (int64_t)rank * k) + 1] = w.im;
        }
    }
    wave_sync();

    // ---- mode amplitudes b = (W Lambda)^-1 alpha_1 (Sec. 3.3), alpha_1 = the
    // POD coefficients of the first snapshot = Sigma_r V_r^* e_1 (first row
    // of V_r); Gaussian elimination with partial pivoting on W Lambda (in H,
    // free now), lanes over rows.  Then the background mode argmin |log
    // lambda| (Algorithm 3) and its factor b_i lambda_i^m for the newest
    // snapshot.
    __shared__ cplx s_rhs[kRMax];
    __shared__ cplx s_fbg;
    __shared__ int s_bg;
    for (int idx = lane; idx < k * k; idx += 64) {
        const int i = idx % k, q = idx / k;
        H[i + q * LDH] = Y[i + q * LDH] * s_ls[q];
    }
    if (lane < k) {
        const cplx v0 = a.cplx ? cplx{a.V[2 * ((int64_t)lane * ldv)], a.V[2 * ((int64_t)lane * ldv) + 1]}
                               : mkc(a.V[(int64_t)lane * ldv]);
        s_rhs[lane] = s_sig[lane] * conj(v0);
    }
    wave_sync();
    for (int c = 0; c < k; ++c) {
        double best = -1.0;
        int bi = c;
        if (lane >= c && lane < k) {
            best = abs2(H[lane + c * LDH]);
            bi = lane;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (bi != c) {
            for (int j = lane; j < k; j += 64) {
                const cplx t = H[c + j * LDH];
                H[c + j * LDH] = H[bi + j * LDH];
                H[bi + j * LDH] = t;
            }
            if (lane == 0) {
                const cplx t = s_rhs[c];
                s_rhs[c] = s_rhs[bi];
                s_rhs[bi] = t;
            }
        }
        wave_sync();
        const cplx piv = H[c + c * LDH];
        if (lane > c && lane < k) {
            const cplx f = cdiv(H[lane + c * LDH], piv);
            for (int j = c + 1; j < k; ++j) H[lane + j * LDH] = H[lane + j * LDH] - f * H[c + j * LDH];
            s_rhs[lane] = s_rhs[lane] - f * s_rhs[c];
        }
        wave_sync();
    }
    for (int c = k - 1; c >= 0; --c) {
        if (lane == 0) s_rhs[c] = cdiv(s_rhs[c], H[c + c * LDH]);
        wave_sync();
        if (lane < c) s_rhs[lane] = s_rhs[lane] - H[lane + c * LDH] * s_rhs[c];
        wave_sync();
    }
    if (lane < k) {
        a.amp[2 * lane] = s_rhs[lane].re;
        a.amp[2 * lane + 1] = s_rhs[lane].im;
    }
    // background mode: lane q evaluates |log lambda_q|, then the smallest
    // (lowest q on ties) over the lanes with lambda_q != 0; mode 0 if none
    {
        bool ok = false;
        double d = 0.0;
        if (lane < k) {
            const cplx lq = s_ls[lane];
            const double mod = cabs(lq);
            if (mod > 0.0) {
                ok = true;
                d = hypot(log(mod), atan2(lq.im, lq.re));
            }
        }
        int bi = lane;
        for (int off = 32; off >= 1; off >>= 1) {
            const bool ook = __shfl_xor((int)ok, off, 64) != 0;
            const double od = __shfl_xor(d, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            const bool take = ook && (!ok || od < d || (od == d && oi < bi));
            if (take) {
                ok = true;
                d = od;
                bi = oi;
            }
        }
        if (lane == 0) s_bg = ok ? bi : 0;
    }
    wave_sync();
    if (lane == 0) {
        const int bi = s_bg;
        st->bg_index = bi;
        // lambda^m = |lambda|^m e^{i m arg lambda}
        const cplx lb = s_ls[bi];
        const double pm = pow(cabs(lb), (double)m), th = (double)m * atan2(lb.im, lb.re);
        s_fbg = s_rhs[bi] * cplx{pm * cos(th), pm * sin(th)};
    }
    wave_sync();
    const int bgq = s_bg;
    const cplx fbg = s_fbg;

    // ---- C = V_r Sigma^-1 W (m x k complex), row-major with row stride 2 r;
    // lane i keeps row i of V_r Sigma^-1 in registers, W (sorted) is in LDS
    for (int i = lane; i < m; i += 64) {
        // (columns past k-1 read column k-1 and are zeroed: every load in flight at once)
        cplx vrow[kRMax];
#pragma unroll
        for (int p = 0; p < kRMax; ++p) {
            const int pc = p < k ? p : k - 1;
            cplx v;
            if (a.cplx) v = cplx{a.V[2 * (i + (int64_t)pc * ldv)], a.V[2 * (i + (int64_t)pc * ldv) + 1]};
            else v = mkc(a.V[i + (int64_t)pc * ldv]);
            vrow[p] = p < k ? v * (1.0 / s_sig[pc]) : mkc(0.0);
        }
        // two columns q at a time: four independent accumulation chains (the
        // sums of each column keep their order)
        auto emit = [&](int q, const cplx& acc) {
            if (q == bgq && a.Bbg) {
                // background coefficients beta_i = C[i][bg] b_bg lambda_bg^m
                const cplx bt = acc * fbg;
                if (a.coef_f64) {
                    reinterpret_cast<double*>(a.Bbg)[2 * i] = bt.re;
                    reinterpret_cast<double*>(a.Bbg)[2 * i + 1] = bt.im;
                } else {
                    reinterpret_cast<float*>(a.Bbg)[2 * i] = (float)bt.re;
                    reinterpret_cast<float*>(a.Bbg)[2 * i + 1] = (float)bt.im;
                }
            }
            const int64_t o = (int64_t)i * 2 * a.r + 2 * q;
            if (a.coef_f64) {
                double* B = reinterpret_cast<double*>(a.Bphi);
                B[o] = acc.re;
                B[o + 1] = acc.im;
            } else {
                float* B = reinterpret_cast<float*>(a.Bphi);
                B[o] = (float)acc.re;
                B[o + 1] = (float)acc.im;
            }
        };
        for (int q = 0; q < k; q += 2) {
            const int q1 = q + 1 < k ? q + 1 : q;
            cplx a0 = mkc(0.0), a1 = mkc(0.0), b0 = mkc(0.0), b1 = mkc(0.0);
            // (the reads of Y stay under p < k: unconditional, the compiler
            // hoists them all and the grouped kernel needs more registers
            // than a retiring projection workgroup frees)
#pragma unroll
            for (int p = 0; p < kRMax; p += 2) {
                if (p < k) {
                    a0 = a0 + vrow[p] * Y[p + q * LDH];
                    b0 = b0 + vrow[p] * Y[p + q1 * LDH];
                }
                if (p + 1 < k) {
                    a1 = a1 + vrow[p + 1] * Y[p + 1 + q * LDH];
                    b1 = b1 + vrow[p + 1] * Y[p + 1 + q1 * LDH];
                }
            }
            emit(q, a0 + a1);
            if (q + 1 < k) emit(q + 1, b0 + b1);
        }
    }
    if (lane == 0) {
        st->qr_iters = total;
        if (failed) st->solve_status = ST_E_CONVERGENCE;
        st->solves += 1;
    }
    publish(a);
}

__global__ __launch_bounds__(64)
void k_solve_eig(SolveArgs a) {
    solve_eig_body(a);
    if (a.snap_st) {
        // the snapshot of this solve (state and mode coefficients) for the
        // projections that may run beside the next push
        __syncthreads();
        const uint4* B = static_cast<const uint4*>(a.Bphi);
        uint4* out = static_cast<uint4*>(a.snap_B);
        for (int i = threadIdx.x; i < a.snap_n16; i += blockDim.x) out[i] = B[i];
        if (threadIdx.x == 0) *a.snap_st = *a.st;
    }
}

__global__ __launch_bounds__(64)
void k_solve_eig_grouped(const SolveArgs* __restrict__ items) {
    const SolveArgs a = items[blockIdx.x];
    solve_eig_body(a);
}

// --------------------------------------------------------------------------
// k_solve_trid: the symmetric solve of k_solve_sym by a method with O(m)
// dependent steps instead of O(m) per Jacobi sweep, for large windows:
//   1. Householder reduction of xtx to a real symmetric tridiagonal T
//      (Hermitian input: complex reflectors, T still real);
//   2. all eigenvalues of T by multisection: 256 / m lanes per eigenvalue
//      (m rounded up to a power of two) evaluate Sturm counts at equally
//      spaced points of its bracket;
//   3. eigenvectors of T for the r largest |eigenvalues| by twisted
//      factorizations (forward L D L^T and backward U D U^T of T - lambda I,
//      twist where |gamma_k| is smallest, then the two one-term recurrences),
//      re-orthogonalized where two eigenvalues nearly coincide;
//   4. back-transformation by the reflectors, one half-wavefront per vector.
// The result feeds the same tail as the Jacobi solve.
// --------------------------------------------------------------------------

// Eigenvalues of the tridiagonal (d, e2 = e^2), scaled so that every Gershgorin
// radius is at most 1, below x: sign changes of the leading principal minors
// p_k = (d_k - x) p_{k-1} - e_{k-1}^2 p_{k-2} (an exact zero counts as a sign
// change), rescaled by powers of two to stay in range.  |p_k| grows at most
// threefold per step, so the range is checked every fourth step.
__device__ __forceinline__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n,
                                           double x) {
    double a = 1.0, b = d[0] - x;
    if (b == 0.0) b = -0x1p-900;
    int cnt = b < 0.0;
    auto step = [&](int k) {
        double c = fma(d[k] - x, b, -e2[k - 1] * a);
        if (c == 0.0) c = -copysign(0x1p-900, b);
        cnt += (int)(((unsigned long long)__double_as_longlong(c) ^ (unsigned long long)__double_as_longlong(b)) >> 63);
        a = b;
        b = c;
    };
    auto rescale = [&]() {
        const double ab = fabs(b);
        if (ab > 0x1p500 || ab < 0x1p-500) {
            const double sc = ab > 1.0 ? 0x1p-500 : 0x1p500;
            a *= sc;
            b *= sc;
        }
    };
    int k = 1;
    for (; k + 3 < n; k += 4) {
        step(k);
        step(k + 1);
        step(k + 2);
        step(k + 3);
        rescale();
    }
    for (; k < n; ++k) {
        step(k);
        rescale();
    }
    return cnt;
}

template <typename S> __device__ __forceinline__ S shfl_xor_s(S v, int off, int width);
template <> __device__ __forceinline__ double shfl_xor_s<double>(double v, int off, int width) {
    return __shfl_xor(v, off, width);
}
template <> __device__ __forceinline__ cplx shfl_xor_s<cplx>(cplx v, int off, int width) {
    return cplx{__shfl_xor(v.re, off, width), __shfl_xor(v.im, off, width)};
}

__device__ __forceinline__ double div_s(double a, double b) { return a / b; }
__device__ __forceinline__ cplx div_s(cplx a, cplx b) { return cdiv(a, b); }

// Householder reflector of column j (one wavefront): H = I - tau v v^* maps
// x = A[j+1.., j] to (beta, 0, ..); v = (1, x[1..] / (alpha - beta)) is stored
// over x[1..] and into vbuf, with tau, beta = e_j and d_j = A[j][j].
template <typename S>
__device__ void householder_col(S* A, int ld, int n, int j, S* vbuf, S* s_tau, double* s_e, double* s_d) {
    using SC = Scal<S>;
    const int lane = threadIdx.x & 63;
    const int L = n - j - 1;
    S* col = A + (size_t)j * ld + (j + 1);
    double xn2 = 0.0;
    for (int i = 1 + lane; i < L; i += 64) {
        const double ax = SC::absv(col[i]);
        xn2 += ax * ax;
    }
    xn2 = wave_sum(xn2);
    const S alpha = col[0];
    const double ar = SC::re(alpha), aa = SC::absv(alpha);
    S tau = SC::zero(), scal = SC::zero();
    double beta = ar;
    if (!(xn2 == 0.0 && aa == ar)) {
        beta = -copysign(sqrt(aa * aa + xn2), ar);
        tau = (SC::fromc(mkc(beta)) - alpha) * (1.0 / beta);
        scal = div_s(SC::one(), alpha - SC::fromc(mkc(beta)));
    }
    for (int i = 1 + lane; i < L; i += 64) {
        const S v = mulr(col[i], scal);
        col[i] = v;
        vbuf[i] = v;
    }
    if (lane == 0) {
        vbuf[0] = SC::one();
        s_tau[j] = tau;
        s_e[j] = beta;
        s_d[j] = SC::re(A[j + (size_t)j * ld]);
    }
}

template <typename S, int NT, bool LDS>
__device__ void solve_trid_body(const SolveArgs& a) {
    using SC = Scal<S>;
    extern __shared__ double dyn[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int slots = a.slots;
    DevState* st = a.st;
    const int m = window_cols(a.m, a.buildup, st), n = m;  // fewer columns during a build-up start
    if (m == 0) {
        if (tid == 0) {
            st->solve_status = ST_E_NOT_READY;
            st->r_eff = 0;
        }
        return;
    }
    if (st->vprev_valid && st->pushes == st->vprev_push) {
        if (tid == 0) st->skipped = 1;
        return;
    }
    const int oldest = st->oldest;
    const int ld = n + 1;
    const int nv = a.r < n ? a.r : n;  // eigenvectors computed: the r largest |eigenvalues|

    __shared__ double s_d[kMaxM], s_e[kMaxM], s_e2[kMaxM], s_lam[kMaxM];
    __shared__ S s_tau[kMaxM], s_v0[kMaxM], s_v1[kMaxM], s_p[kMaxM];
    __shared__ double s_sig[kMaxM];
    __shared__ int s_perm[kMaxM], s_sel[kRMax], s_tw[kRMax];
    __shared__ double s_zsc[kRMax];
    __shared__ double s_scale;

    // storage: A (n x ld) in LDS for small windows, else in the workspace;
    // the multipliers of the twisted factorizations (2 n nv doubles) in LDS,
    // later the eigenvectors during the back-transformation; Z (n x nv) and
    // the tail's scratch after A in the workspace
    S* A = LDS ? reinterpret_cast<S*>(dyn) : reinterpret_cast<S*>(a.work);
    double* LU = LDS ? dyn + (size_t)n * ld * (sizeof(S) / sizeof(double)) : dyn;
    S* Z = reinterpret_cast<S*>(a.work) + (size_t)n * ld;
    S* spare1 = Z + (size_t)n * ld;
    S* spare2 = spare1 + (size_t)n * ld;

    for (int idx = tid; idx < n * n; idx += NT) {
        const int i = idx % n, j = idx / n;
        A[i + (size_t)j * ld] = gram_at<S>(a.G, slot_of(oldest, i, slots), slot_of(oldest, j, slots), slots);
    }
    __syncthreads();

    // ---- 1. Householder tridiagonalization: T = Q^* xtx Q, Q = H_0 ... H_{n-2},
    // H_j = I - tau_j v_j v_j^*, v_j = (1, A[j+2.., j]) acting on rows j+1..
    // Per column: p = tau A22 v, then A22 -= v w^* + w v^* with w = p + c v,
    // c = -tau (p^* v) / 2.  Wavefront 0 updates the next column first and
    // builds its reflector while the others update the rest (two barriers
    // per column).  Row j+1 of A22 is never used again and is not updated.
    if (wv == 0) householder_col<S>(A, ld, n, 0, s_v0, s_tau, s_e, s_d);
    __syncthreads();
    for (int j = 0; j + 1 < n; ++j) {
        const int L = n - j - 1;
        const S* v = (j & 1) ? s_v1 : s_v0;
        S* vnext = (j & 1) ? s_v0 : s_v1;
        const S tau = s_tau[j];
        S* A22 = A + (size_t)(j + 1) * ld + (j + 1);
        {
            int G = 64;
            while (G > 1 && G * L > NT) G >>= 1;
            const int gi = tid / G, gl = tid % G;
            for (int i = gi; i < L; i += NT / G) {
                const S* ci = A22 + (size_t)i * ld;
                S acc = ordered_dot<kAhead<S, LDS>>(SC::zero(), gl, G, L, [&](int k) { return SC::cj(ci[k]); },
                                       [&](int k) { return v[k]; });
                acc = group_sum(acc, G);
                if (gl == 0) s_p[i] = mulr(tau, acc);
            }
        }
        __syncthreads();
        S pv = SC::zero();
        for (int k = lane; k < L; k += 64) pv = pv + mulr(SC::cj(s_p[k]), v[k]);
        pv = group_sum(pv, 64);
        const S c = mulr(tau, pv) * (-0.5);
        if (wv == 0) {
            const S v0 = v[0], w0 = s_p[0] + mulr(c, v0);
            for (int k = lane; k < L; k += 64) {
                const S vk = v[k], wk = s_p[k] + mulr(c, vk);
                A22[k] = A22[k] - (mulr(vk, SC::cj(w0)) + mulr(wk, SC::cj(v0)));
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (j + 2 < n) householder_col<S>(A, ld, n, j + 1, vnext, s_tau, s_e, s_d);
        } else {
            // every element is read before the chunk's writes (no two
            // iterations touch the same element), so that the reads of a
            // chunk overlap instead of waiting behind the previous write
            const int L1 = L - 1, NW = NT - 64;
            auto upd = [&](int idx, S a) {
                const int k = 1 + idx % L1, i = 1 + idx / L1;
                const S vk = v[k], vi = v[i];
                const S wk = s_p[k] + mulr(c, vk), wi = s_p[i] + mulr(c, vi);
                return a - (mulr(vk, SC::cj(wi)) + mulr(wk, SC::cj(vi)));
            };
            auto at = [&](int idx) -> S& { return A22[(1 + idx % L1) + (size_t)(1 + idx / L1) * ld]; };
            constexpr int U = LDS ? 1 : 4;
            int idx = tid - 64;
            if constexpr (U > 1) {
                for (; idx + (U - 1) * NW < L1 * L1; idx += U * NW) {
                    S x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = at(idx + u * NW);
#pragma unroll
                    for (int u = 0; u < U; ++u) at(idx + u * NW) = upd(idx + u * NW, x[u]);
                }
            }
            for (; idx < L1 * L1; idx += NW) at(idx) = upd(idx, at(idx));
        }
        __syncthreads();
    }
    if (tid == 0) {
        s_d[n - 1] = SC::re(A[(n - 1) + (size_t)(n - 1) * ld]);
        s_e[n - 1] = 0.0;
        double g = 0.0;
        for (int i = 0; i < n; ++i) {
            const double r = fabs(s_d[i]) + (i > 0 ? fabs(s_e[i - 1]) : 0.0) + fabs(s_e[i]);
            g = r > g ? r : g;
        }
        s_scale = g;
    }
    __syncthreads();
    const double scale = s_scale;
    const double inv = scale > 0.0 ? 1.0 / scale : 0.0;
    for (int i = tid; i < n; i += NT) {
        s_d[i] *= inv;
        s_e[i] *= inv;
        s_e2[i] = s_e[i] * s_e[i];
    }
    __syncthreads();

    // ---- 2. eigenvalues: G lanes per eigenvalue, bracket [-1, 1] split into
    // G+1 parts per iteration until its width is at most eps (absolute,
    // ||T|| <= 1).  The Sturm counts are FP64 work on one CU, so about 256
    // lanes (G = 256 / m) finish first: more lanes per eigenvalue save
    // iterations but cost more in total than they save.
    {
        int np2 = 1;
        while (np2 < n) np2 <<= 1;
        int G = 256 / np2;
        G = G > 64 ? 64 : (G < 1 ? 1 : G);
        const int gi = tid / G, gl = tid % G;
        const int gshift = (tid & 63) / G * G;  // first lane of the group inside the wavefront
        int iters = 1;
        {
            double w = 2.0;
            while (w > kEps) {
                w /= (double)(G + 1);
                ++iters;
            }
        }
        double lo = -1.0 - 4.0 * kEps, hi = 1.0 + 4.0 * kEps;
        if (64 * wv < G * n)  // wavefronts with no eigenvalue skip the search
        for (int it = 0; it < iters; ++it) {
            const double x = lo + (hi - lo) * (double)(gl + 1) / (double)(G + 1);
            const bool above = gi < n ? sturm_count(s_d, s_e2, n, x) > gi : true;
            const uint64_t mask = __ballot(above);
            const uint64_t grp = (G == 64) ? mask : ((mask >> gshift) & ((1ull << G) - 1));
            if (grp == 0) {
                lo = lo + (hi - lo) * (double)G / (double)(G + 1);
            } else {
                const int f = __builtin_ctzll(grp);  // first point above the eigenvalue
                const double nlo = f == 0 ? lo : lo + (hi - lo) * (double)f / (double)(G + 1);
                hi = lo + (hi - lo) * (double)(f + 1) / (double)(G + 1);
                lo = nlo;
            }
        }
        if (gi < n && gl == 0) s_lam[gi] = 0.5 * (lo + hi);
    }
    __syncthreads();

    // order by |lambda| descending (ties: larger lambda first); sigma = sqrt(|lambda|)
    for (int i = tid; i < n; i += NT) {
        const double li = s_lam[i], ai = fabs(li);
        int rank = 0;
        for (int j2 = 0; j2 < n; ++j2) {
            const double aj = fabs(s_lam[j2]);
            rank += (aj > ai) || (aj == ai && j2 > i);
        }
        s_perm[rank] = i;
        s_sig[rank] = sqrt(ai * scale);
        if (rank < nv) s_sel[rank] = i;
    }
    __syncthreads();

    // ---- 3. eigenvectors of T by twisted factorizations.  The forward
    // L D L^T (wavefront 0, lane v) and backward U D U^T (wavefront 1, lane v)
    // factorizations of T - lambda_v I run side by side; the twist index
    // (argmin |gamma_k|, lowest k on ties) is a wavefront reduction; the two
    // one-term recurrences from the twist run side by side again; the norm is
    // summed in the order of a single serial pass (up, then down), so the
    // vectors do not depend on how the work is split.
    double* Lm = LU;                   // Lm[i * nv + v], i < n-1
    double* Um = LU + (size_t)n * nv;  // Um[i * nv + v], 1 <= i < n
    const double tiny = 0x1p-900;
    if (tid < nv) {
        const int v = tid;
        const double lam = s_lam[s_sel[v]];
        double Dp = s_d[0] - lam;
        for (int i = 0; i + 1 < n; ++i) {
            if (Dp == 0.0) Dp = tiny;
            const double l = s_e[i] * rcp_fast(Dp);
            Lm[(size_t)i * nv + v] = l;
            Dp = s_d[i + 1] - lam - l * s_e[i];
        }
    } else if (tid >= 64 && tid < 64 + nv) {
        const int v = tid - 64;
        const double lam = s_lam[s_sel[v]];
        double Dm = s_d[n - 1] - lam;
        for (int i = n - 1; i >= 1; --i) {
            if (Dm == 0.0) Dm = tiny;
            const double u = s_e[i - 1] * rcp_fast(Dm);
            Um[(size_t)i * nv + v] = u;
            Dm = s_d[i - 1] - lam - u * s_e[i - 1];
        }
    }
    __syncthreads();
    // twist index: argmin |gamma_k|, gamma_k = (d_k - lam) - L_{k-1} e_{k-1} - U_{k+1} e_k
    for (int v = wv; v < nv; v += NT / 64) {
        const double lam = s_lam[s_sel[v]];
        double best = 1e308;
        int tw = 0;
        for (int k = lane; k < n; k += 64) {
            double g = s_d[k] - lam;
            if (k > 0) g -= Lm[(size_t)(k - 1) * nv + v] * s_e[k - 1];
            if (k + 1 < n) g -= Um[(size_t)(k + 1) * nv + v] * s_e[k];
            if (fabs(g) < best) {
                best = fabs(g);
                tw = k;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int ot = __shfl_xor(tw, off, 64);
            if (ob < best || (ob == best && ot < tw)) {
                best = ob;
                tw = ot;
            }
        }
        if (lane == 0) s_tw[v] = tw;
    }
    __syncthreads();
    // z_tw = 1, z_i = -L_i z_{i+1} (i < tw; wavefront 0), z_{i+1} = -U_{i+1} z_i (i >= tw; wavefront 1)
    if (tid < nv) {
        const int v = tid, tw = s_tw[v];
        S* zc = Z + (size_t)v * ld;
        double z = 1.0;
        zc[tw] = SC::one();
        for (int i = tw - 1; i >= 0; --i) {
            z = -Lm[(size_t)i * nv + v] * z;
            zc[i] = SC::fromc(mkc(z));
        }
    } else if (tid >= 64 && tid < 64 + nv) {
        const int v = tid - 64, tw = s_tw[v];
        S* zc = Z + (size_t)v * ld;
        double z = 1.0;
        for (int i = tw; i + 1 < n; ++i) {
            z = -Um[(size_t)(i + 1) * nv + v] * z;
            zc[i + 1] = SC::fromc(mkc(z));
        }
    }
    __syncthreads();
    if (tid < nv) {
        const int v = tid, tw = s_tw[v];
        const S* zc = Z + (size_t)v * ld;
        double nrm2 = 1.0;
        for (int i = tw - 1; i >= 0; --i) {
            const double z = SC::re(zc[i]);
            nrm2 += z * z;
        }
        for (int i = tw; i + 1 < n; ++i) {
            const double z = SC::re(zc[i + 1]);
            nrm2 += z * z;
        }
        s_zsc[v] = rsqrt_acc(nrm2);
    }
    __syncthreads();
    for (int idx = tid; idx < n * nv; idx += NT) {
        const int i = idx % n, v = idx / n;
        S* zc = Z + (size_t)v * ld;
        zc[i] = zc[i] * s_zsc[v];
    }
    __syncthreads();
    // the eigenvectors move into LDS (over the multipliers) for the rest of the work
    S* Zs = reinterpret_cast<S*>(LU);  // Zs[i + v n]
    for (int idx = tid; idx < n * nv; idx += NT) {
        const int i = idx % n, v = idx / n;
        Zs[i + (size_t)v * n] = Z[i + (size_t)v * ld];
    }
    __syncthreads();
    // nearly coincident eigenvalues: Gram-Schmidt in selection order (one wavefront)
    if (wv == 0) {
        for (int q = 1; q < nv; ++q) {
            for (int p = 0; p < q; ++p) {
                if (fabs(s_lam[s_sel[q]] - s_lam[s_sel[p]]) > 1e-8) continue;
                S* zq = Zs + (size_t)q * n;
                const S* zp = Zs + (size_t)p * n;
                double dot = 0.0;
                for (int i = lane; i < n; i += 64) dot += SC::re(zp[i]) * SC::re(zq[i]);
                dot = wave_sum(dot);
                double nn = 0.0;
                for (int i = lane; i < n; i += 64) {
                    const double zi = SC::re(zq[i]) - dot * SC::re(zp[i]);
                    zq[i] = SC::fromc(mkc(zi));
                    nn += zi * zi;
                }
                nn = wave_sum(nn);
                const double sc = nn > 0.0 ? rsqrt_acc(nn) : 0.0;
                for (int i = lane; i < n; i += 64) zq[i] = zq[i] * sc;
            }
        }
    }
    __syncthreads();

    // ---- 4. back-transformation Z <- H_0 ... H_{n-2} Z, one half-wavefront per
    // vector (columns are independent: no barrier between reflectors)
    {
        const int hw = tid >> 5, hl = tid & 31;
        for (int v = hw; v < nv; v += NT / 32) {
            S* zc = Zs + (size_t)v * n;
            for (int j = n - 2; j >= 0; --j) {
                const S tau = s_tau[j];
                const int L = n - j - 1;
                const S* vj = A + (size_t)j * ld + (j + 1);  // v_0 = 1 is implicit
                S w = SC::zero();
                for (int i = hl; i < L; i += 32) {
                    const S vi = i == 0 ? SC::one() : vj[i];
                    w = w + mulr(SC::cj(vi), zc[j + 1 + i]);
                }
                for (int off = 16; off >= 1; off >>= 1) w = w + shfl_xor_s<S>(w, off, 32);
                const S f = mulr(tau, w);
                for (int i = hl; i < L; i += 32) {
                    const S vi = i == 0 ? SC::one() : vj[i];
                    zc[j + 1 + i] = zc[j + 1 + i] - mulr(vi, f);
                }
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < n * nv; idx += NT) {
        const int i = idx % n, v = idx / n;
        Z[i + (size_t)v * ld] = Zs[i + (size_t)v * n];
    }
    // eigenvector index k of the tail = selection rank k (columns of Z)
    for (int i = tid; i < n; i += NT) s_perm[i] = i;
    __syncthreads();
    sym_tail<S, NT, kAhead<S, LDS>>(a, ld, Z, spare1, spare2, s_sig, s_perm, nv, 0, true, 0);
}

template <typename S, int NT, bool LDS>
__global__ __launch_bounds__(NT)
void k_solve_trid(SolveArgs a) {
    solve_trid_body<S, NT, LDS>(a);
}

// A dense push's Gram finalize (1024 threads, as its own kernel) followed by
// the tridiagonal solve of the window it completes, in one launch: one
// kernel boundary fewer on the single-push step.  A rejected snapshot leaves
// the state as it was, and the solve then finds nothing new (skipped), as
// after the two separate launches.
template <bool LDS>
__global__ __launch_bounds__(1024)
void k_finalize_solve_trid(double* G, const double* partials, int nblk, SolveArgs a) {
    gram_finalize_body(G, partials, nblk, a.m, a.slots, a.st);
    __syncthreads();
    solve_trid_body<double, 1024, LDS>(a);
}

template <typename S, int NT, bool LDS>
__global__ __launch_bounds__(NT)
void k_solve_trid_grouped(const SolveArgs* __restrict__ items) {
    const SolveArgs a = items[blockIdx.x];
    solve_trid_body<S, NT, LDS>(a);
}

}  // namespace

hipError_t launch_solve_sym(const SolveArgs& a, hipStream_t s) {
    if (a.r > kRMax || a.m > kMaxM) return hipErrorInvalidValue;
    const int M = a.m + (a.m & 1);
    if (!a.cplx && M <= 64) {
        const size_t lds = 3 * sizeof(double) * (size_t)M * (M + 1);
        auto kern = k_solve_sym<double, 1024, true, 32>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(1), dim3(1024), lds, s, a, M);
    } else if (!a.cplx) {
        hipLaunchKernelGGL((k_solve_sym<double, 1024, false, kMaxM / 2>), dim3(1), dim3(1024), 0, s, a, M);
    } else {
        hipLaunchKernelGGL((k_solve_sym<cplx, 1024, false, kMaxM / 2>), dim3(1), dim3(1024), 0, s, a, M);
    }
    return hipGetLastError();
}

template <typename S, bool LDS>
static hipError_t launch_trid_one(const SolveArgs& a, hipStream_t s) {
    const int n = a.m, nv = a.r < n ? a.r : n;
    size_t lds = sizeof(double) * 2 * (size_t)n * nv;
    if (LDS) lds += sizeof(S) * (size_t)n * (n + 1);
    auto kern = k_solve_trid<S, 1024, LDS>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(1024), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_solve_trid(const SolveArgs& a, hipStream_t s) {
    if (a.r > kRMax || a.m > kMaxM) return hipErrorInvalidValue;
    if (a.cplx) return a.m <= 32 ? launch_trid_one<cplx, true>(a, s) : launch_trid_one<cplx, false>(a, s);
    return a.m <= 64 ? launch_trid_one<double, true>(a, s) : launch_trid_one<double, false>(a, s);
}

hipError_t launch_finalize_solve_trid(double* G, const double* partials, int nblk, const SolveArgs& a,
                                      hipStream_t s) {
    if (a.r > kRMax || a.m > kMaxM || a.cplx) return hipErrorInvalidValue;
    const int n = a.m, nv = a.r < n ? a.r : n;
    const bool lds_form = a.m <= 64;
    size_t lds = sizeof(double) * 2 * (size_t)n * nv;
    if (lds_form) lds += sizeof(double) * (size_t)n * (n + 1);
    const void* kern = lds_form ? reinterpret_cast<const void*>(k_finalize_solve_trid<true>)
                                : reinterpret_cast<const void*>(k_finalize_solve_trid<false>);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (lds_form) hipLaunchKernelGGL(k_finalize_solve_trid<true>, dim3(1), dim3(1024), lds, s, G, partials, nblk, a);
    else hipLaunchKernelGGL(k_finalize_solve_trid<false>, dim3(1), dim3(1024), lds, s, G, partials, nblk, a);
    return hipGetLastError();
}

hipError_t launch_solve_eig(const SolveArgs& a, hipStream_t s) {
    if (a.r > kRMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_solve_eig, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace dmd

namespace dmd {

hipError_t launch_trid_grouped(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                               hipStream_t s) {
    // real windows; items_lds: m <= 64, items_glb: m > 64 (dynamic LDS sized for the largest)
    if (n_lds > 0) {
        const size_t lds = sizeof(double) * (2 * 64 * kRMax + 64 * 65);
        auto kern = k_solve_trid_grouped<double, 1024, true>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(n_lds), dim3(1024), lds, s, items_lds);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_glb > 0) {
        const size_t lds = sizeof(double) * 2 * kMaxM * kRMax;
        auto kern = k_solve_trid_grouped<double, 1024, false>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(n_glb), dim3(1024), lds, s, items_glb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_trid_grouped_cplx(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                                    hipStream_t s) {
    // Hermitian windows (sparse streams); items_lds: m <= 32, items_glb: m > 32
    if (n_lds > 0) {
        const size_t lds = sizeof(double) * 2 * 32 * kRMax + sizeof(cplx) * 32 * 33;
        auto kern = k_solve_trid_grouped<cplx, 1024, true>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(n_lds), dim3(1024), lds, s, items_lds);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_glb > 0) {
        const size_t lds = sizeof(double) * 2 * kMaxM * kRMax;
        auto kern = k_solve_trid_grouped<cplx, 1024, false>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(n_glb), dim3(1024), lds, s, items_glb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_eig_grouped(const SolveArgs* items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve_eig_grouped, dim3(n), dim3(64), 0, s, items);
    return hipGetLastError();
}

hipError_t launch_jacobi_grouped(const SolveArgs* items_lds, int n_lds, const SolveArgs* items_glb, int n_glb,
                                 hipStream_t s) {
    if (n_lds > 0) {
        const size_t lds = 3 * sizeof(double) * 64 * 65;  // sized for M <= 64
        auto kern = k_solve_sym_grouped<double, 1024, true, 32>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(n_lds), dim3(1024), lds, s, items_lds);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_glb > 0) {
        hipLaunchKernelGGL((k_solve_sym_grouped<double, 1024, false, kMaxM / 2>), dim3(n_glb), dim3(1024), 0, s,
                           items_glb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


}  // namespace dmd
