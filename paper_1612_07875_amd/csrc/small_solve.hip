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
//   * DMD coefficients C = V Sigma^-1 W for the projection Phi = X' C (Eq. Phi).
#include <cfloat>

#include "cplx.h"
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kRMax = 32;         // largest truncation rank handled by k_solve_eig
constexpr double kEps = DBL_EPSILON;

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
template <typename S, int NT>
__global__ __launch_bounds__(NT)
void k_solve_sym(SolveArgs a, int M, int use_lds) {
    using SC = Scal<S>;
    extern __shared__ double dyn[];
    const int tid = threadIdx.x;
    const int m = a.m;
    const int slots = a.slots;
    DevState* st = a.st;

    const int count = st->count;
    if (count < m + 1) {
        if (tid == 0) {
            st->solve_status = ST_E_NOT_READY;
            st->r_eff = 0;
        }
        return;
    }
    const int oldest = st->oldest;

    S* A;
    S* V;
    if (use_lds) {
        A = reinterpret_cast<S*>(dyn);
        V = A + (size_t)M * M;
    } else {
        A = reinterpret_cast<S*>(a.work);
        V = A + (size_t)M * M;
    }
    const int P = M / 2;

    __shared__ double s_c[kMaxM / 2], s_s[kMaxM / 2], s_t[kMaxM / 2];
    __shared__ S s_e[kMaxM / 2];
    __shared__ int s_p[kMaxM / 2], s_q[kMaxM / 2];
    __shared__ int s_rot;
    __shared__ double s_red[NT / 64];
    __shared__ double s_sig[kMaxM];
    __shared__ int s_perm[kMaxM];
    __shared__ int s_reff;

    // gather xtx (logical window columns 0 .. m-1); pad to even M with a decoupled zero
    for (int idx = tid; idx < M * M; idx += NT) {
        const int i = idx % M, j = idx / M;
        S v = SC::zero();
        if (i < m && j < m) v = gram_at<S>(a.G, slot_of(oldest, i, slots), slot_of(oldest, j, slots), slots);
        A[idx] = v;
        V[idx] = (i == j) ? SC::one() : SC::zero();
    }
    __syncthreads();

    // rotation floor: entries below 1e-18 * trace cannot move any eigenvalue
    // that a Gram accumulated in FP64 resolves
    double tr = 0.0;
    for (int i = tid; i < m; i += NT) tr += fabs(SC::re(A[i + i * M]));
    for (int off = 32; off >= 1; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = tr;
    __syncthreads();
    tr = 0.0;
    for (int w = 0; w < NT / 64; ++w) tr += s_red[w];
    const double floor_abs = 1e-18 * tr;
    const double tol = a.tol;

    int sweep = 0;
    bool converged = false;
    for (; sweep < a.max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int rd = 0; rd < M - 1; ++rd) {
            if (tid < P) {
                int p, q;
                rr_pair(rd, tid, M, p, q);
                const S apq = A[p + q * M];
                const double app = SC::re(A[p + p * M]);
                const double aqq = SC::re(A[q + q * M]);
                const double g = SC::absv(apq);
                double c = 1.0, s = 0.0, t = 0.0;
                S e = SC::one();
                if (g > floor_abs && g > tol * sqrt(fabs(app * aqq))) {
                    const double theta = (aqq - app) / (2.0 * g);
                    if (fabs(theta) > 1e100) {
                        t = 0.5 / theta;
                    } else {
                        t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                    }
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    e = SC::phase(apq);
                    s_rot = 1;
                }
                s_c[tid] = c;
                s_s[tid] = s;
                s_t[tid] = t * g;
                s_e[tid] = e;
                s_p[tid] = p;
                s_q[tid] = q;
            }
            __syncthreads();
            // A <- J^* A J, 2x2 blocks of (pair k rows, pair l columns), k <= l,
            // mirrored so that A stays exactly Hermitian
            for (int idx = tid; idx < P * P; idx += NT) {
                const int k = idx / P, l = idx % P;
                if (k > l) continue;
                const double sk = s_s[k], sl = s_s[l];
                if (sk == 0.0 && sl == 0.0) continue;
                const int p = s_p[k], q = s_q[k];
                if (k == l) {
                    const double dt = s_t[k];
                    A[p + p * M] = SC::fromc(SC::toc(A[p + p * M]) - mkc(dt));
                    A[q + q * M] = SC::fromc(SC::toc(A[q + q * M]) + mkc(dt));
                    A[p + q * M] = SC::zero();
                    A[q + p * M] = SC::zero();
                    continue;
                }
                const int u = s_p[l], v = s_q[l];
                const double ck = s_c[k], cl = s_c[l];
                const S ek = s_e[k], el = s_e[l];
                const S apu = A[p + u * M], apv = A[p + v * M];
                const S aqu = A[q + u * M], aqv = A[q + v * M];
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
                A[p + u * M] = npu;
                A[u + p * M] = SC::cj(npu);
                A[p + v * M] = npv;
                A[v + p * M] = SC::cj(npv);
                A[q + u * M] = nqu;
                A[u + q * M] = SC::cj(nqu);
                A[q + v * M] = nqv;
                A[v + q * M] = SC::cj(nqv);
            }
            // V <- V J
            for (int idx = tid; idx < M * P; idx += NT) {
                const int i = idx % M, k = idx / M;
                const double sk = s_s[k];
                if (sk == 0.0) continue;
                const int p = s_p[k], q = s_q[k];
                const double ck = s_c[k];
                const S ek = s_e[k];
                const S vp = V[i + p * M], vq = V[i + q * M];
                V[i + p * M] = ck * vp - sk * mulr(SC::cj(ek), vq);
                V[i + q * M] = sk * mulr(ek, vp) + ck * vq;
            }
            __syncthreads();
        }
        if (s_rot == 0) {
            converged = true;
            break;
        }
        __syncthreads();
    }

    // sigma = sqrt(|d|), sorted descending (stable in the index)
    for (int i = tid; i < m; i += NT) s_sig[i] = sqrt(fabs(SC::re(A[i + i * M])));
    __syncthreads();
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
    __syncthreads();
    const int k_eff = s_reff;

    // canonical V_r: column perm[k] of V, phase so that its largest-modulus
    // entry (lowest index on ties) is real positive.  Stored in A's space.
    S* Vr = A;  // m x k_eff, leading dimension m
    const int nw = NT / 64, lane = tid & 63, wv = tid >> 6;
    for (int k = wv; k < k_eff; k += nw) {
        const int col = s_perm[k];
        double best = -1.0;
        int bi = 0;
        for (int i = lane; i < m; i += 64) {
            const double v = SC::absv(V[i + col * M]);
            if (v > best) { best = v; bi = i; }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const S ph = SC::cj(SC::phase(V[bi + col * M]));
        // every lane has read V[bi][col] before any lane overwrites A (distinct storage)
        for (int i = lane; i < m; i += 64) {
            const S v = mulr(V[i + col * M], ph);
            Vr[i + (size_t)k * m] = v;
            store_s<S>(a.V, i + (int64_t)k * m, v);
        }
    }
    __syncthreads();

    // T = xty V_r (m x k_eff) with xty[i][j] = <x_i, x_{j+1}>; stored in V's space
    S* T = V;
    for (int idx = tid; idx < m * k_eff; idx += NT) {
        const int i = idx % m, b = idx / m;
        const int si = slot_of(oldest, i, slots);
        S acc = SC::zero();
        for (int j = 0; j < m; ++j)
            acc = acc + mulr(gram_at<S>(a.G, si, slot_of(oldest, j + 1, slots), slots), Vr[j + (size_t)b * m]);
        T[i + (size_t)b * m] = acc;
    }
    __syncthreads();

    // A~[p][q] = (V_r^* T)[p][q] / (sigma_p sigma_q)
    for (int idx = tid; idx < k_eff * k_eff; idx += NT) {
        const int p = idx % k_eff, q = idx / k_eff;
        S acc = SC::zero();
        for (int i = 0; i < m; ++i) acc = acc + mulr(SC::cj(Vr[i + (size_t)p * m]), T[i + (size_t)q * m]);
        const double sp = s_sig[s_perm[p]], sq = s_sig[s_perm[q]];
        store_s<S>(a.At, p + (int64_t)q * k_eff, acc * (1.0 / (sp * sq)));
    }
    // POD coefficients V_r Sigma^-1 (row-major m x kmax, real or interleaved complex)
    const int cw = (sizeof(S) == sizeof(cplx)) ? 2 : 1;
    for (int idx = tid; idx < m * k_eff; idx += NT) {
        const int i = idx / k_eff, q = idx % k_eff;
        const S v = Vr[i + (size_t)q * m] * (1.0 / s_sig[s_perm[q]]);
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
        st->r_eff = k_eff;
        st->sweeps = sweep + (converged ? 1 : 0);
        st->solve_status = converged ? (k_eff < (a.r < m ? a.r : m) ? ST_W_RANK : ST_OK) : ST_E_CONVERGENCE;
        if (k_eff == 0) st->solve_status = ST_W_RANK;
    }
}

// --------------------------------------------------------------------------
// k_solve_eig: one wavefront, A~ (k x k, k <= 32) in LDS
// --------------------------------------------------------------------------
constexpr int LDH = kRMax;

__global__ __launch_bounds__(64)
void k_solve_eig(SolveArgs a) {
    const int lane = threadIdx.x;
    DevState* st = a.st;
    const int status0 = st->solve_status;
    const int k = st->r_eff;
    const int m = a.m;
    if (status0 == ST_E_NOT_READY || k == 0) {
        if (lane == 0 && status0 != ST_E_NOT_READY) st->solves += 1;
        publish(a);
        return;
    }

    __shared__ cplx H[LDH * LDH];
    __shared__ cplx Z[LDH * LDH];
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
    }
    if (lane < k) s_sig[lane] = a.sigma[lane];
    __syncthreads();

    // ---- Householder reduction to upper Hessenberg form, Z accumulates
    for (int c = 0; c + 2 < k; ++c) {
        const int len = k - c - 1;  // rows c+1 .. k-1
        double tail2 = 0.0;
        if (lane >= 1 && lane < len) tail2 = abs2(H[(c + 1 + lane) + c * LDH]);
        for (int off = 32; off >= 1; off >>= 1) tail2 += __shfl_xor(tail2, off, 64);
        const cplx x0 = H[(c + 1) + c * LDH];
        const double ax0 = cabs(x0);
        const double alpha = sqrt(ax0 * ax0 + tail2);
        if (tail2 == 0.0) {
            __syncthreads();
            continue;
        }
        const cplx ph = ax0 > 0.0 ? cplx{x0.re / ax0, x0.im / ax0} : mkc(1.0);
        // v = x + ph*alpha e1 ; v^* v = 2 alpha (alpha + |x0|) ; P = I - tau v v^*
        if (lane < len) hv[lane] = (lane == 0) ? x0 + ph * alpha : H[(c + 1 + lane) + c * LDH];
        __syncthreads();
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
        __syncthreads();
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
        __syncthreads();
        if (lane < len) H[(c + 1 + lane) + c * LDH] = (lane == 0) ? -(ph * alpha) : mkc(0.0);
        __syncthreads();
    }

    // ---- single-shift complex QR to Schur form (full T and Z)
    double hmax = 0.0;
    for (int idx = lane; idx < k * k; idx += 64) hmax = fmax(hmax, cabs(H[(idx % k) + (idx / k) * LDH]));
    for (int off = 32; off >= 1; off >>= 1) hmax = fmax(hmax, __shfl_xor(hmax, off, 64));
    const double smallnum = (hmax > 0.0 ? hmax : 1.0) * kEps;

    int hi = k - 1, iter = 0, total = 0;
    bool failed = false;
    const int max_iter = a.max_qr_iter;
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
        __syncthreads();
        if (l > 0 && lane == 0) H[l + (l - 1) * LDH] = mkc(0.0);
        __syncthreads();
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
        for (int kk = l; kk < hi; ++kk) {
            cplx x, y;
            if (kk == l) {
                x = H[l + l * LDH] - mu;
                y = H[(l + 1) + l * LDH];
            } else {
                x = H[kk + (kk - 1) * LDH];
                y = H[(kk + 1) + (kk - 1) * LDH];
            }
            // G = [[c, s], [-conj(s), c]] with G [x; y] = [rho; 0]
            double c;
            cplx s;
            const double ax = cabs(x), ay = cabs(y);
            if (ay == 0.0) {
                c = 1.0;
                s = mkc(0.0);
            } else if (ax == 0.0) {
                c = 0.0;
                s = mkc(1.0);
            } else {
                const double rr = hypot(ax, ay);
                c = ax / rr;
                s = (1.0 / rr) * mul_conj(cplx{x.re / ax, x.im / ax}, y);
            }
            __syncthreads();
            // rows kk, kk+1 over columns jlo .. k-1
            {
                const int jlo = kk > l ? kk - 1 : l;
                const int j = lane;
                if (j >= jlo && j < k) {
                    const cplx u = H[kk + j * LDH], v = H[(kk + 1) + j * LDH];
                    H[kk + j * LDH] = c * u + s * v;
                    H[(kk + 1) + j * LDH] = c * v - conj_mul(s, u);
                }
            }
            __syncthreads();
            if (kk > l && lane == 0) H[(kk + 1) + (kk - 1) * LDH] = mkc(0.0);
            // columns kk, kk+1 over rows 0 .. min(kk+2, hi); Z over all rows
            {
                const int i = lane;
                const int ihi = kk + 2 < hi ? kk + 2 : hi;
                if (i <= ihi) {
                    const cplx u = H[i + kk * LDH], v = H[i + (kk + 1) * LDH];
                    H[i + kk * LDH] = c * u + mul_conj(v, s);
                    H[i + (kk + 1) * LDH] = c * v - u * s;
                }
                if (i < k) {
                    const cplx u = Z[i + kk * LDH], v = Z[i + (kk + 1) * LDH];
                    Z[i + kk * LDH] = c * u + mul_conj(v, s);
                    Z[i + (kk + 1) * LDH] = c * v - u * s;
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();

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
    __syncthreads();
    // W = Z Y (lane = row), written over T
    cplx lam_q = mkc(0.0);
    if (lane < k) lam_q = H[lane + lane * LDH];
    __syncthreads();
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
    __syncthreads();
    // normalise column q (lane q): unit norm, largest-modulus entry (lowest
    // index on ties) real positive; rank by |lambda| descending, arg ascending
    __shared__ cplx s_lam[kRMax];
    if (lane < k) s_lam[lane] = lam_q;
    __syncthreads();
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
        const double mq = cabs(lam_q), aq = atan2(lam_q.im, lam_q.re);
        int rank = 0;
        for (int p = 0; p < k; ++p) {
            const cplx lp = s_lam[p];
            const double mp = cabs(lp), app = atan2(lp.im, lp.re);
            rank += (mp > mq) || (mp == mq && app < aq) || (mp == mq && app == aq && p < q);
        }
        s_rank[q] = rank;
        a.lam[2 * rank] = lam_q.re;
        a.lam[2 * rank + 1] = lam_q.im;
        for (int i = 0; i < k; ++i) {
            const cplx w = H[i + q * LDH] * scale_q;
            Y[i + rank * LDH] = w;  // sorted, canonical W
            a.W[2 * (i + (int64_t)rank * k)] = w.re;
            a.W[2 * (i + (int64_t)rank * k) + 1] = w.im;
        }
    }
    __syncthreads();

    // ---- C = V_r Sigma^-1 W (m x k complex), row-major with row stride 2 r
    for (int i = lane; i < m; i += 64) {
        for (int q = 0; q < k; ++q) {
            cplx acc = mkc(0.0);
            for (int p = 0; p < k; ++p) {
                cplx vip;
                if (a.cplx) vip = cplx{a.V[2 * (i + (int64_t)p * m)], a.V[2 * (i + (int64_t)p * m) + 1]};
                else vip = mkc(a.V[i + (int64_t)p * m]);
                acc = acc + (vip * (1.0 / s_sig[p])) * Y[p + q * LDH];
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
        }
    }
    if (lane == 0) {
        st->qr_iters = total;
        if (failed) st->solve_status = ST_E_CONVERGENCE;
        st->solves += 1;
    }
    publish(a);
}

}  // namespace

hipError_t launch_solve_sym(const SolveArgs& a, hipStream_t s) {
    if (a.r > kRMax || a.m > kMaxM) return hipErrorInvalidValue;
    const int M = a.m + (a.m & 1);
    if (!a.cplx && M <= 64) {
        const size_t lds = 2 * sizeof(double) * (size_t)M * M;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve_sym<double, 256>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_solve_sym<double, 256>), dim3(1), dim3(256), lds, s, a, M, 1);
    } else if (!a.cplx) {
        hipLaunchKernelGGL((k_solve_sym<double, 1024>), dim3(1), dim3(1024), 0, s, a, M, 0);
    } else {
        hipLaunchKernelGGL((k_solve_sym<cplx, 1024>), dim3(1), dim3(1024), 0, s, a, M, 0);
    }
    return hipGetLastError();
}

hipError_t launch_solve_eig(const SolveArgs& a, hipStream_t s) {
    if (a.r > kRMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_solve_eig, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace dmd
