// Streaming background subtraction of the newest snapshot (Sec. 3.3,
// Algorithm 3).
//
// The eig solve leaves beta = b_i lambda_i^m C[:, i] (m complex values) for
// the background mode i, so the background of the newest snapshot is
// l = b_i lambda_i^m phi_i = X' beta and the foreground s = x_new - |l|, x_new
// being the last column of X'.  One pass reads the m columns of X' (16-byte
// loads, four consecutive rows per thread for FP32 data, two for FP64) and
// writes |l| and s: m n bytes-per-element in, up to 2 n out, bound by HBM.
// Accumulation and outputs use the projection precision (FP32 for FP32
// projections, else FP64); sums run over the columns in index order.  Loads
// and stores are nontemporal: each value is touched once per call, and the
// window is far larger than the caches (103 -> 100 us for a 1080p FP32
// window of 64 columns, 0.68 of the HBM peak).
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;

// 16-byte vectors of the ring's element type (clang vectors: the
// nontemporal builtins take them)
template <typename TX> struct V16;
template <> struct V16<float>  { typedef float type __attribute__((ext_vector_type(4))); static constexpr int N = 4; };
template <> struct V16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int N = 2; };

// TX: ring element type; T: coefficient, accumulation and output type.
template <typename TX, typename T>
__global__ __launch_bounds__(kThreads)
void k_background(BackgroundArgs a) {
    using VT = typename V16<TX>::type;
    constexpr int N = V16<TX>::N;
    __shared__ T s_beta[2 * kMaxM];
    const DevState* st = a.st;
    const int m = window_cols(a.m, a.buildup, st);  // columns of X' (fewer during a build-up start)
    if (m == 0 || (st->solve_status != ST_OK && st->solve_status != ST_W_RANK) || st->r_eff == 0)
        return;
    const T* beta = static_cast<const T*>(a.beta);
    for (int i = threadIdx.x; i < 2 * m; i += kThreads) s_beta[i] = beta[i];
    __syncthreads();

    const int64_t r0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * N;
    if (r0 >= a.n) return;
    const TX* ring = static_cast<const TX*>(a.ring);
    const int oldest = st->oldest;
    T re[N], im[N], xn[N];
#pragma unroll
    for (int e = 0; e < N; ++e) re[e] = im[e] = xn[e] = T(0);
    // rows r0 .. r0+N-1 lie inside the padded column (ld is a multiple of 64)
#pragma unroll 4
    for (int j = 0; j < m; ++j) {
        const VT v = __builtin_nontemporal_load(
            reinterpret_cast<const VT*>(ring + (int64_t)slot_of(oldest, 1 + j, a.slots) * a.ld + r0));
        TX pv[N];
#pragma unroll
        for (int e = 0; e < N; ++e) pv[e] = v[e];
        const T br = s_beta[2 * j], bi = s_beta[2 * j + 1];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const T x = (T)pv[e];
            re[e] = fma(x, br, re[e]);
            im[e] = fma(x, bi, im[e]);
            xn[e] = x;  // after the loop: the last column of X', the newest snapshot
        }
    }
    T* fg = static_cast<T*>(a.fg);
    T* bg = static_cast<T*>(a.bg);
#pragma unroll
    for (int e = 0; e < N; ++e) {
        if (r0 + e >= a.n) break;
        const T l = sqrt(re[e] * re[e] + im[e] * im[e]);
        if (fg) __builtin_nontemporal_store(xn[e] - l, &fg[r0 + e]);
        if (bg) __builtin_nontemporal_store(l, &bg[r0 + e]);
    }
}

}  // namespace

hipError_t launch_background(const BackgroundArgs& a, hipStream_t s) {
    if (a.m > kMaxM || a.ld % 64 || (a.elem_f64 && !a.coef_f64)) return hipErrorInvalidValue;
    const int N = a.elem_f64 ? 2 : 4;
    const int64_t per = (int64_t)kThreads * N;
    const unsigned gx = (unsigned)((a.n + per - 1) / per);
    if (a.elem_f64) hipLaunchKernelGGL((k_background<double, double>), dim3(gx), dim3(kThreads), 0, s, a);
    else if (a.coef_f64) hipLaunchKernelGGL((k_background<float, double>), dim3(gx), dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_background<float, float>), dim3(gx), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace dmd
