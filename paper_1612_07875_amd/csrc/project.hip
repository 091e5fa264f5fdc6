// Tall-skinny projections of the window: DMD modes Phi = X' (V Sigma^-1 W)
// (Eq. Phi) and POD modes U = X (V Sigma^-1) (Sec. 2.1, step 2).
//
// out (n x kcols) = X_sub (n x m, ring columns in window order) * B (m x kcols),
// B row-major.  For the modes B holds the complex m x r_eff matrix
// C = V Sigma^-1 W as 2 r_eff interleaved real columns, so a real window gives
// interleaved complex output directly.  Each thread owns one row; the
// coefficient block sits in LDS and is read as a broadcast.
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;

// TX: ring element type; T: coefficient, accumulation and output type.
template <typename TX, typename T, int KC>
__global__ __launch_bounds__(kThreads)
void k_project_rows(ProjectArgs a) {
    extern __shared__ char dyn_lds[];
    T* Bs = reinterpret_cast<T*>(dyn_lds);  // m x KC coefficient block
    const DevState* st = a.st;
    if (st->solve_status == ST_E_NOT_READY) return;
    const int k_eff = st->r_eff;
    const int kcols = a.cplx_out ? 2 * k_eff : k_eff;
    const int col0 = blockIdx.y * KC;
    if (col0 >= kcols) return;
    const int m = a.m;
    const int rowstride = a.cplx_out ? 2 * a.kmax : a.kmax;
    const T* B = reinterpret_cast<const T*>(a.B);
    for (int idx = threadIdx.x; idx < m * KC; idx += kThreads) {
        const int j = idx / KC, c = idx % KC;
        Bs[idx] = (col0 + c < kcols) ? B[(int64_t)j * rowstride + col0 + c] : T(0);
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.n) return;
    const int oldest = st->oldest;
    const TX* ring = reinterpret_cast<const TX*>(a.ring);
    T acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = T(0);
    int j = 0;
    for (; j + 4 <= m; j += 4) {
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            x[u] = (T)ring[(int64_t)slot_of(oldest, a.first + j + u, a.slots) * a.ld + i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(x[u], Bs[(j + u) * KC + c], acc[c]);
    }
    for (; j < m; ++j) {
        const T x = (T)ring[(int64_t)slot_of(oldest, a.first + j, a.slots) * a.ld + i];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = fma(x, Bs[j * KC + c], acc[c]);
    }
    T* out = reinterpret_cast<T*>(a.out);
    if (a.cplx_out) {
#pragma unroll
        for (int c = 0; c < KC; c += 2) {
            if (col0 + c < kcols) {
                const int64_t o = 2 * (i + (int64_t)((col0 + c) / 2) * a.ldo);
                out[o] = acc[c];
                out[o + 1] = acc[c + 1];
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (col0 + c < kcols) out[i + (int64_t)(col0 + c) * a.ldo] = acc[c];
    }
}

template <typename TX, typename T, int KC>
hipError_t launch_kc(const ProjectArgs& a, hipStream_t s, int kc_max) {
    const unsigned gx = (unsigned)((a.n + kThreads - 1) / kThreads);
    dim3 grid(gx, (kc_max + KC - 1) / KC);
    const size_t lds = sizeof(T) * (size_t)a.m * KC;
    auto kern = k_project_rows<TX, T, KC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

// One pass over the window: the column block covers all output columns.
template <typename TX, typename T>
hipError_t launch_rows(const ProjectArgs& a, hipStream_t s, int kc_max) {
    if (kc_max <= 8) return launch_kc<TX, T, 8>(a, s, kc_max);
    if (kc_max <= 16) return launch_kc<TX, T, 16>(a, s, kc_max);
    if (kc_max <= 24) return launch_kc<TX, T, 24>(a, s, kc_max);
    if (kc_max <= 32) return launch_kc<TX, T, 32>(a, s, kc_max);
    if (kc_max <= 40) return launch_kc<TX, T, 40>(a, s, kc_max);
    if (kc_max <= 48) return launch_kc<TX, T, 48>(a, s, kc_max);
    return launch_kc<TX, T, 64>(a, s, kc_max);
}

}  // namespace

hipError_t launch_project(const ProjectArgs& a, hipStream_t s) {
    const int kc_max = a.cplx_out ? 2 * a.kmax : a.kmax;
    if (a.elem_f64) return launch_rows<double, double>(a, s, kc_max);
    if (a.coef_f64) return launch_rows<float, double>(a, s, kc_max);
    return launch_rows<float, float>(a, s, kc_max);
}

}  // namespace dmd
