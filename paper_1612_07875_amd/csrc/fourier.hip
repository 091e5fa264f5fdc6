// Spatial -> Fourier ingest of the sparse path (Sec. 3.5).
//
// SVD and DMD do not change under a unitary change of basis of the
// snapshots, so a dense H x W frame may enter the sparse (CSR) path as its
// unitary 2-D DFT restricted to a fixed support S (the lowest wavenumbers):
//   xhat[ky, kx] = (H W)^-1/2 sum_y e^{-2 pi i ky y / H} sum_x x[y, x] e^{-2 pi i kx x / W}.
// Only |S| coefficients are needed, so instead of a full FFT the transform
// is evaluated separably for exactly those: first, for every row y and every
// distinct kx bin of S, R[y, j] = sum_x x[y, x] w_W^(kx_j x) (one pass over
// the frame); then, per kept coefficient c = (ky, kx_j), xhat_c =
// (H W)^-1/2 sum_y R[y, j] w_H^(ky y).  Phases come from tables of the N-th
// roots of unity indexed by the exact integer (k * t) mod N, and sums are in
// FP64 on FP32 data: the coefficients are exact to FP64 rounding before
// they are stored as complex64.
#include "dmd_internal.h"

namespace dmd {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double2 dsum_wave(double2 v) {
    for (int off = 32; off >= 1; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    return v;
}

// One workgroup per row: the row is staged in LDS; wavefront w takes the kx
// bins w, w+4, ...; lanes split the row and a butterfly sums them.
__global__ __launch_bounds__(kThreads)
void k_dft_rows(FourierArgs a) {
    extern __shared__ float row[];
    const int y = blockIdx.x;
    const float* src = a.frame + (int64_t)y * a.ld_row;
    for (int x = threadIdx.x; x < a.W; x += kThreads) row[x] = src[x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < a.nkx; j += kThreads / 64) {
        const int kx = a.kx[j];
        double2 acc{0.0, 0.0};
        for (int x = lane; x < a.W; x += 64) {
            const double2 w = a.twW[(int)(((int64_t)kx * x) % a.W)];
            const double v = row[x];
            acc.x = fma(v, w.x, acc.x);
            acc.y = fma(v, w.y, acc.y);
        }
        acc = dsum_wave(acc);
        if (lane == 0) a.R[(int64_t)y * a.nkx + j] = acc;
    }
}

// One wavefront per kept coefficient: lanes split the rows.
__global__ __launch_bounds__(kThreads)
void k_dft_cols(FourierArgs a) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (c >= a.nkeep) return;
    const int ky = a.ky[c], j = a.col[c];
    double2 acc{0.0, 0.0};
    for (int y = lane; y < a.H; y += 64) {
        const double2 r = a.R[(int64_t)y * a.nkx + j];
        const double2 w = a.twH[(int)(((int64_t)ky * y) % a.H)];
        acc.x += r.x * w.x - r.y * w.y;
        acc.y += r.x * w.y + r.y * w.x;
    }
    acc = dsum_wave(acc);
    if (lane == 0) a.val[c] = float2{(float)(acc.x * a.scale), (float)(acc.y * a.scale)};
}

}  // namespace

hipError_t launch_fourier(const FourierArgs& a, hipStream_t s) {
    if (a.H < 1 || a.W < 1 || a.W > kFourierMaxW || a.nkx < 1 || a.nkeep < 1 || a.ld_row < a.W)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dft_rows, dim3((unsigned)a.H), dim3(kThreads), sizeof(float) * (size_t)a.W, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned g = (unsigned)((a.nkeep + kThreads / 64 - 1) / (kThreads / 64));
    hipLaunchKernelGGL(k_dft_cols, dim3(g), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace dmd
