// Stateless whole-window Gram, G = X^* X of k snapshot columns (Algorithm 1's
// first step; Sec. 2.1 step 1), without a stream handle: the MFMA Gram kernel
// of the bulk window load (k_gram_tiles + k_gram_reduce) run on a caller's
// column-major matrix, writing the k x k FP64 result into a caller's buffer.
//
// The row-split partial tiles of the kernel (splits x upper-triangle tiles x
// 64 x 64 FP64) are stream-ordered scratch: allocated with hipMallocAsync on
// the caller's stream and freed after the reduction with hipFreeAsync.
//
// The allocation-free variant (dmd_window_gram_noalloc) takes the partial
// tiles from a fixed device array instead, sized for the largest window the
// call accepts; its address on each device is looked up once, with that
// device current, and used for every later call there.
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "dmd_internal.h"
#include "dmd_stream.h"

#define DMD_API extern "C" __attribute__((visibility("default")))

namespace dmd {
namespace {

// Checks of the stateless Gram call; returns DMD_OK or sets the error message.
int check_window_gram(const void* X, int64_t ldx, int64_t n, int32_t ncols, int32_t dtype, int32_t precision,
                      const double* G, int64_t ldg, int* elem_bytes) {
    if (!X || !G) return api_fail(DMD_E_INVAL, "null X or G");
    if (dtype != DMD_F32 && dtype != DMD_F64) return api_fail(DMD_E_INVAL, "dtype must be DMD_F32 or DMD_F64");
    if (precision < DMD_PREC_DEFAULT || precision > DMD_PREC_FP64)
        return api_fail(DMD_E_INVAL, "unknown precision %d", precision);
    if (dtype == DMD_F64 && precision == DMD_PREC_BF16X3)
        return api_fail(DMD_E_UNSUPPORTED, "BF16X3 applies to FP32 data");
    if (n < 1) return api_fail(DMD_E_INVAL, "n must be >= 1");
    if (ncols < 1 || ncols > kMaxM + 1) return api_fail(DMD_E_INVAL, "ncols must be in [1, %d]", kMaxM + 1);
    if (ldx < n || ldg < ncols) return api_fail(DMD_E_INVAL, "ldx < n or ldg < ncols");
    const int eb = dtype == DMD_F64 ? 8 : 4;
    if ((uintptr_t)X % 16 || (ldx * eb) % 16)
        return api_fail(DMD_E_INVAL, "X and its columns must be 16-byte aligned");
    if ((uintptr_t)G % 8) return api_fail(DMD_E_INVAL, "G must be 8-byte aligned");
    *elem_bytes = eb;
    return DMD_OK;
}

}  // namespace

size_t window_gram_scratch_bytes(int32_t ncols) {
    return sizeof(double) * 64 * 64 * (size_t)gram_full_tiles(ncols - 1) * gram_full_splits(ncols - 1);
}

// Window columns are X's columns (slot l = column l, oldest 0); no stream
// state is read or written.
hipError_t launch_window_gram(const void* X, int64_t ldx, int64_t n, int32_t ncols, int elem_f64, int32_t precision,
                              double* G, int64_t ldg, double* partial, hipStream_t s) {
    return launch_gram_full(X, ldx, n, ncols - 1, (int)ldg, elem_f64, precision, ncols, 0, partial, G, nullptr, 0, s);
}

// Scratch of the allocation-free call: the partial tiles of the largest window
// (257 columns: 15 upper-triangle tiles x 35 row splits; no smaller window
// needs more), one copy per device, held until the process ends.  Every
// partial tile is written in full by each call, so nothing needs clearing.
// Host code never uses this name as an address: the device address comes
// from noalloc_scratch() below.
constexpr size_t kNoAllocTiles = 525;
constexpr size_t kNoAllocBytes = kNoAllocTiles * 64 * 64 * sizeof(double);  // 17,203,200 bytes
static __device__ __align__(256) double scratch[kNoAllocTiles * 64 * 64];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of `scratch` on the device that runs `s`; looked up once
// per device (with that device current) and kept.
int noalloc_scratch(hipStream_t s, void** out) {
    int cur = 0, dev = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return api_fail(DMD_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    dev = cur;
    if (s) {
        e = hipStreamGetDevice(s, &dev);
        if (e != hipSuccess) return api_fail(DMD_E_INVAL, "hipStreamGetDevice: %s", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices) return api_fail(DMD_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess)
            return api_fail(DMD_E_DEVICE, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t eback = dev != cur ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess || !p)
            return api_fail(DMD_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        if (eback != hipSuccess)
            return api_fail(DMD_E_DEVICE, "hipSetDevice(%d): %s", cur, hipGetErrorString(eback));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DMD_OK;
}

}  // namespace dmd

DMD_API int dmd_window_gram_noalloc(const void* X, int64_t ldx, int64_t n, int32_t ncols, int32_t dtype,
                                    int32_t precision, double* G, int64_t ldg, void* stream) {
    int eb = 0;
    if (int rc = dmd::check_window_gram(X, ldx, n, ncols, dtype, precision, G, ldg, &eb)) return rc;
    if (ldg > INT32_MAX) return dmd::api_fail(DMD_E_INVAL, "ldg too large");
    const size_t need = dmd::window_gram_scratch_bytes(ncols);
    if (need > dmd::kNoAllocBytes)
        return dmd::api_fail(DMD_E_INVAL, "%d columns need %zu bytes of scratch; the allocation-free call holds %zu",
                             ncols, need, dmd::kNoAllocBytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void* partial = nullptr;
    if (int rc = dmd::noalloc_scratch(s, &partial)) return rc;
    const hipError_t e =
        dmd::launch_window_gram(X, ldx, n, ncols, eb == 8, precision, G, ldg, static_cast<double*>(partial), s);
    if (e != hipSuccess) return dmd::api_fail(DMD_E_DEVICE, "window Gram launch: %s", hipGetErrorString(e));
    return DMD_OK;
}

DMD_API int dmd_window_gram(const void* X, int64_t ldx, int64_t n, int32_t ncols, int32_t dtype,
                            int32_t precision, double* G, int64_t ldg, void* stream) {
    int eb = 0;
    if (int rc = dmd::check_window_gram(X, ldx, n, ncols, dtype, precision, G, ldg, &eb)) return rc;
    if (ldg > INT32_MAX) return dmd::api_fail(DMD_E_INVAL, "ldg too large");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void* partial = nullptr;
    hipError_t e = hipMallocAsync(&partial, dmd::window_gram_scratch_bytes(ncols), s);
    if (e != hipSuccess)
        return dmd::api_fail(DMD_E_NOMEM, "hipMallocAsync(%zu): %s", dmd::window_gram_scratch_bytes(ncols),
                                     hipGetErrorString(e));
    e = dmd::launch_window_gram(X, ldx, n, ncols, eb == 8, precision, G, ldg, static_cast<double*>(partial), s);
    const hipError_t ef = hipFreeAsync(partial, s);
    if (e != hipSuccess) return dmd::api_fail(DMD_E_DEVICE, "window Gram launch: %s", hipGetErrorString(e));
    if (ef != hipSuccess) return dmd::api_fail(DMD_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(ef));
    return DMD_OK;
}
