// Minimal FP64 complex arithmetic for device code.
#pragma once
#include <hip/hip_runtime.h>

namespace dmd {

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx mkc(double re, double im = 0.0) { return cplx{re, im}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator-(cplx a) { return {-a.re, -a.im}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cplx operator*(cplx a, double s) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cplx conj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ double abs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
// a * conj(b) and conj(a) * b without forming the conjugate
__device__ __forceinline__ cplx mul_conj(cplx a, cplx b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
__device__ __forceinline__ cplx conj_mul(cplx a, cplx b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// Smith's division, robust against overflow in |b|^2.
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        const double r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
// Principal square root.
__device__ __forceinline__ cplx csqrt(cplx z) {
    const double a = cabs(z);
    if (a == 0.0) return {0.0, 0.0};
    if (z.re >= 0.0) {
        const double t = sqrt(0.5 * (a + z.re));
        return {t, z.im / (2.0 * t)};
    } else {
        const double t = sqrt(0.5 * (a - z.re));
        return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
    }
}

// Scalar traits so that one Jacobi implementation serves real symmetric and
// complex Hermitian Gram matrices.
template <typename S> struct Scal;
template <> struct Scal<double> {
    static __device__ __forceinline__ double zero() { return 0.0; }
    static __device__ __forceinline__ double one() { return 1.0; }
    static __device__ __forceinline__ double re(double a) { return a; }
    static __device__ __forceinline__ double absv(double a) { return fabs(a); }
    static __device__ __forceinline__ double cj(double a) { return a; }
    static __device__ __forceinline__ double phase(double a) { return a < 0.0 ? -1.0 : 1.0; }
    static __device__ __forceinline__ cplx toc(double a) { return {a, 0.0}; }
    static __device__ __forceinline__ double fromc(cplx a) { return a.re; }
};
template <> struct Scal<cplx> {
    static __device__ __forceinline__ cplx zero() { return {0.0, 0.0}; }
    static __device__ __forceinline__ cplx one() { return {1.0, 0.0}; }
    static __device__ __forceinline__ double re(cplx a) { return a.re; }
    static __device__ __forceinline__ double absv(cplx a) { return cabs(a); }
    static __device__ __forceinline__ cplx cj(cplx a) { return conj(a); }
    static __device__ __forceinline__ cplx phase(cplx a) {
        const double m = cabs(a);
        return m > 0.0 ? cplx{a.re / m, a.im / m} : cplx{1.0, 0.0};
    }
    static __device__ __forceinline__ cplx toc(cplx a) { return a; }
    static __device__ __forceinline__ cplx fromc(cplx a) { return a; }
};

__device__ __forceinline__ double mulr(double a, double b) { return a * b; }
__device__ __forceinline__ cplx mulr(cplx a, cplx b) { return a * b; }
__device__ __forceinline__ cplx mulr(double a, cplx b) { return a * b; }
__device__ __forceinline__ cplx mulr(cplx a, double b) { return a * b; }

}  // namespace dmd
