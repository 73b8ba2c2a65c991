// Shared device/host helpers of the mireg HIP library (gfx950).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mireg {

// Complex number held in two registers; 8 bytes (float) or 16 bytes (double).
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> make_cx(T r, T i) {
    cx<T> z;
    z.re = r;
    z.im = i;
    return z;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return make_cx(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return make_cx(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return make_cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return make_cx(a.re * s, a.im * s); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return make_cx(a.re, -a.im); }
// multiply by i
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return make_cx(-a.im, a.re); }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return make_cx(a.im, -a.re); }

// Storage conversions: fields may be held in a narrower type S than the
// arithmetic type T (FP16 storage of transported fields, FP32 arithmetic).
template <typename T, typename S>
__device__ __forceinline__ T load_as(const S *p, long long i) {
    return (T)p[i];
}
template <>
__device__ __forceinline__ float load_as<float, __half>(const __half *p, long long i) {
    return __half2float(p[i]);
}
template <>
__device__ __forceinline__ double load_as<double, __half>(const __half *p, long long i) {
    return (double)__half2float(p[i]);
}
template <typename S, typename T>
__device__ __forceinline__ void store_as(S *p, long long i, T v) {
    p[i] = (S)v;
}
template <>
__device__ __forceinline__ void store_as<__half, float>(__half *p, long long i, float v) {
    p[i] = __float2half_rn(v);
}

// Integer wavenumber of FFT index j on an axis of length n (the Nyquist
// index n/2 maps to -n/2).
__device__ __forceinline__ int wavenumber(int j, int n) { return j < n / 2 ? j : j - n; }

// Grid geometry passed by value to kernels.
struct Grid {
    int n1, n2, n3;
    int k3;          // n3/2 + 1, length of the half-spectrum rows
    long long N;     // n1 n2 n3
    long long NS;    // n1 n2 k3 (complex entries of one half spectrum)
    int lds_cap;     // largest stencil box (points) staged in LDS; 0: gather from global memory
    int sl_tile;     // tile shape of the semi-Lagrangian kernels (0, 1, 2)
    int x1_narrow;   // Krylov x1 passes on FP32 256-point lines: 16-column workgroups instead of 32
};

}  // namespace mireg
