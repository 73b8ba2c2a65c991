// Vector kernels and FP64 reductions for the Krylov and line-search scalars.
//
// Reductions are two-stage and deterministic: kRedBlocks workgroups each
// reduce a grid-stride share into one FP64 partial, then a single workgroup
// combines the partials in a fixed order.  FP32 inputs are widened to FP64
// before any arithmetic, so dot products, norms and the objective are FP64
// for both storage types.
#include <float.h>

#include "kernels.hpp"

namespace mireg {

constexpr int kRedThreads = 256;

// Block-wide sum of NV doubles per thread; thread 0 ends with the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double sh[NV][kRedThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[k][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0;
            for (int w = 0; w < kRedThreads / 64; ++w) s += sh[k][w];
            v[k] = s;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_scalar(const T *__restrict__ a, const T *__restrict__ b,
                                                            long long n, double *__restrict__ part) {
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads)
        v[0] += (double)a[i] * (double)b[i];
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Four consecutive elements per step (one 16- or 32-byte load per operand),
// four independent FP64 accumulators; the n % 4 tail is added by block 0.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot(const T *__restrict__ a, const T *__restrict__ b,
                                                     long long n, double *__restrict__ part) {
    using V4 = typename Vec4<T>::type;
    const long long n4 = n / 4;
    const V4 *a4 = reinterpret_cast<const V4 *>(a), *b4 = reinterpret_cast<const V4 *>(b);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n4;
         i += (long long)gridDim.x * kRedThreads) {
        const V4 x = a4[i], y = b4[i];
        s0 += (double)x.x * (double)y.x;
        s1 += (double)x.y * (double)y.y;
        s2 += (double)x.z * (double)y.z;
        s3 += (double)x.w * (double)y.w;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) s0 += (double)a[4 * n4 + threadIdx.x] * (double)b[4 * n4 + threadIdx.x];
    double v[1] = {(s0 + s1) + (s2 + s3)};
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename TA, typename TB>
__global__ __launch_bounds__(kRedThreads) void k_sumsq_diff(const TA *__restrict__ a, const TB *__restrict__ b,
                                                            long long n, double *__restrict__ part) {
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double d = load_as<double>(a, i) - load_as<double>(b, i);
        v[0] += d * d;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename T>
__device__ __forceinline__ T pcg_step(double k, T s, T Hs, T &x, T &r, double &acc);

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_pcg_update_scalar(long long n, double k, const T *__restrict__ s,
                                                                   const T *__restrict__ Hs, T *__restrict__ x,
                                                                   T *__restrict__ r, double *__restrict__ part) {
    double v[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads)
        pcg_step(k, s[i], Hs[i], x[i], r[i], v[0]);
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename T>
__device__ __forceinline__ T pcg_step(double k, T s, T Hs, T &x, T &r, double &acc) {
    x = (T)((double)x + k * (double)s);
    r = (T)((double)r - k * (double)Hs);
    acc += (double)r * (double)r;
    return r;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_pcg_update(long long n, double k, const T *__restrict__ s,
                                                            const T *__restrict__ Hs, T *__restrict__ x,
                                                            T *__restrict__ r, double *__restrict__ part) {
    using V4 = typename Vec4<T>::type;
    const long long n4 = n / 4;
    const V4 *s4 = reinterpret_cast<const V4 *>(s), *h4 = reinterpret_cast<const V4 *>(Hs);
    V4 *x4 = reinterpret_cast<V4 *>(x), *r4 = reinterpret_cast<V4 *>(r);
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n4;
         i += (long long)gridDim.x * kRedThreads) {
        const V4 sv = s4[i], hv = h4[i];
        V4 xv = x4[i], rv = r4[i];
        pcg_step(k, sv.x, hv.x, xv.x, rv.x, a0);
        pcg_step(k, sv.y, hv.y, xv.y, rv.y, a1);
        pcg_step(k, sv.z, hv.z, xv.z, rv.z, a2);
        pcg_step(k, sv.w, hv.w, xv.w, rv.w, a3);
        x4[i] = xv;
        r4[i] = rv;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {
        const long long i = 4 * n4 + threadIdx.x;
        pcg_step(k, s[i], Hs[i], x[i], r[i], a0);
    }
    double v[1] = {(a0 + a1) + (a2 + a3)};
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Final stage for sums: result[k] = sum_b part[b * NV + k] ... partials are
// stored field-major: part[k * kRedBlocks + b].
template <int NV>
__global__ __launch_bounds__(kRedThreads) void k_finish_sum(const double *__restrict__ part, double *__restrict__ res) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0;
        for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads) s += part[k * kRedBlocks + b];
        v[k] = s;
    }
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) res[k] = v[k];
    }
}

// min, max and non-finite count in one sweep
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_minmax(const T *__restrict__ a, long long n,
                                                        double *__restrict__ part) {
    __shared__ double smin[kRedThreads], smax[kRedThreads], sbad[kRedThreads];
    double mn = DBL_MAX, mx = -DBL_MAX, bad = 0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double x = (double)a[i];
        if (!isfinite(x)) {
            bad += 1;
        } else {
            mn = fmin(mn, x);
            mx = fmax(mx, x);
        }
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            sbad[threadIdx.x] += sbad[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = smin[0];
        part[kRedBlocks + blockIdx.x] = smax[0];
        part[2 * kRedBlocks + blockIdx.x] = sbad[0];
    }
}

__global__ __launch_bounds__(kRedThreads) void k_finish_minmax(const double *__restrict__ part,
                                                               double *__restrict__ res) {
    if (threadIdx.x == 0) {
        double mn = DBL_MAX, mx = -DBL_MAX, bad = 0;
        for (int b = 0; b < kRedBlocks; ++b) {
            mn = fmin(mn, part[b]);
            mx = fmax(mx, part[kRedBlocks + b]);
            bad += part[2 * kRedBlocks + b];
        }
        res[0] = mn;
        res[1] = mx;
        res[2] = bad;
    }
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_max_norm2(const T *__restrict__ v, long long N,
                                                           double *__restrict__ part) {
    __shared__ double sm[kRedThreads];
    double mx = 0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < N;
         i += (long long)gridDim.x * kRedThreads) {
        const double a = v[i], b = v[N + i], c = v[2 * N + i];
        mx = fmax(mx, a * a + b * b + c * c);
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kRedThreads) void k_finish_max(const double *__restrict__ part,
                                                            double *__restrict__ res) {
    if (threadIdx.x == 0) {
        double mx = 0;
        for (int b = 0; b < kRedBlocks; ++b) mx = fmax(mx, part[b]);
        res[0] = mx;
    }
}

template <typename T>
__global__ void k_axpby(long long n, double a, const T *__restrict__ x, double b, T *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}

template <typename T>
__global__ void k_xpay(long long n, const T *x, double a, const T *y, T *z) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        z[i] = (T)((double)x[i] + a * (double)y[i]);
}

template <typename T>
__global__ void k_affine(long long n, const T *__restrict__ x, double a, double b, T *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = (T)(a * (double)x[i] + b);
}

template <typename T>
__global__ void k_fill(long long n, T val, T *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = val;
}

static inline unsigned stream_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

thread_local KernelHook *g_hook = nullptr;
const char *const kKernelNames[K_COUNT] = {
    "fft_r2c_x3", "fft_c2c_x2_fwd", "fft_c2c_x2_inv", "fft_x1_scale", "fft_x1_grad", "fft_x1_div",
    "fft_x1_proj", "fft_x1_tail", "fft_c2r_x3", "sl_departure", "sl_interp", "sl_adjoint_init",
    "sl_adjoint_step", "sl_adjoint_accum", "sl_incstate_init", "sl_incstate_step", "reduce", "vector",
    "fft_x1_krylov", "krylov_update"};

// Vector kernels read 4 elements at once when the pointer allows it.
template <typename T>
static bool aligned4(const T *p) {
    return (reinterpret_cast<uintptr_t>(p) % (4 * sizeof(T))) == 0;
}

template <typename T>
void dot(const T *a, const T *b, long long n, double *partials, double *result, hipStream_t s) {
    HookScope hs(K_REDUCE, 2.0 * n * sizeof(T));
    if (aligned4(a) && aligned4(b))
        hipLaunchKernelGGL((k_dot<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, partials);
    else
        hipLaunchKernelGGL((k_dot_scalar<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, partials);
    hipLaunchKernelGGL((k_finish_sum<1>), dim3(1), dim3(kRedThreads), 0, s, partials, result);
}
template <typename TA, typename TB>
void sumsq_diff(const TA *a, const TB *b, long long n, double *partials, double *result, hipStream_t s) {
    HookScope hs(K_REDUCE, (double)n * (sizeof(TA) + sizeof(TB)));
    hipLaunchKernelGGL((k_sumsq_diff<TA, TB>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, partials);
    hipLaunchKernelGGL((k_finish_sum<1>), dim3(1), dim3(kRedThreads), 0, s, partials, result);
}
template <typename T>
void pcg_update(long long n, double k, const T *sdir, const T *Hs, T *x, T *r, double *partials,
                double *result, hipStream_t s) {
    HookScope hs(K_VECTOR, 6.0 * n * sizeof(T));
    if (aligned4(sdir) && aligned4(Hs) && aligned4(x) && aligned4(r))
        hipLaunchKernelGGL((k_pcg_update<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, k, sdir, Hs, x, r,
                           partials);
    else
        hipLaunchKernelGGL((k_pcg_update_scalar<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, k, sdir, Hs, x,
                           r, partials);
    hipLaunchKernelGGL((k_finish_sum<1>), dim3(1), dim3(kRedThreads), 0, s, partials, result);
}
template <typename T>
void minmax_nonfinite(const T *a, long long n, double *partials, double *result, hipStream_t s) {
    HookScope hs(K_REDUCE, 1.0 * n * sizeof(T));
    hipLaunchKernelGGL((k_minmax<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, n, partials);
    hipLaunchKernelGGL(k_finish_minmax, dim3(1), dim3(kRedThreads), 0, s, partials, result);
}
template <typename T>
void max_norm2(const T *v, long long N, double *partials, double *result, hipStream_t s) {
    HookScope hs(K_REDUCE, 3.0 * N * sizeof(T));
    hipLaunchKernelGGL((k_max_norm2<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, v, N, partials);
    hipLaunchKernelGGL(k_finish_max, dim3(1), dim3(kRedThreads), 0, s, partials, result);
}
template <typename T>
void axpby(long long n, double a, const T *x, double b, T *y, hipStream_t s) {
    HookScope hs(K_VECTOR, 3.0 * n * sizeof(T));
    hipLaunchKernelGGL((k_axpby<T>), dim3(stream_blocks(n)), dim3(256), 0, s, n, a, x, b, y);
}
template <typename T>
void xpay(long long n, const T *x, double a, const T *y, T *z, hipStream_t s) {
    HookScope hs(K_VECTOR, 3.0 * n * sizeof(T));
    hipLaunchKernelGGL((k_xpay<T>), dim3(stream_blocks(n)), dim3(256), 0, s, n, x, a, y, z);
}
template <typename T>
void affine(long long n, const T *x, double a, double b, T *y, hipStream_t s) {
    HookScope hs(K_VECTOR, 2.0 * n * sizeof(T));
    hipLaunchKernelGGL((k_affine<T>), dim3(stream_blocks(n)), dim3(256), 0, s, n, x, a, b, y);
}
template <typename T>
void fill(long long n, T val, T *y, hipStream_t s) {
    HookScope hs(K_VECTOR, 1.0 * n * sizeof(T));
    hipLaunchKernelGGL((k_fill<T>), dim3(stream_blocks(n)), dim3(256), 0, s, n, val, y);
}

#define MIREG_INST(T)                                                                                 \
    template void dot<T>(const T *, const T *, long long, double *, double *, hipStream_t);           \
    template void sumsq_diff<T, T>(const T *, const T *, long long, double *, double *, hipStream_t); \
    template void pcg_update<T>(long long, double, const T *, const T *, T *, T *, double *, double *, \
                                hipStream_t);                                                         \
    template void minmax_nonfinite<T>(const T *, long long, double *, double *, hipStream_t);         \
    template void max_norm2<T>(const T *, long long, double *, double *, hipStream_t);                \
    template void axpby<T>(long long, double, const T *, double, T *, hipStream_t);                   \
    template void xpay<T>(long long, const T *, double, const T *, T *, hipStream_t);                 \
    template void affine<T>(long long, const T *, double, double, T *, hipStream_t);                  \
    template void fill<T>(long long, T, T *, hipStream_t);
MIREG_INST(float)
MIREG_INST(double)
#undef MIREG_INST

}  // namespace mireg
