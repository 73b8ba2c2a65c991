// Register/LDS building blocks of the pencil FFT passes.
//
// A line of length L (2^a, 3 2^a or 5 2^a) is held by TPC = L/EPT threads; thread
// t keeps the elements at positions t + TPC*e, e = 0..EPT-1, in registers.
// The transform is a mixed-radix Stockham sequence (radices R0, R1, R2 from
// FftCfg): every stage takes butterflies j = t + TPC*b, reads inputs
// j + m*L/R (which are exactly the thread's own registers b + m*EPT/R),
// twiddles them by w_{Ns R}^{m (j mod Ns)}, applies an R-point DFT and sends
// output m to position (j / Ns) Ns R + (j mod Ns) + m Ns.  Between stages the
// outputs pass through LDS; after the last stage they land back on the
// thread's own positions, so loads and stores of a pass use the same
// coalesced pattern.
#pragma once

#include "common.hpp"

namespace mireg {

// cos / sin of 2 pi j / 16, exact to double rounding.
__host__ __device__ constexpr double cos16(int j) {
    return ((j & 15) == 0)   ? 1.0
           : ((j & 15) == 1) ? 0.92387953251128675613
           : ((j & 15) == 2) ? 0.70710678118654752440
           : ((j & 15) == 3) ? 0.38268343236508977173
           : ((j & 15) == 4) ? 0.0
           : ((j & 15) == 5) ? -0.38268343236508977173
           : ((j & 15) == 6) ? -0.70710678118654752440
           : ((j & 15) == 7) ? -0.92387953251128675613
           : ((j & 15) == 8) ? -1.0
           : ((j & 15) == 9) ? -0.92387953251128675613
           : ((j & 15) == 10) ? -0.70710678118654752440
           : ((j & 15) == 11) ? -0.38268343236508977173
           : ((j & 15) == 12) ? 0.0
           : ((j & 15) == 13) ? 0.38268343236508977173
           : ((j & 15) == 14) ? 0.70710678118654752440
                              : 0.92387953251128675613;
}
__host__ __device__ constexpr double sin16(int j) { return cos16(j - 4); }

// cos / sin of 2 pi j / 6 and 2 pi j / 10, exact to double rounding.
__host__ __device__ constexpr double cos6(int j) {
    return (j % 6 == 0) ? 1.0 : (j % 6 == 1 || j % 6 == 5) ? 0.5 : (j % 6 == 3) ? -1.0 : -0.5;
}
__host__ __device__ constexpr double sin6(int j) {
    return (j % 6 == 0 || j % 6 == 3) ? 0.0
           : (j % 6 == 1 || j % 6 == 2) ? 0.86602540378443864676
                                         : -0.86602540378443864676;
}
__host__ __device__ constexpr double cos10(int j) {
    return (j % 10 == 0)                    ? 1.0
           : (j % 10 == 1 || j % 10 == 9)   ? 0.80901699437494742410
           : (j % 10 == 2 || j % 10 == 8)   ? 0.30901699437494742410
           : (j % 10 == 3 || j % 10 == 7)   ? -0.30901699437494742410
           : (j % 10 == 4 || j % 10 == 6)   ? -0.80901699437494742410
                                            : -1.0;
}
__host__ __device__ constexpr double sin10(int j) {
    return (j % 10 == 0 || j % 10 == 5)   ? 0.0
           : (j % 10 == 1 || j % 10 == 4) ? 0.58778525229247312917
           : (j % 10 == 2 || j % 10 == 3) ? 0.95105651629515357212
           : (j % 10 == 6 || j % 10 == 9) ? -0.58778525229247312917
                                          : -0.95105651629515357212;
}

// w_R^p = exp(DIR * 2 pi i p / R) for R dividing 16, 6 or 10 (DIR = -1 forward).
template <typename T, int R, int DIR>
__device__ __forceinline__ cx<T> root(int p) {
    if constexpr (16 % R == 0) {
        const int j = (p * (16 / R)) & 15;
        return make_cx<T>((T)cos16(j), (T)(DIR * sin16(j)));
    } else if constexpr (6 % R == 0) {
        const int j = (p * (6 / R)) % 6;
        return make_cx<T>((T)cos6(j), (T)(DIR * sin6(j)));
    } else {
        static_assert(10 % R == 0, "unsupported root of unity");
        const int j = (p * (10 / R)) % 10;
        return make_cx<T>((T)cos10(j), (T)(DIR * sin10(j)));
    }
}

// In-register DFT of length R in {1, 2, 4, 8, 16}, natural order in and out.
template <typename T, int R, int DIR>
struct Dft {
    static __device__ __forceinline__ void run(cx<T> *x) {
        // R = R1 * R2 with R1 = 4: inputs n = R2 n1 + n2, outputs k = k1 + 4 k2
        constexpr int R1 = 4, R2 = R / 4;
        cx<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            cx<T> a[4];
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n1] = x[R2 * n1 + n2];
            Dft<T, 4, DIR>::run(a);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2 * 4 + k1] = (n2 * k1 == 0) ? a[k1] : a[k1] * root<T, R, DIR>(n2 * k1);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cx<T> b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = y[n2 * 4 + k1];
            Dft<T, R2, DIR>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) x[k1 + 4 * k2] = b[k2];
        }
    }
};
template <typename T, int DIR>
struct Dft<T, 1, DIR> {
    static __device__ __forceinline__ void run(cx<T> *) {}
};
template <typename T, int DIR>
struct Dft<T, 2, DIR> {
    static __device__ __forceinline__ void run(cx<T> *x) {
        cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    }
};
template <typename T, int DIR>
struct Dft<T, 4, DIR> {
    static __device__ __forceinline__ void run(cx<T> *x) {
        cx<T> s02 = x[0] + x[2], d02 = x[0] - x[2];
        cx<T> s13 = x[1] + x[3], d13 = x[1] - x[3];
        // w_4 = -i forward, +i inverse
        cx<T> r = (DIR < 0) ? mul_mi(d13) : mul_i(d13);
        x[0] = s02 + s13;
        x[2] = s02 - s13;
        x[1] = d02 + r;
        x[3] = d02 - r;
    }
};
template <typename T, int DIR>
struct Dft<T, 8, DIR> {
    static __device__ __forceinline__ void run(cx<T> *x) {
        // 8 = 4 x 2: inputs n = 2 n1 + n2, outputs k = k1 + 4 k2
        cx<T> y[8];
#pragma unroll
        for (int n2 = 0; n2 < 2; ++n2) {
            cx<T> a[4] = {x[n2], x[2 + n2], x[4 + n2], x[6 + n2]};
            Dft<T, 4, DIR>::run(a);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2 * 4 + k1] = (n2 * k1 == 0) ? a[k1] : a[k1] * root<T, 8, DIR>(n2 * k1);
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            x[k1] = y[k1] + y[4 + k1];
            x[k1 + 4] = y[k1] - y[4 + k1];
        }
    }
};

// Odd radices: the DFT of length 3 and 5 written out with the real and
// imaginary parts of their roots, and 6 = 2 x 3, 10 = 2 x 5 by one radix-2
// step over two odd-length DFTs (even and odd inputs).
template <typename T, int DIR>
struct Dft<T, 3, DIR> {
    static __device__ __forceinline__ void run(cx<T> *x) {
        const cx<T> s = x[1] + x[2], d = x[1] - x[2];
        const cx<T> a = x[0] - scale(s, (T)0.5);
        const cx<T> id = (DIR < 0) ? mul_mi(d) : mul_i(d);
        const cx<T> b = scale(id, (T)0.86602540378443864676);
        x[0] = x[0] + s;
        x[1] = a + b;
        x[2] = a - b;
    }
};
template <typename T, int DIR>
struct Dft<T, 5, DIR> {
    static __device__ __forceinline__ void run(cx<T> *x) {
        constexpr T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        constexpr T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        const cx<T> a1 = x[1] + x[4], b1 = x[1] - x[4], a2 = x[2] + x[3], b2 = x[2] - x[3];
        const cx<T> p1 = x[0] + scale(a1, c1) + scale(a2, c2);
        const cx<T> p2 = x[0] + scale(a1, c2) + scale(a2, c1);
        const cx<T> q1 = scale(b1, s1) + scale(b2, s2), q2 = scale(b1, s2) - scale(b2, s1);
        const cx<T> iq1 = (DIR < 0) ? mul_mi(q1) : mul_i(q1), iq2 = (DIR < 0) ? mul_mi(q2) : mul_i(q2);
        x[0] = x[0] + a1 + a2;
        x[1] = p1 + iq1;
        x[4] = p1 - iq1;
        x[2] = p2 + iq2;
        x[3] = p2 - iq2;
    }
};
template <typename T, int Q, int DIR>
struct DftTwoOdd {
    static __device__ __forceinline__ void run(cx<T> *x) {
        cx<T> e[Q], o[Q];
#pragma unroll
        for (int n = 0; n < Q; ++n) {
            e[n] = x[2 * n];
            o[n] = x[2 * n + 1];
        }
        Dft<T, Q, DIR>::run(e);
        Dft<T, Q, DIR>::run(o);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const cx<T> t = k == 0 ? o[0] : o[k] * root<T, 2 * Q, DIR>(k);
            x[k] = e[k] + t;
            x[k + Q] = e[k] - t;
        }
    }
};
template <typename T, int DIR>
struct Dft<T, 6, DIR> : DftTwoOdd<T, 3, DIR> {};
template <typename T, int DIR>
struct Dft<T, 10, DIR> : DftTwoOdd<T, 5, DIR> {};

// Elements per thread and radices per line length, in two variants: V = 0
// (16 elements per thread for FP32 at L >= 128) and V = 1 (at most 8, for
// kernels that keep several lines in registers).  Every radix divides EPT
// so that a thread's butterflies read only its own registers.
template <typename T, int L, int V>
struct FftCfg;
#define MIREG_FFTCFG(TY, LL, VV, E, A, B, C) \
    template <>                              \
    struct FftCfg<TY, LL, VV> {              \
        static constexpr int EPT = E;        \
        static constexpr int R0 = A;         \
        static constexpr int R1 = B;         \
        static constexpr int R2 = C;         \
    };
#define MIREG_FFTCFG2(TY, LL, E, A, B, C) MIREG_FFTCFG(TY, LL, 0, E, A, B, C) MIREG_FFTCFG(TY, LL, 1, E, A, B, C)
MIREG_FFTCFG2(float, 2, 2, 2, 1, 1)
MIREG_FFTCFG2(float, 4, 4, 4, 1, 1)
MIREG_FFTCFG2(float, 8, 4, 4, 2, 1)
MIREG_FFTCFG2(float, 16, 4, 4, 4, 1)
MIREG_FFTCFG2(float, 32, 8, 8, 4, 1)
MIREG_FFTCFG2(float, 64, 8, 8, 8, 1)
MIREG_FFTCFG(float, 128, 0, 16, 16, 8, 1)
MIREG_FFTCFG(float, 128, 1, 8, 8, 4, 4)
MIREG_FFTCFG(float, 256, 0, 16, 16, 16, 1)
MIREG_FFTCFG(float, 256, 1, 8, 8, 8, 4)
MIREG_FFTCFG(float, 512, 0, 16, 16, 8, 4)
MIREG_FFTCFG(float, 512, 1, 8, 8, 8, 8)
MIREG_FFTCFG2(double, 2, 2, 2, 1, 1)
MIREG_FFTCFG2(double, 4, 4, 4, 1, 1)
MIREG_FFTCFG2(double, 8, 4, 4, 2, 1)
MIREG_FFTCFG2(double, 16, 4, 4, 4, 1)
MIREG_FFTCFG2(double, 32, 8, 8, 4, 1)
MIREG_FFTCFG2(double, 64, 8, 8, 8, 1)
MIREG_FFTCFG2(double, 128, 8, 8, 4, 4)
MIREG_FFTCFG2(double, 256, 8, 8, 8, 4)
MIREG_FFTCFG2(double, 512, 8, 8, 8, 8)
// 3 2^a and 5 2^a (grids of 48, 80, 96 and 160 points per axis and their
// half-length x3 lines); one configuration for both variants
#define MIREG_FFTCFG_T(LL, E, A, B, C) MIREG_FFTCFG2(float, LL, E, A, B, C) MIREG_FFTCFG2(double, LL, E, A, B, C)
MIREG_FFTCFG_T(24, 12, 4, 6, 1)
MIREG_FFTCFG_T(40, 20, 4, 10, 1)
MIREG_FFTCFG_T(48, 12, 4, 4, 3)
MIREG_FFTCFG_T(80, 20, 4, 4, 5)
MIREG_FFTCFG_T(96, 12, 4, 4, 6)
MIREG_FFTCFG_T(160, 20, 4, 4, 10)
#undef MIREG_FFTCFG_T
#undef MIREG_FFTCFG2
#undef MIREG_FFTCFG

__host__ __device__ constexpr bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Register array of one thread's share of a line.
template <typename T, int L, int V>
using Regs = cx<T>[FftCfg<T, L, V>::EPT];

// Workgroup shape of a pass: NT threads, TPC per line, W lines.
template <typename T, int L, int V, int NT>
struct FftShape {
    static constexpr int EPT = FftCfg<T, L, V>::EPT;
    static constexpr int TPC = L / EPT;  // threads per line
    static constexpr int W = NT / TPC;   // lines per workgroup
};

// LDS index of (line c, position p): strided passes keep lines (columns)
// fastest, the contiguous x3 passes keep positions fastest (padded rows).
template <int W>
struct LayoutCols {
    static __device__ __forceinline__ int at(int c, int p) { return p * W + c; }
    static constexpr int size(int L) { return L * W; }
};
// Rows of power-of-two lines of 32 points and more carry one element of
// padding after every 2^SH positions (SH = 4 from 128 points, else 3): the
// first Stockham stage stores R consecutive positions per thread, at a
// stride of R between the threads of a line, and a flat row would put those
// threads on one bank; the skew spreads them, and the reads of consecutive
// positions that follow stay spread too.  Shorter and 3/5-smooth lines keep
// one element of padding per row.
template <int W, int L>
struct LayoutRows {
    static constexpr int SH = (is_pow2(L) && L >= 32) ? (L >= 128 ? 4 : 3) : 0;
    static constexpr int PITCH = SH ? L + (L >> SH) : L + 1;
    static __device__ __forceinline__ int at(int c, int p) { return c * PITCH + (SH ? p + (p >> SH) : p); }
    static constexpr int size(int) { return W * PITCH; }
};

// One Stockham stage of radix R after sub-transforms of length NS.
// tw: table exp(-2 pi i j / Ltab), read at stride Ltab / L.
template <typename T, int L, int V, int R, int NS, int DIR, bool LAST, class Lay>
__device__ __forceinline__ void stockham_stage(Regs<T, L, V> &reg, int t, int c,
                                               const cx<T> *__restrict__ tw, int twstride,
                                               cx<T> *lds) {
    constexpr int EPT = FftCfg<T, L, V>::EPT;
    constexpr int TPC = L / EPT;
    constexpr int NB = EPT / R;
    cx<T> out[EPT];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + TPC * b;
        const int k = j % NS;
        cx<T> v[R];
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = reg[b + m * NB];
        if (NS > 1) {
#pragma unroll
            for (int m = 1; m < R; ++m) {
                cx<T> w = tw[(m * k) * (L / (NS * R)) * twstride];
                if (DIR > 0) w.im = -w.im;
                v[m] = v[m] * w;
            }
        }
        Dft<T, R, DIR>::run(v);
#pragma unroll
        for (int m = 0; m < R; ++m) out[b + m * NB] = v[m];
    }
    if (LAST) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) reg[e] = out[e];
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + TPC * b;
            const int k = j % NS;
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int m = 0; m < R; ++m) lds[Lay::at(c, base + m * NS)] = out[b + m * NB];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) reg[e] = lds[Lay::at(c, t + TPC * e)];
        __syncthreads();
    }
}

// Full unnormalised transform of one line: X[k] = sum_n x[n] exp(DIR 2 pi i n k / L).
template <typename T, int L, int V, int DIR, class Lay>
__device__ __forceinline__ void fft_line(Regs<T, L, V> &reg, int t, int c,
                                         const cx<T> *__restrict__ tw, int twstride, cx<T> *lds) {
    using C = FftCfg<T, L, V>;
    constexpr bool one = (C::R1 == 1);
    constexpr bool two = (C::R1 > 1 && C::R2 == 1);
    stockham_stage<T, L, V, C::R0, 1, DIR, one, Lay>(reg, t, c, tw, twstride, lds);
    if constexpr (C::R1 > 1)
        stockham_stage<T, L, V, C::R1, C::R0, DIR, two, Lay>(reg, t, c, tw, twstride, lds);
    if constexpr (C::R2 > 1)
        stockham_stage<T, L, V, C::R2, C::R0 * C::R1, DIR, true, Lay>(reg, t, c, tw, twstride, lds);
}

}  // namespace mireg
