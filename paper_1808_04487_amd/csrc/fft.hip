// Pencil FFT passes and fused pseudospectral operators for gfx950.
//
// Spectral derivatives and their inverses follow the paper's scheme (Sec.
// 2.3.1): forward FFT, pointwise weights, inverse FFT.  A real field
// [n1][n2][n3] maps to a half spectrum [n1][n2][n3/2+1] (complex).  Each
// operator is five launches, every one a single coalesced sweep over HBM:
//   1. x3: real-to-complex along the contiguous axis (an n3/2-point complex
//      FFT of the even/odd pairs, then the split into n3/2+1 modes),
//   2. x2: complex transform of the columns at stride n3/2+1,
//   3. x1: forward transform, the operator's weights for every field at
//      this mode, inverse transform -- one kernel, the spectrum of the
//      operator's inputs never goes back to HBM,
//   4. x2 inverse, 5. x3 complex-to-real.
// Odd symbols (i k_a: gradient, divergence and the wavenumbers inside K)
// vanish at the Nyquist index; even symbols (|k|^2, |k|^4, Gaussian) keep it.
#include <type_traits>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace mireg {

// ---------------------------------------------------------------------------
// x3 real-to-complex and complex-to-real passes (lines contiguous in memory)
// ---------------------------------------------------------------------------
constexpr int kLineThreads = 256;  // x3 passes
constexpr int kColThreads = 512;   // strided passes: wide column tiles
// Workgroup sizes: the above for power-of-two lines; for 3 2^a and 5 2^a
// lines (fewer threads per line) as many lines as keep the LDS tile below
// about 40 KB -- 64 x3 lines or 32 columns in FP32, half of that in FP64.
template <typename T, int M>
constexpr int line_threads() {
    return is_pow2(M) ? kLineThreads : (sizeof(T) == 4 ? 64 : 32) * (M / FftCfg<T, M, 0>::EPT);
}
template <typename T, int L, int V>
constexpr int col_threads() {
    return is_pow2(L) ? kColThreads : (sizeof(T) == 4 ? 32 : 16) * (L / FftCfg<T, L, V>::EPT);
}

// SI: element type of the real input (FP32 input of an FP64 transform is
// widened at the load)
// tab (device, or null): problem blockIdx.z's (src, dst) pair at
// tab[2 z], tab[2 z + 1] in place of src and dst (several problems of one
// grid size in one launch); the same convention in the other passes.
template <typename T, int M, typename SI = T, bool TAB = false>
__global__ __launch_bounds__(kLineThreads) void k_r2c_x3(FieldPtrs src, FieldPtrs dst,
                                                         long long lines,
                                                         const cx<T> *__restrict__ tw,
                                                         const FieldPtrs *__restrict__ tab) {
    using S = FftShape<T, M, 0, line_threads<T, M>()>;
    constexpr int EPT = S::EPT, TPC = S::TPC, W = S::W;
    using Lay = LayoutRows<W, M>;
    __shared__ cx<T> lds[Lay::size(M)];
    const int t = threadIdx.x % TPC, c = threadIdx.x / TPC;
    const long long line = (long long)blockIdx.x * W + c;
    const bool ok = line < lines;
    void *dp = TAB ? tab[2 * blockIdx.z + 1].p[blockIdx.y] : dst.p[blockIdx.y];
    const void *sp = TAB ? tab[2 * blockIdx.z].p[blockIdx.y] : src.p[blockIdx.y];
    cx<T> *out = reinterpret_cast<cx<T> *>(dp) + line * (M + 1);
    cx<T> reg[EPT];
    const cx<SI> *in = reinterpret_cast<const cx<SI> *>(sp) + line * M;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const cx<SI> z = ok ? in[t + TPC * e] : make_cx<SI>(0, 0);
        reg[e] = make_cx<T>((T)z.re, (T)z.im);
    }
    fft_line<T, M, 0, -1, Lay>(reg, t, c, tw, 2, lds);
#pragma unroll
    for (int e = 0; e < EPT; ++e) lds[Lay::at(c, t + TPC * e)] = reg[e];
    __syncthreads();
    if (ok) {
        // X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[M-k])/2, O = (Z[k] - conj Z[M-k])/(2i)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int k = t + TPC * e;
            const cx<T> zk = lds[Lay::at(c, k)];
            const cx<T> zm = conj(lds[Lay::at(c, (M - k) % M)]);
            const cx<T> E = scale(zk + zm, (T)0.5);
            const cx<T> O = scale(mul_mi(zk - zm), (T)0.5);
            out[k] = E + tw[k] * O;
        }
        if (t == 0) {
            const cx<T> z0 = lds[Lay::at(c, 0)];
            out[M] = make_cx<T>(z0.re - z0.im, (T)0);
        }
    }
}

template <typename T, int M, bool TAB = false>
__global__ __launch_bounds__(kLineThreads) void k_c2r_x3(FieldPtrs src, FieldPtrs dst,
                                                         long long lines,
                                                         const cx<T> *__restrict__ tw,
                                                         const FieldPtrs *__restrict__ tab) {
    using S = FftShape<T, M, 0, line_threads<T, M>()>;
    constexpr int EPT = S::EPT, TPC = S::TPC, W = S::W;
    using Lay = LayoutRows<W, M>;
    __shared__ cx<T> lds[Lay::size(M)];
    const int t = threadIdx.x % TPC, c = threadIdx.x / TPC;
    const long long line = (long long)blockIdx.x * W + c;
    const bool ok = line < lines;
    const void *sp = TAB ? tab[2 * blockIdx.z].p[blockIdx.y] : src.p[blockIdx.y];
    void *dp = TAB ? tab[2 * blockIdx.z + 1].p[blockIdx.y] : dst.p[blockIdx.y];
    const cx<T> *in = reinterpret_cast<const cx<T> *>(sp) + line * (M + 1);
    cx<T> *out = reinterpret_cast<cx<T> *>(dp) + line * M;
    cx<T> reg[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int k = t + TPC * e;
        if (ok) {
            cx<T> xk = in[k], xm = in[M - k];
            if (k == 0) {  // self-conjugate modes of a real line
                xk.im = 0;
                xm.im = 0;
            }
            const cx<T> E = xk + conj(xm);
            const cx<T> O = (xk - conj(xm)) * conj(tw[k]);
            reg[e] = E + mul_i(O);
        } else {
            reg[e] = make_cx<T>(0, 0);
        }
    }
    fft_line<T, M, 0, +1, Lay>(reg, t, c, tw, 2, lds);
    if (ok) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) out[t + TPC * e] = reg[e];
    }
}

// ---------------------------------------------------------------------------
// Strided complex pass: columns q < Q, column base (q / inner) * ostride +
// q % inner, element p of a column at base + p * pstride.
// ---------------------------------------------------------------------------
// Workgroup -> (field, column group) with contiguous runs of column groups
// per XCD (workgroups are dispatched round-robin over the 8 XCDs): the rows
// of neighbouring groups share cache lines at their unaligned ends, and
// neighbours on one XCD share its L2.
__device__ __forceinline__ void xcd_block(int &bx, int &by) {
    const int nb = (int)(gridDim.x * gridDim.y), lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int q = nb / 8, r = nb % 8, x = lin % 8, j = lin / 8;
    const int g = x * q + (x < r ? x : r) + j;
    bx = g % (int)gridDim.x;
    by = g / (int)gridDim.x;
}

template <typename T, int L, int DIR, bool TAB = false>
__global__ __launch_bounds__(kColThreads) void k_c2c_cols(FieldPtrs f, long long Q, long long inner,
                                                          long long ostride, long long pstride,
                                                          const cx<T> *__restrict__ tw,
                                                          const FieldPtrs *__restrict__ tab) {
    using S = FftShape<T, L, 0, col_threads<T, L, 0>()>;
    constexpr int EPT = S::EPT, TPC = S::TPC, W = S::W;
    using Lay = LayoutCols<W>;
    __shared__ cx<T> lds[Lay::size(L)];
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    int bx, by;
    xcd_block(bx, by);
    const long long q = (long long)bx * W + c;
    const bool ok = q < Q;
    const long long base = ok ? (q / inner) * ostride + (q % inner) : 0;
    cx<T> *p = reinterpret_cast<cx<T> *>(TAB ? tab[blockIdx.z].p[by] : f.p[by]) + base;
    cx<T> reg[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) reg[e] = ok ? p[(long long)(t + TPC * e) * pstride] : make_cx<T>(0, 0);
    fft_line<T, L, 0, DIR, Lay>(reg, t, c, tw, 1, lds);
    if (ok) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) p[(long long)(t + TPC * e) * pstride] = reg[e];
    }
}

// ---------------------------------------------------------------------------
// x1 pass with the operator in the middle.
// ---------------------------------------------------------------------------
template <typename T>
struct OpConst {
    int n1, n2, n3, k3;
    int sym, nf, reg, div;
    T alpha, beta_v, beta_w;
    T gs1, gs2, gs3;  // Gaussian: (2 pi sigma / n_a)^2 / 2
    T norm;           // 1 / (n1 n2 n3)
    double *red;      // per-workgroup partials of sum_x in out, or null
};

template <typename T>
struct Mode {
    T k1, k2, k3;     // full wavenumbers (Nyquist as -n/2 or n3/2)
    T t1, t2, t3;     // odd-symbol wavenumbers (Nyquist -> 0)
};

template <typename T>
__device__ __forceinline__ T ksq(const Mode<T> &m) { return m.k1 * m.k1 + m.k2 * m.k2 + m.k3 * m.k3; }
template <typename T>
__device__ __forceinline__ T reg_symbol(const Mode<T> &m, int reg) {
    const T s = ksq(m);
    return reg == 2 ? s * s : s;
}

template <typename T>
__device__ __forceinline__ T scalar_symbol(const Mode<T> &m, const OpConst<T> &oc) {
    switch (oc.sym) {
        case SYM_A: return oc.alpha * reg_symbol(m, oc.reg);
        case SYM_AINV: {
            const T s = oc.alpha * reg_symbol(m, oc.reg);
            return ksq(m) == (T)0 ? (T)1 : (T)1 / s;  // zero singular value set to one
        }
        case SYM_LAP: return -ksq(m);
        case SYM_GRADSQ: return m.t1 * m.t1 + m.t2 * m.t2 + m.t3 * m.t3;
        case SYM_GAUSS:
            return exp(-(oc.gs1 * m.k1 * m.k1 + oc.gs2 * m.k2 * m.k2 + oc.gs3 * m.k3 * m.k3));
        case SYM_AINV_SQRT: {
            const T s = oc.alpha * reg_symbol(m, oc.reg);
            return ksq(m) == (T)0 ? (T)1 : (T)1 / sqrt(s);
        }
        case SYM_HIGHPASS: {
            const bool low = 4 * fabs(m.k1) < (T)oc.n1 && 4 * fabs(m.k2) < (T)oc.n2 && 4 * fabs(m.k3) < (T)oc.n3;
            return low ? (T)0 : (T)1;
        }
        default: return (T)1;
    }
}

// K b per mode: b - c(k) kt (kt . b) / |kt|^2
template <typename T>
__device__ __forceinline__ void project(const Mode<T> &m, const OpConst<T> &oc, cx<T> &b1, cx<T> &b2,
                                        cx<T> &b3) {
    if (oc.div == 0) return;
    const T kts = m.t1 * m.t1 + m.t2 * m.t2 + m.t3 * m.t3;
    if (kts == (T)0) return;
    T cw = (T)1;
    if (oc.div == 1) {
        const T w = oc.beta_w * (kts + (T)1);
        cw = w / (oc.beta_v + w);
    }
    const T f = cw / kts;
    const cx<T> s = scale(scale(b1, m.t1) + scale(b2, m.t2) + scale(b3, m.t3), f);
    b1 = b1 - scale(s, m.t1);
    b2 = b2 - scale(s, m.t2);
    b3 = b3 - scale(s, m.t3);
}

// The x1 operators keep several lines (or the operator's symbols) in
// registers: they use the low-register variant of the line transform.
template <int KIND>
constexpr int x1_variant() { return 1; }

template <typename T, int L, int KIND>
__global__ __launch_bounds__(kColThreads) void k_x1_op(FieldPtrs f, long long Q, OpConst<T> oc,
                                                       const cx<T> *__restrict__ tw) {
    constexpr int V = x1_variant<KIND>();
    constexpr int NT = col_threads<T, L, V>();
    using S = FftShape<T, L, V, NT>;
    constexpr int EPT = S::EPT, TPC = S::TPC, W = S::W;
    using Lay = LayoutCols<W>;
    __shared__ cx<T> lds[Lay::size(L)];
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    const long long q = (long long)blockIdx.x * W + c;
    const bool ok = q < Q;
    const long long qq = ok ? q : 0;
    const long long pstride = Q;
    // mode of register e: k1 index t + TPC e, column q -> (k2, k3)
    const int i2 = (int)(qq / oc.k3), i3 = (int)(qq % oc.k3);
    const T k2 = (T)wavenumber(i2, oc.n2), k3 = (T)i3;
    const T t2 = (2 * i2 == oc.n2) ? (T)0 : k2, t3 = (2 * i3 == oc.n3) ? (T)0 : k3;
    auto mode = [&](int e) {
        Mode<T> m;
        const int i1 = t + TPC * e;
        m.k1 = (T)wavenumber(i1, oc.n1);
        m.t1 = (2 * i1 == oc.n1) ? (T)0 : m.k1;
        m.k2 = k2;
        m.t2 = t2;
        m.k3 = k3;
        m.t3 = t3;
        return m;
    };
    auto load = [&](int slot, cx<T>(&r)[EPT]) {
        const cx<T> *p = reinterpret_cast<const cx<T> *>(f.p[slot]) + qq;
#pragma unroll
        for (int e = 0; e < EPT; ++e) r[e] = ok ? p[(long long)(t + TPC * e) * pstride] : make_cx<T>(0, 0);
    };
    auto store = [&](int slot, cx<T>(&r)[EPT]) {
        cx<T> *p = reinterpret_cast<cx<T> *>(f.p[slot]) + qq;
        if (ok) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) p[(long long)(t + TPC * e) * pstride] = r[e];
        }
    };
    cx<T> reg[EPT];
    // Parseval: sum_x in out = sum over the half spectrum of w Re(conj(in^) out^ / N),
    // w = 1 on the k3 = 0 and Nyquist planes, 2 elsewhere
    double dacc = 0;
    const double wk3 = (i3 == 0 || 2 * i3 == oc.n3) ? 1.0 : 2.0;
    auto dot_mode = [&](const cx<T> &a, const cx<T> &b) {
        dacc += wk3 * ((double)a.re * (double)b.re + (double)a.im * (double)b.im);
    };
    if constexpr (KIND == SPEC_SCALE) {
        for (int fi = 0; fi < oc.nf; ++fi) {
            load(fi, reg);
            fft_line<T, L, V, -1, Lay>(reg, t, c, tw, 1, lds);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const cx<T> in = reg[e];
                reg[e] = scale(in, scalar_symbol(mode(e), oc) * oc.norm);
                if (oc.red && ok) dot_mode(in, reg[e]);
            }
            fft_line<T, L, V, +1, Lay>(reg, t, c, tw, 1, lds);
            store(fi, reg);
        }
    } else if constexpr (KIND == SPEC_GRAD) {
        cx<T> u[EPT];
        load(0, u);
        fft_line<T, L, V, -1, Lay>(u, t, c, tw, 1, lds);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const Mode<T> m = mode(e);
                const T ka = a == 0 ? m.t1 : (a == 1 ? m.t2 : m.t3);
                reg[e] = scale(mul_i(u[e]), ka * oc.norm);
            }
            fft_line<T, L, V, +1, Lay>(reg, t, c, tw, 1, lds);
            store(a, reg);
        }
    } else if constexpr (KIND == SPEC_DIV) {
        cx<T> acc[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = make_cx<T>(0, 0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            load(a, reg);
            fft_line<T, L, V, -1, Lay>(reg, t, c, tw, 1, lds);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const Mode<T> m = mode(e);
                const T ka = a == 0 ? m.t1 : (a == 1 ? m.t2 : m.t3);
                acc[e] = acc[e] + scale(mul_i(reg[e]), ka * oc.norm);
            }
        }
        fft_line<T, L, V, +1, Lay>(acc, t, c, tw, 1, lds);
        store(0, acc);
    } else if constexpr (KIND == SPEC_REG) {
        // Regulariser of v by Parseval, nothing transformed back: per mode
        // beta_v/2 a(k) sum_a |v_a|^2 and, for the near-incompressible model
        // (w = div v = i kt . v eliminated), beta_w/2 (|kt|^2 + 1) |w|^2.
        cx<T> w[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) w[e] = make_cx<T>(0, 0);
        double pv = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            load(a, reg);
            fft_line<T, L, V, -1, Lay>(reg, t, c, tw, 1, lds);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const Mode<T> m = mode(e);
                const T ka = a == 0 ? m.t1 : (a == 1 ? m.t2 : m.t3);
                pv += (double)reg_symbol(m, oc.reg) * ((double)reg[e].re * reg[e].re + (double)reg[e].im * reg[e].im);
                w[e] = w[e] + scale(mul_i(reg[e]), ka);
            }
        }
        double pw = 0;
        if (oc.div == 1) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const Mode<T> m = mode(e);
                const double kts = (double)m.t1 * m.t1 + (double)m.t2 * m.t2 + (double)m.t3 * m.t3;
                pw += (kts + 1.0) * ((double)w[e].re * w[e].re + (double)w[e].im * w[e].im);
            }
        }
        if (ok) dacc = wk3 * (double)oc.norm * (0.5 * (double)oc.beta_v * pv + 0.5 * (double)oc.beta_w * pw);
    } else {
        // SPEC_PROJ: K u for u in slots 0..2.
        // SPEC_TAIL: alpha A u + K b, u in slots 0..2, b in slots 3..5.
        constexpr int boff = (KIND == SPEC_TAIL) ? 3 : 0;
        cx<T> b0[EPT], b1[EPT], b2[EPT];
        load(boff + 0, b0);
        fft_line<T, L, V, -1, Lay>(b0, t, c, tw, 1, lds);
        load(boff + 1, b1);
        fft_line<T, L, V, -1, Lay>(b1, t, c, tw, 1, lds);
        load(boff + 2, b2);
        fft_line<T, L, V, -1, Lay>(b2, t, c, tw, 1, lds);
#pragma unroll
        for (int e = 0; e < EPT; ++e) project(mode(e), oc, b0[e], b1[e], b2[e]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T>(&ba)[EPT] = a == 0 ? b0 : (a == 1 ? b1 : b2);
            if constexpr (KIND == SPEC_TAIL) {
                load(a, reg);
                fft_line<T, L, V, -1, Lay>(reg, t, c, tw, 1, lds);
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const T s = oc.alpha * reg_symbol(mode(e), oc.reg);
                    const cx<T> in = reg[e];
                    reg[e] = scale(scale(in, s) + ba[e], oc.norm);
                    if (oc.red && ok) dot_mode(in, reg[e]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < EPT; ++e) reg[e] = scale(ba[e], oc.norm);
            }
            fft_line<T, L, V, +1, Lay>(reg, t, c, tw, 1, lds);
            store(a, reg);
        }
    }
    if constexpr (KIND == SPEC_SCALE || KIND == SPEC_TAIL || KIND == SPEC_REG) {
        if (oc.red) {
            __shared__ double red_sh[NT / 64];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) dacc += __shfl_down(dacc, off, 64);
            if ((threadIdx.x & 63) == 0) red_sh[threadIdx.x >> 6] = dacc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tot = 0;
                for (int w = 0; w < NT / 64; ++w) tot += red_sh[w];
                oc.red[blockIdx.x] = tot;
            }
        }
    }
}

// out[0] = sum of n partials in a fixed order (one workgroup)
// out[0] = sum of part[0 .. n-1]; with jobs (device, or null), job
// blockIdx.x's (part, out) in their place.
struct SumJob {
    const double *part;
    double *out;
};
__global__ __launch_bounds__(256) void k_sum_partials(int n, const double *__restrict__ part_arg,
                                                      double *__restrict__ out_arg, const SumJob *__restrict__ jobs) {
    const double *part = jobs ? jobs[blockIdx.x].part : part_arg;
    double *out = jobs ? jobs[blockIdx.x].out : out_arg;
    __shared__ double sh[4];
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ---------------------------------------------------------------------------
// Krylov vectors held as spectra.  PCG keeps x, r and the direction s as
// their half spectra F u (all three axes transformed, unnormalised forward
// DFT, the [k1][k2][k3] order the x1 pass leaves), three arrays of NS modes
// per vector field.  The preconditioner is a pointwise multiplier there and
// the Hessian's spectral tail needs the spectrum of s, which is kept: one
// forward transform (of the transport output b) and one inverse (of the new
// direction) per iteration instead of the five of the physical-space
// iteration.  Sums over the grid come from Parseval: sum_x u v =
// (1/N) sum over the half spectrum of w Re(conj(F u) F v), w = 1 on the
// k3 = 0 and Nyquist planes, 2 elsewhere.
// ---------------------------------------------------------------------------
struct KrylovPtrs {
    void *w[3];        // x2/x3-transformed work spectra
    const void *a[3];  // spectral operand
    void *o[3];        // spectral output (read first in KP_DIR; read only, the old direction, in KP_INV)
    void *x[3];        // iterate updated with the old direction (KP_DIR with KF_XUPD)
    const double *alpha;  // device step length of the KF_XUPD updates
    double mu;            // KP_DIR's mu, when read from a table
    double *red;          // KP_HESS's reduction partials, when read from a table
};

// x1 passes of the Krylov iteration (flags: KF_*, kernels.hpp):
//   KP_FWD:  o = x1 forward transform of w                      (F u from the x2/x3 spectra)
//   KP_HESS: o = alpha a(k) a_in + K F b, with F b from w;       red: sum_x s . Hs
//            KF_SQRT: the symmetrically scaled operator c (alpha a(k) c a_in + K F b),
//            c = (alpha a(k))^{-1/2} (1 at k = 0), F b being the transport of c a_in
//   KP_DIR:  o = z + mu o (o not read with KF_FIRST), z = M^{-1}(k) a_in, or a_in
//            with KF_ZRAW; w = x1 inverse of o / N (of c o / N with KF_SQRT);
//            KF_XUPD: first x += alpha o with the old o (the iterate's update of
//            the previous iteration, deferred to this pass, which reads o anyway)
//   KP_INV:  w = x1 inverse of a_in / N; KF_XUPD: of (a_in + alpha o) / N
// KP_FWD, KP_DIR and KP_INV treat component blockIdx.y; KP_HESS all three.
template <typename T>
__device__ __forceinline__ T ainv_sqrt_symbol(const Mode<T> &m, const OpConst<T> &oc) {
    return ksq(m) == (T)0 ? (T)1 : (T)1 / sqrt(oc.alpha * reg_symbol(m, oc.reg));
}
// Workgroup size of the Krylov x1 passes: 1024 threads (32 columns, 256-byte
// rows, still over a thousand workgroups per component) for FP32 lines of
// 256 points, where they fit 128 registers without spilling; the column
// default otherwise.
template <typename T, int L, bool NARROW = false>
constexpr int krylov_threads() {
    return (sizeof(T) == 4 && L == 256 && !NARROW) ? 1024 : col_threads<T, L, 1>();
}
// Launch bound: at least that of the other column passes, so the other
// instantiations keep their register budget.
template <typename T, int L>
constexpr int krylov_bound() {
    return krylov_threads<T, L>() > kColThreads ? krylov_threads<T, L>() : kColThreads;
}
// SA: element type of the spectral operand a_in of KP_HESS (an FP64
// spectrum read by an FP32 pass is rounded at the load)
// NARROW: the 16-column workgroups (Grid::x1_narrow) where 32 is the default
template <typename T, int L, int PASS, typename SA = T, bool TAB = false, bool NARROW = false>
__global__ __launch_bounds__((krylov_bound<T, L>())) void k_x1_krylov(KrylovPtrs farg, long long Q, OpConst<T> oc,
                                                                      T mu_arg, int flags,
                                                                      const cx<T> *__restrict__ tw,
                                                                      const KrylovPtrs *__restrict__ tab) {
    // problem blockIdx.z's operands (its mu and reduction partials) from tab
    const KrylovPtrs f = TAB ? tab[blockIdx.z] : farg;
    const T mu = TAB ? (T)f.mu : mu_arg;
    double *const red = TAB ? f.red : oc.red;
    const bool first = flags & KF_FIRST, sqrt_scaled = flags & KF_SQRT, zraw = flags & KF_ZRAW;
    const bool xupd = flags & KF_XUPD;
    const T alpha = xupd ? (T)*f.alpha : (T)0;
    constexpr int V = 1;
    constexpr int NT = krylov_threads<T, L, NARROW>();
    using S = FftShape<T, L, V, NT>;
    constexpr int EPT = S::EPT, TPC = S::TPC, W = S::W;
    using Lay = LayoutCols<W>;
    __shared__ cx<T> lds[Lay::size(L)];
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    const long long q = (long long)blockIdx.x * W + c;
    const bool ok = q < Q;
    const long long qq = ok ? q : 0;
    const int i2 = (int)(qq / oc.k3), i3 = (int)(qq % oc.k3);
    const T k2 = (T)wavenumber(i2, oc.n2), k3 = (T)i3;
    const T t2 = (2 * i2 == oc.n2) ? (T)0 : k2, t3 = (2 * i3 == oc.n3) ? (T)0 : k3;
    auto mode = [&](int e) {
        Mode<T> m;
        const int i1 = t + TPC * e;
        m.k1 = (T)wavenumber(i1, oc.n1);
        m.t1 = (2 * i1 == oc.n1) ? (T)0 : m.k1;
        m.k2 = k2;
        m.t2 = t2;
        m.k3 = k3;
        m.t3 = t3;
        return m;
    };
    auto load = [&](const void *base, cx<T>(&r)[EPT]) {
        const cx<T> *p = reinterpret_cast<const cx<T> *>(base) + qq;
#pragma unroll
        for (int e = 0; e < EPT; ++e) r[e] = ok ? p[(long long)(t + TPC * e) * Q] : make_cx<T>(0, 0);
    };
    auto store = [&](void *base, cx<T>(&r)[EPT]) {
        cx<T> *p = reinterpret_cast<cx<T> *>(base) + qq;
        if (ok) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) p[(long long)(t + TPC * e) * Q] = r[e];
        }
    };
    cx<T> reg[EPT];
    double dacc = 0;
    const double wk3 = (i3 == 0 || 2 * i3 == oc.n3) ? 1.0 : 2.0;
    if constexpr (PASS == KP_FWD) {
        {
            const int a = blockIdx.y;
            load(f.w[a], reg);
            fft_line<T, L, V, -1, Lay>(reg, t, c, tw, 1, lds);
            store(f.o[a], reg);
        }
    } else if constexpr (PASS == KP_HESS) {
        cx<T> b0[EPT], b1[EPT], b2[EPT];
        load(f.w[0], b0);
        fft_line<T, L, V, -1, Lay>(b0, t, c, tw, 1, lds);
        load(f.w[1], b1);
        fft_line<T, L, V, -1, Lay>(b1, t, c, tw, 1, lds);
        load(f.w[2], b2);
        fft_line<T, L, V, -1, Lay>(b2, t, c, tw, 1, lds);
#pragma unroll
        for (int e = 0; e < EPT; ++e) project(mode(e), oc, b0[e], b1[e], b2[e]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T>(&ba)[EPT] = a == 0 ? b0 : (a == 1 ? b1 : b2);
            if constexpr (std::is_same<SA, T>::value) {
                load(f.a[a], reg);
            } else {
                const cx<SA> *p = reinterpret_cast<const cx<SA> *>(f.a[a]) + qq;
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const cx<SA> z = ok ? p[(long long)(t + TPC * e) * Q] : make_cx<SA>(0, 0);
                    reg[e] = make_cx<T>((T)z.re, (T)z.im);
                }
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const cx<T> sh = reg[e];
                const Mode<T> m = mode(e);
                if (sqrt_scaled) {
                    const T c = ainv_sqrt_symbol(m, oc);
                    reg[e] = scale(scale(scale(sh, c), oc.alpha * reg_symbol(m, oc.reg)) + ba[e], c);
                } else {
                    reg[e] = scale(sh, oc.alpha * reg_symbol(m, oc.reg)) + ba[e];
                }
                if (ok) dacc += wk3 * ((double)sh.re * (double)reg[e].re + (double)sh.im * (double)reg[e].im);
            }
            store(f.o[a], reg);
        }
    } else if constexpr (PASS == KP_DIR) {
        {
            const int a = blockIdx.y;
            if (!first) load(f.o[a], reg);
            if (xupd && !first) {  // before r is read, so the three sets are never live together
                cx<T> xv[EPT];
                load(f.x[a], xv);
#pragma unroll
                for (int e = 0; e < EPT; ++e) xv[e] = xv[e] + scale(reg[e], alpha);
                store(f.x[a], xv);
            }
            cx<T> rh[EPT];
            load(f.a[a], rh);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const cx<T> z = zraw ? rh[e] : scale(rh[e], scalar_symbol(mode(e), oc));
                reg[e] = first ? z : z + scale(reg[e], mu);
            }
            store(f.o[a], reg);
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                reg[e] = scale(reg[e], sqrt_scaled ? ainv_sqrt_symbol(mode(e), oc) * oc.norm : oc.norm);
            fft_line<T, L, V, +1, Lay>(reg, t, c, tw, 1, lds);
            store(f.w[a], reg);
        }
    } else {
        {
            const int a = blockIdx.y;
            load(f.a[a], reg);
            if (xupd) {
                cx<T> sv[EPT];
                load(f.o[a], sv);
#pragma unroll
                for (int e = 0; e < EPT; ++e) reg[e] = reg[e] + scale(sv[e], alpha);
            }
#pragma unroll
            for (int e = 0; e < EPT; ++e) reg[e] = scale(reg[e], oc.norm);
            fft_line<T, L, V, +1, Lay>(reg, t, c, tw, 1, lds);
            store(f.w[a], reg);
        }
    }
    if constexpr (PASS == KP_HESS) {
        if (red) {
            __shared__ double red_sh[NT / 64];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) dacc += __shfl_down(dacc, off, 64);
            if ((threadIdx.x & 63) == 0) red_sh[threadIdx.x >> 6] = dacc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double tot = 0;
                for (int w = 0; w < NT / 64; ++w) tot += red_sh[w];
                red[blockIdx.x] = tot * (double)oc.norm;
            }
        }
    }
}

// x, r, s, Hs spectra (three components each), by value.
template <typename T>
struct KrylovSet {
    cx<T> *p[12];
};

// Pointwise step of the spectral PCG: with update, alpha = res[num] / res[0]
// (the step length from the sums of the previous passes, on the device) and,
// when res[0] > 0, r -= alpha Hs (the iterate takes alpha s in the next
// direction pass; res[3] = alpha, or 0 when res[0] <= 0 and r is kept);
// then per-workgroup partials of sum_x r . M^{-1} r (part[b]) and
// sum_x r . r (part[nb + b]) from r.  Grid-stride over the NS modes with a
// fixed grid, so the sums are reproducible.
// One problem of a multi-problem k_krylov_update (problem blockIdx.y).
template <typename T>
struct KrylovUpd {
    KrylovSet<T> v;
    double *res, *part;
};

template <typename T, bool TAB = false>
__global__ __launch_bounds__(256) void k_krylov_update(unsigned NS, int n1, int n2, int n3, int k3, int reg,
                                                       T beta_v, int update, int num, double *res_arg,
                                                       KrylovSet<T> v_arg, double norm, double *__restrict__ part_arg,
                                                       const KrylovUpd<T> *__restrict__ tab) {
    const KrylovSet<T> v = TAB ? tab[blockIdx.y].v : v_arg;
    double *res = TAB ? tab[blockIdx.y].res : res_arg;
    double *part = TAB ? tab[blockIdx.y].part : part_arg;
    cx<T> *const *r = v.p;
    const cx<T> *const *h = v.p + 3;
    const double den = update ? res[0] : 0.0, step = update ? res[num] / den : 0.0;
    const bool write = update && den > 0;
    const T alpha = (T)step;
    if (update && blockIdx.x == 0 && threadIdx.x == 0) res[3] = write ? step : 0.0;
    double rz = 0, rr = 0;
    for (unsigned j = blockIdx.x * 256u + threadIdx.x; j < NS; j += gridDim.x * 256u) {
        const unsigned i3 = j % (unsigned)k3, row = j / (unsigned)k3;
        const unsigned i2 = row % (unsigned)n2, i1 = row / (unsigned)n2;
        const T w1 = (T)wavenumber((int)i1, n1), w2 = (T)wavenumber((int)i2, n2), w3 = (T)i3;
        const T ks = w1 * w1 + w2 * w2 + w3 * w3;
        const T sym = reg == 2 ? ks * ks : ks;
        const double sigma = ks == (T)0 ? 1.0 : (double)((T)1 / (beta_v * sym));
        const double wk3 = (i3 == 0 || 2 * i3 == (unsigned)n3) ? 1.0 : 2.0;
        double m2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<T> rv = r[a][j];
            if (write) {
                rv = rv - scale(h[a][j], alpha);
                r[a][j] = rv;
            }
            m2 += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
        }
        rr += wk3 * m2;
        rz += wk3 * sigma * m2;
    }
    __shared__ double sh[2][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rz += __shfl_down(rz, off, 64);
        rr += __shfl_down(rr, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = rz;
        sh[1][threadIdx.x >> 6] = rr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ((sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3])) * norm;
        part[gridDim.x + blockIdx.x] = ((sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3])) * norm;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
// x3 lines (n3 / 2) and strided lines (n1, n2) of the supported grids:
// powers of two and 48, 80, 96, 160
#define MIREG_SWITCH_LINE(n, MACRO) \
    switch (n) {                    \
        case 4: MACRO(4); break;    \
        case 8: MACRO(8); break;    \
        case 16: MACRO(16); break;  \
        case 24: MACRO(24); break;  \
        case 32: MACRO(32); break;  \
        case 40: MACRO(40); break;  \
        case 48: MACRO(48); break;  \
        case 64: MACRO(64); break;  \
        case 80: MACRO(80); break;  \
        case 128: MACRO(128); break;\
        case 256: MACRO(256); break;\
        default: break;             \
    }
#define MIREG_SWITCH_COL(n, MACRO)  \
    switch (n) {                    \
        case 8: MACRO(8); break;    \
        case 16: MACRO(16); break;  \
        case 32: MACRO(32); break;  \
        case 48: MACRO(48); break;  \
        case 64: MACRO(64); break;  \
        case 80: MACRO(80); break;  \
        case 96: MACRO(96); break;  \
        case 128: MACRO(128); break;\
        case 160: MACRO(160); break;\
        case 256: MACRO(256); break;\
        case 512: MACRO(512); break;\
        default: break;             \
    }

template <typename T, typename SI = T>
static void launch_r2c(const Grid &g, FieldPtrs src, FieldPtrs dst, int nf, const cx<T> *tw,
                       hipStream_t s, const FieldPtrs *tab = nullptr, int np = 1) {
    const long long lines = (long long)g.n1 * g.n2;
    HookScope hs(K_R2C, (double)np * nf * (sizeof(SI) * g.N + 2.0 * sizeof(T) * g.NS));
#define MIREG_L(M)                                                                                     \
    {                                                                                                  \
        constexpr int NT = line_threads<T, M>();                                                       \
        constexpr int W = FftShape<T, M, 0, NT>::W;                                                    \
        dim3 grid((unsigned)((lines + W - 1) / W), nf, np);                                            \
        if (tab)                                                                                       \
            hipLaunchKernelGGL((k_r2c_x3<T, M, SI, true>), grid, dim3(NT), 0, s, src, dst, lines, tw, tab); \
        else                                                                                           \
            hipLaunchKernelGGL((k_r2c_x3<T, M, SI>), grid, dim3(NT), 0, s, src, dst, lines, tw, tab);  \
    }
    MIREG_SWITCH_LINE(g.n3 / 2, MIREG_L)
#undef MIREG_L
}

template <typename T>
static void launch_c2r(const Grid &g, FieldPtrs src, FieldPtrs dst, int nf, const cx<T> *tw,
                       hipStream_t s, const FieldPtrs *tab = nullptr, int np = 1) {
    const long long lines = (long long)g.n1 * g.n2;
    HookScope hs(K_C2R, (double)np * nf * sizeof(T) * (g.N + 2.0 * g.NS));
#define MIREG_L(M)                                                                                     \
    {                                                                                                  \
        constexpr int NT = line_threads<T, M>();                                                       \
        constexpr int W = FftShape<T, M, 0, NT>::W;                                                    \
        dim3 grid((unsigned)((lines + W - 1) / W), nf, np);                                            \
        if (tab)                                                                                       \
            hipLaunchKernelGGL((k_c2r_x3<T, M, true>), grid, dim3(NT), 0, s, src, dst, lines, tw, tab); \
        else                                                                                           \
            hipLaunchKernelGGL((k_c2r_x3<T, M>), grid, dim3(NT), 0, s, src, dst, lines, tw, tab);      \
    }
    MIREG_SWITCH_LINE(g.n3 / 2, MIREG_L)
#undef MIREG_L
}

template <typename T, int DIR>
static void launch_x2(const Grid &g, FieldPtrs f, int nf, const cx<T> *tw, hipStream_t s,
                      const FieldPtrs *tab = nullptr, int np = 1) {
    const long long Q = (long long)g.n1 * g.k3, inner = g.k3, ostride = (long long)g.n2 * g.k3,
                    pstride = g.k3;
    HookScope hs(DIR < 0 ? K_C2C_FWD : K_C2C_INV, (double)np * nf * sizeof(T) * 4.0 * g.NS);
#define MIREG_L(L)                                                                           \
    {                                                                                        \
        constexpr int NT = col_threads<T, L, 0>();                                           \
        constexpr int W = FftShape<T, L, 0, NT>::W;                                          \
        dim3 grid((unsigned)((Q + W - 1) / W), nf, np);                                      \
        if (tab)                                                                             \
            hipLaunchKernelGGL((k_c2c_cols<T, L, DIR, true>), grid, dim3(NT), 0, s, f, Q, inner, \
                               ostride, pstride, tw, tab);                                   \
        else                                                                                 \
            hipLaunchKernelGGL((k_c2c_cols<T, L, DIR>), grid, dim3(NT), 0, s, f, Q, inner,   \
                               ostride, pstride, tw, tab);                                   \
    }
    MIREG_SWITCH_COL(g.n2, MIREG_L)
#undef MIREG_L
}

template <typename T, int KIND>
static int launch_x1(const Grid &g, FieldPtrs f, int nin, int nout, const OpConst<T> &oc,
                     const cx<T> *tw, hipStream_t s) {
    const long long Q = (long long)g.n2 * g.k3;
    HookScope hs(K_X1_SCALE + KIND, (double)(nin + nout) * sizeof(T) * 2.0 * g.NS);
    int blocks = 0;
#define MIREG_L(L)                                                                              \
    {                                                                                           \
        constexpr int NT = col_threads<T, L, x1_variant<KIND>()>();                             \
        constexpr int W = FftShape<T, L, x1_variant<KIND>(), NT>::W;                            \
        dim3 grid((unsigned)((Q + W - 1) / W));                                                 \
        blocks = (int)grid.x;                                                                   \
        hipLaunchKernelGGL((k_x1_op<T, L, KIND>), grid, dim3(NT), 0, s, f, Q, oc, tw);          \
    }
    MIREG_SWITCH_COL(g.n1, MIREG_L)
#undef MIREG_L
    return blocks;
}

template <typename T>
void spectral_apply(const Grid &g, int kind, int nin, int nout, const void *const *in, T *const *out,
                    cx<T> *spec, const Twiddles<T> &tw, const SpecParams &sp, hipStream_t s) {
    FieldPtrs fin{}, fspec{}, fout{};
    for (int i = 0; i < nin; ++i) fin.p[i] = const_cast<void *>(in[i]);
    for (int i = 0; i < 6; ++i) fspec.p[i] = spec + (long long)i * g.NS;
    for (int i = 0; i < nout; ++i) fout.p[i] = out[i];

    OpConst<T> oc;
    oc.n1 = g.n1;
    oc.n2 = g.n2;
    oc.n3 = g.n3;
    oc.k3 = g.k3;
    oc.sym = sp.sym;
    oc.nf = sp.nf;
    oc.reg = sp.reg;
    oc.div = sp.div;
    oc.alpha = (T)sp.alpha;
    oc.beta_v = (T)sp.beta_v;
    oc.beta_w = (T)sp.beta_w;
    const double two_pi = 6.283185307179586476925;
    oc.gs1 = (T)(0.5 * (two_pi * sp.sigma / g.n1) * (two_pi * sp.sigma / g.n1));
    oc.gs2 = (T)(0.5 * (two_pi * sp.sigma / g.n2) * (two_pi * sp.sigma / g.n2));
    oc.gs3 = (T)(0.5 * (two_pi * sp.sigma / g.n3) * (two_pi * sp.sigma / g.n3));
    oc.norm = (T)(1.0 / ((double)g.n1 * g.n2 * g.n3));
    oc.red = (kind == SPEC_SCALE || kind == SPEC_TAIL || kind == SPEC_REG) ? sp.red : nullptr;

    launch_r2c<T>(g, fin, fspec, nin, tw.t[2], s);
    launch_x2<T, -1>(g, fspec, nin, tw.t[1], s);
    int blocks = 0;
    switch (kind) {
        case SPEC_SCALE: blocks = launch_x1<T, SPEC_SCALE>(g, fspec, nin, nout, oc, tw.t[0], s); break;
        case SPEC_GRAD: launch_x1<T, SPEC_GRAD>(g, fspec, nin, nout, oc, tw.t[0], s); break;
        case SPEC_DIV: launch_x1<T, SPEC_DIV>(g, fspec, nin, nout, oc, tw.t[0], s); break;
        case SPEC_PROJ: launch_x1<T, SPEC_PROJ>(g, fspec, nin, nout, oc, tw.t[0], s); break;
        case SPEC_REG: blocks = launch_x1<T, SPEC_REG>(g, fspec, nin, nout, oc, tw.t[0], s); break;
        default: blocks = launch_x1<T, SPEC_TAIL>(g, fspec, nin, nout, oc, tw.t[0], s); break;
    }
    if (oc.red) {
        HookScope hs(K_REDUCE, 8.0 * blocks);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, blocks, oc.red, sp.red_out, nullptr);
    }
    if (nout > 0) {
        launch_x2<T, +1>(g, fspec, nout, tw.t[1], s);
        launch_c2r<T>(g, fspec, fout, nout, tw.t[2], s);
    }
}

// Destination half spectrum from the source one (both x1, x2, x3
// transformed): kept modes |k_a| < c_a scaled by `scale`, zero elsewhere.
template <typename T>
__global__ void k_mode_copy(int n1s, int n2s, int k3s, int n1d, int n2d, int k3d, int c1, int c2, int c3,
                            long long NSs, long long NSd, T factor, const cx<T> *__restrict__ src,
                            cx<T> *__restrict__ dst) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NSd) return;
    const int f = blockIdx.y;
    const int i3 = (int)(j % k3d), i2 = (int)((j / k3d) % n2d), i1 = (int)(j / ((long long)k3d * n2d));
    const int w1 = wavenumber(i1, n1d), w2 = wavenumber(i2, n2d), w3 = i3;
    cx<T> v = make_cx<T>(0, 0);
    if (abs(w1) < c1 && abs(w2) < c2 && w3 < c3) {
        const int s1 = w1 >= 0 ? w1 : w1 + n1s, s2 = w2 >= 0 ? w2 : w2 + n2s;
        v = scale(src[(long long)f * NSs + ((long long)s1 * n2s + s2) * k3s + w3], factor);
    }
    dst[(long long)f * NSd + j] = v;
}

// Full x1 transform of nf half spectra in place (a strided column pass).
template <typename T, int DIR>
static void launch_x1_fft(const Grid &g, FieldPtrs f, int nf, const cx<T> *tw, hipStream_t s) {
    const long long Q = (long long)g.n2 * g.k3;
    HookScope hs(DIR < 0 ? K_C2C_FWD : K_C2C_INV, (double)nf * sizeof(T) * 4.0 * g.NS);
#define MIREG_L(L)                                                                                          \
    {                                                                                                       \
        constexpr int NT = col_threads<T, L, 0>();                                                          \
        constexpr int W = FftShape<T, L, 0, NT>::W;                                                         \
        dim3 grid((unsigned)((Q + W - 1) / W), nf);                                                         \
        hipLaunchKernelGGL((k_c2c_cols<T, L, DIR>), grid, dim3(NT), 0, s, f, Q, Q, 0LL, Q, tw,            \
                           (const FieldPtrs *)nullptr);                                                     \
    }
    MIREG_SWITCH_COL(g.n1, MIREG_L)
#undef MIREG_L
}

template <typename T>
void spectral_resample(const Grid &gs, const Grid &gd, int nf, const T *const *in, T *const *out, cx<T> *spec_s,
                       cx<T> *spec_d, const Twiddles<T> &tws, const Twiddles<T> &twd, hipStream_t s) {
    FieldPtrs fin{}, fs{}, fd{}, fout{};
    for (int i = 0; i < nf; ++i) {
        fin.p[i] = const_cast<T *>(in[i]);
        fs.p[i] = spec_s + (long long)i * gs.NS;
        fd.p[i] = spec_d + (long long)i * gd.NS;
        fout.p[i] = out[i];
    }
    launch_r2c<T>(gs, fin, fs, nf, tws.t[2], s);
    launch_x2<T, -1>(gs, fs, nf, tws.t[1], s);
    launch_x1_fft<T, -1>(gs, fs, nf, tws.t[0], s);
    const int c1 = (gs.n1 < gd.n1 ? gs.n1 : gd.n1) / 2, c2 = (gs.n2 < gd.n2 ? gs.n2 : gd.n2) / 2,
              c3 = (gs.n3 < gd.n3 ? gs.n3 : gd.n3) / 2;
    const T scale = (T)(1.0 / ((double)gs.n1 * gs.n2 * gs.n3));
    {
        HookScope hs(K_VECTOR, (double)nf * 2.0 * sizeof(T) * 2 * gd.NS);
        dim3 grid((unsigned)((gd.NS + 255) / 256), nf);
        hipLaunchKernelGGL((k_mode_copy<T>), grid, dim3(256), 0, s, gs.n1, gs.n2, gs.k3, gd.n1, gd.n2, gd.k3, c1, c2, c3,
                           gs.NS, gd.NS, scale, spec_s, spec_d);
    }
    launch_x1_fft<T, +1>(gd, fd, nf, twd.t[0], s);
    launch_x2<T, +1>(gd, fd, nf, twd.t[1], s);
    launch_c2r<T>(gd, fd, fout, nf, twd.t[2], s);
}
template void spectral_resample<float>(const Grid &, const Grid &, int, const float *const *, float *const *,
                                       cx<float> *, cx<float> *, const Twiddles<float> &, const Twiddles<float> &,
                                       hipStream_t);
template void spectral_resample<double>(const Grid &, const Grid &, int, const double *const *, double *const *,
                                        cx<double> *, cx<double> *, const Twiddles<double> &,
                                        const Twiddles<double> &, hipStream_t);

// ---- Krylov host passes ----
template <typename T, int PASS, typename SA = T>
static void launch_x1_krylov(const Grid &g, const KrylovPtrs &f, const OpConst<T> &oc, T mu, int flags,
                             const cx<T> *tw, hipStream_t s, int *blocks, const KrylovPtrs *tab = nullptr,
                             int np = 1) {
    const long long Q = (long long)g.n2 * g.k3;
    // operands moved per launch (complex modes): FWD 3 + 3, HESS 3 + 3 + 3, DIR 3 + 3 + 3 + 3, INV 3 + 3;
    // KF_XUPD adds x read and written (DIR) or the old direction read (INV)
    const bool xupd = flags & KF_XUPD;
    const double fields = PASS == KP_HESS ? 6.0 + 3.0 * sizeof(SA) / sizeof(T)
                          : PASS == KP_DIR ? (xupd ? 18.0 : 12.0)
                                           : (PASS == KP_INV && xupd ? 9.0 : 6.0);
    HookScope hs(K_X1_KRYLOV, np * fields * 2.0 * sizeof(T) * g.NS);
#define MIREG_L(L)                                                                                       \
    {                                                                                                    \
        constexpr int NT = krylov_threads<T, L>();                                                       \
        constexpr int W = FftShape<T, L, 1, NT>::W;                                                      \
        dim3 grid((unsigned)((Q + W - 1) / W), PASS == KP_HESS ? 1 : 3, np);                             \
        if (blocks) *blocks = (int)grid.x;                                                               \
        if (tab)                                                                                         \
            hipLaunchKernelGGL((k_x1_krylov<T, L, PASS, SA, true>), grid, dim3(NT), 0, s, f, Q, oc, mu, flags, \
                               tw, tab);                                                                 \
        else                                                                                             \
            hipLaunchKernelGGL((k_x1_krylov<T, L, PASS, SA>), grid, dim3(NT), 0, s, f, Q, oc, mu, flags, tw, \
                               tab);                                                                     \
    }
    if constexpr (sizeof(T) == 4) {
        if (g.x1_narrow && g.n1 == 256 && !tab) {
            constexpr int NT = krylov_threads<T, 256, true>();
            constexpr int W = FftShape<T, 256, 1, NT>::W;
            dim3 grid((unsigned)((Q + W - 1) / W), PASS == KP_HESS ? 1 : 3, np);
            if (blocks) *blocks = (int)grid.x;
            hipLaunchKernelGGL((k_x1_krylov<T, 256, PASS, SA, false, true>), grid, dim3(NT), 0, s, f, Q, oc, mu,
                               flags, tw, tab);
            return;
        }
    }
    MIREG_SWITCH_COL(g.n1, MIREG_L)
#undef MIREG_L
}

template <typename T>
static OpConst<T> krylov_const(const Grid &g, const SpecParams &sp) {
    OpConst<T> oc{};
    oc.n1 = g.n1;
    oc.n2 = g.n2;
    oc.n3 = g.n3;
    oc.k3 = g.k3;
    oc.sym = SYM_AINV;
    oc.nf = 3;
    oc.reg = sp.reg;
    oc.div = sp.div;
    oc.alpha = (T)sp.beta_v;
    oc.beta_v = (T)sp.beta_v;
    oc.beta_w = (T)sp.beta_w;
    oc.norm = (T)(1.0 / ((double)g.n1 * g.n2 * g.n3));
    oc.red = nullptr;
    return oc;
}

template <typename T>
void krylov_forward(const Grid &g, const T *const *u, cx<T> *const *hat, cx<T> *work, const Twiddles<T> &tw,
                    hipStream_t s) {
    FieldPtrs fin{}, fw{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fin.p[a] = const_cast<T *>(u[a]);
        fw.p[a] = work + (long long)a * g.NS;
        kp.w[a] = fw.p[a];
        kp.o[a] = hat[a];
    }
    launch_r2c<T>(g, fin, fw, 3, tw.t[2], s);
    launch_x2<T, -1>(g, fw, 3, tw.t[1], s);
    SpecParams sp{};
    sp.reg = 1;
    launch_x1_krylov<T, KP_FWD>(g, kp, krylov_const<T>(g, sp), (T)0, 0, tw.t[0], s, nullptr);
}

template <typename T>
void krylov_hessian(const Grid &g, const T *const *b, const cx<T> *const *shat, cx<T> *const *hhat, cx<T> *work,
                    const Twiddles<T> &tw, const SpecParams &sp, int flags, hipStream_t s) {
    FieldPtrs fin{}, fw{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fin.p[a] = const_cast<T *>(b[a]);
        fw.p[a] = work + (long long)a * g.NS;
        kp.w[a] = fw.p[a];
        kp.a[a] = shat[a];
        kp.o[a] = hhat[a];
    }
    launch_r2c<T>(g, fin, fw, 3, tw.t[2], s);
    launch_x2<T, -1>(g, fw, 3, tw.t[1], s);
    OpConst<T> oc = krylov_const<T>(g, sp);
    oc.red = sp.red;
    int blocks = 0;
    launch_x1_krylov<T, KP_HESS>(g, kp, oc, (T)0, flags & KF_SQRT, tw.t[0], s, &blocks);
    if (oc.red) {
        HookScope hs(K_REDUCE, 8.0 * blocks);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, blocks, oc.red, sp.red_out, nullptr);
    }
}

void krylov_forward_wide(const Grid &g, const float *const *u, cx<double> *const *hat, cx<double> *work,
                         const Twiddles<double> &tw, hipStream_t s) {
    FieldPtrs fin{}, fw{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fin.p[a] = const_cast<float *>(u[a]);
        fw.p[a] = work + (long long)a * g.NS;
        kp.w[a] = fw.p[a];
        kp.o[a] = hat[a];
    }
    launch_r2c<double, float>(g, fin, fw, 3, tw.t[2], s);
    launch_x2<double, -1>(g, fw, 3, tw.t[1], s);
    SpecParams sp{};
    sp.reg = 1;
    launch_x1_krylov<double, KP_FWD>(g, kp, krylov_const<double>(g, sp), 0.0, 0, tw.t[0], s, nullptr);
}

void krylov_hessian_wide(const Grid &g, const float *const *b, const cx<double> *const *shat,
                         cx<float> *const *hhat, cx<float> *work, const Twiddles<float> &tw, const SpecParams &sp,
                         hipStream_t s) {
    FieldPtrs fin{}, fw{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fin.p[a] = const_cast<float *>(b[a]);
        fw.p[a] = work + (long long)a * g.NS;
        kp.w[a] = fw.p[a];
        kp.a[a] = shat[a];
        kp.o[a] = hhat[a];
    }
    launch_r2c<float>(g, fin, fw, 3, tw.t[2], s);
    launch_x2<float, -1>(g, fw, 3, tw.t[1], s);
    launch_x1_krylov<float, KP_HESS, double>(g, kp, krylov_const<float>(g, sp), 0.0f, 0, tw.t[0], s, nullptr);
}

template <typename T>
void krylov_direction(const Grid &g, const cx<T> *const *rhat, cx<T> *const *shat, double mu, int flags,
                      cx<T> *const *xhat, const double *alpha, T *const *s_out, cx<T> *work, const Twiddles<T> &tw,
                      const SpecParams &sp, hipStream_t s) {
    FieldPtrs fw{}, fout{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fw.p[a] = work + (long long)a * g.NS;
        fout.p[a] = s_out[a];
        kp.w[a] = fw.p[a];
        kp.a[a] = rhat[a];
        kp.o[a] = shat[a];
        kp.x[a] = xhat ? xhat[a] : nullptr;
    }
    kp.alpha = alpha;
    if (xhat && alpha && !(flags & KF_FIRST)) flags |= KF_XUPD;
    launch_x1_krylov<T, KP_DIR>(g, kp, krylov_const<T>(g, sp), (T)mu, flags, tw.t[0], s, nullptr);
    launch_x2<T, +1>(g, fw, 3, tw.t[1], s);
    launch_c2r<T>(g, fw, fout, 3, tw.t[2], s);
}

template <typename T>
void krylov_inverse(const Grid &g, const cx<T> *const *hat, const cx<T> *const *shat, const double *alpha,
                    T *const *u, cx<T> *work, const Twiddles<T> &tw, hipStream_t s) {
    FieldPtrs fw{}, fout{};
    KrylovPtrs kp{};
    for (int a = 0; a < 3; ++a) {
        fw.p[a] = work + (long long)a * g.NS;
        fout.p[a] = u[a];
        kp.w[a] = fw.p[a];
        kp.a[a] = hat[a];
        kp.o[a] = shat ? const_cast<cx<T> *>(shat[a]) : nullptr;
    }
    kp.alpha = alpha;
    SpecParams sp{};
    sp.reg = 1;
    launch_x1_krylov<T, KP_INV>(g, kp, krylov_const<T>(g, sp), (T)0, shat && alpha ? KF_XUPD : 0, tw.t[0], s,
                                nullptr);
    launch_x2<T, +1>(g, fw, 3, tw.t[1], s);
    launch_c2r<T>(g, fw, fout, 3, tw.t[2], s);
}

template <typename T>
void krylov_update(const Grid &g, bool update, int num, double *res, cx<T> *const *rhat, const cx<T> *const *hhat,
                   const SpecParams &sp, double *partials, hipStream_t s) {
    KrylovSet<T> v{};
    for (int a = 0; a < 3; ++a) {
        v.p[a] = rhat[a];
        v.p[3 + a] = const_cast<cx<T> *>(hhat[a]);
    }
    constexpr int nb = kRedBlocks;
    {
        HookScope hs(K_KRYLOV_UPDATE, (update ? 9.0 : 3.0) * 2.0 * sizeof(T) * g.NS);
        hipLaunchKernelGGL((k_krylov_update<T>), dim3(nb), dim3(256), 0, s, (unsigned)g.NS, g.n1, g.n2, g.n3, g.k3,
                           sp.reg, (T)sp.beta_v, update ? 1 : 0, num, res, v,
                           1.0 / ((double)g.n1 * g.n2 * g.n3), partials, (const KrylovUpd<T> *)nullptr);
    }
    HookScope hs(K_REDUCE, 16.0 * nb);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, nb, partials, res + 1, nullptr);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, nb, partials + nb, res + 2, nullptr);
}

// ---- the Krylov passes of several problems of one grid size ----
template <typename T>
bool krylov_hessian_multi(const Grid &g, int np, const T *const *b, const cx<T> *const *shat, cx<T> *const *hhat,
                          cx<T> *const *work, double *const *red, double *const *red_out, const Twiddles<T> &tw,
                          const SpecParams &sp, TabArena &ar, hipStream_t s) {
    const FieldPtrs *d_r2c, *d_x2;
    const KrylovPtrs *d_x1;
    const SumJob *d_sum;
    FieldPtrs *r2c = ar.alloc(2 * np, &d_r2c), *x2 = ar.alloc(np, &d_x2);
    KrylovPtrs *x1 = ar.alloc(np, &d_x1);
    SumJob *sum = ar.alloc(np, &d_sum);
    if (!r2c || !x2 || !x1 || !sum) return false;
    for (int p = 0; p < np; ++p) {
        r2c[2 * p] = FieldPtrs{};
        r2c[2 * p + 1] = FieldPtrs{};
        x1[p] = KrylovPtrs{};
        for (int a = 0; a < 3; ++a) {
            void *w = work[p] + (long long)a * g.NS;
            r2c[2 * p].p[a] = const_cast<T *>(b[3 * p + a]);
            r2c[2 * p + 1].p[a] = w;
            x1[p].w[a] = w;
            x1[p].a[a] = shat[3 * p + a];
            x1[p].o[a] = hhat[3 * p + a];
        }
        x2[p] = r2c[2 * p + 1];
        x1[p].red = red[p];
        sum[p] = SumJob{red[p], red_out[p]};
    }
    ar.upload(s);
    const FieldPtrs none{};
    launch_r2c<T>(g, none, none, 3, tw.t[2], s, d_r2c, np);
    launch_x2<T, -1>(g, none, 3, tw.t[1], s, d_x2, np);
    OpConst<T> oc = krylov_const<T>(g, sp);
    oc.red = red[0];  // the kernels take each problem's partials from the table
    int blocks = 0;
    launch_x1_krylov<T, KP_HESS>(g, KrylovPtrs{}, oc, (T)0, 0, tw.t[0], s, &blocks, d_x1, np);
    HookScope hs(K_REDUCE, 8.0 * blocks * np);
    hipLaunchKernelGGL(k_sum_partials, dim3(np), dim3(256), 0, s, blocks, nullptr, nullptr, d_sum);
    return true;
}

template <typename T>
bool krylov_update_multi(const Grid &g, int np, bool update, int num, double *const *res, cx<T> *const *rhat,
                         const cx<T> *const *hhat, double *const *partials, const SpecParams &sp, TabArena &ar,
                         hipStream_t s) {
    constexpr int nb = kRedBlocks;
    const KrylovUpd<T> *d_tab;
    const SumJob *d_sum;
    KrylovUpd<T> *tab = ar.alloc(np, &d_tab);
    SumJob *sum = ar.alloc(2 * np, &d_sum);
    if (!tab || !sum) return false;
    for (int p = 0; p < np; ++p) {
        for (int a = 0; a < 3; ++a) {
            tab[p].v.p[a] = rhat[3 * p + a];
            tab[p].v.p[3 + a] = const_cast<cx<T> *>(hhat[3 * p + a]);
        }
        for (int a = 6; a < 12; ++a) tab[p].v.p[a] = nullptr;
        tab[p].res = res[p];
        tab[p].part = partials[p];
        sum[2 * p] = SumJob{partials[p], res[p] + 1};
        sum[2 * p + 1] = SumJob{partials[p] + nb, res[p] + 2};
    }
    ar.upload(s);
    {
        HookScope hs(K_KRYLOV_UPDATE, (update ? 9.0 : 3.0) * 2.0 * sizeof(T) * g.NS * np);
        hipLaunchKernelGGL((k_krylov_update<T, true>), dim3(nb, np), dim3(256), 0, s, (unsigned)g.NS, g.n1, g.n2, g.n3,
                           g.k3, sp.reg, (T)sp.beta_v, update ? 1 : 0, num, nullptr, KrylovSet<T>{},
                           1.0 / ((double)g.n1 * g.n2 * g.n3), nullptr, d_tab);
    }
    HookScope hs(K_REDUCE, 16.0 * nb * np);
    hipLaunchKernelGGL(k_sum_partials, dim3(2 * np), dim3(256), 0, s, nb, nullptr, nullptr, d_sum);
    return true;
}

template <typename T>
bool krylov_direction_multi(const Grid &g, int np, const cx<T> *const *rhat, cx<T> *const *shat, const double *mu,
                            int flags, cx<T> *const *xhat, const double *const *alpha, T *const *s_out,
                            cx<T> *const *work, const Twiddles<T> &tw, const SpecParams &sp, TabArena &ar,
                            hipStream_t s) {
    const KrylovPtrs *d_x1;
    const FieldPtrs *d_x2, *d_c2r;
    KrylovPtrs *x1 = ar.alloc(np, &d_x1);
    FieldPtrs *x2 = ar.alloc(np, &d_x2), *c2r = ar.alloc(2 * np, &d_c2r);
    if (!x1 || !x2 || !c2r) return false;
    const bool xupd = xhat && alpha && !(flags & KF_FIRST);
    if (xupd) flags |= KF_XUPD;
    for (int p = 0; p < np; ++p) {
        x1[p] = KrylovPtrs{};
        x2[p] = FieldPtrs{};
        c2r[2 * p + 1] = FieldPtrs{};
        for (int a = 0; a < 3; ++a) {
            void *w = work[p] + (long long)a * g.NS;
            x1[p].w[a] = w;
            x1[p].a[a] = rhat[3 * p + a];
            x1[p].o[a] = shat[3 * p + a];
            x1[p].x[a] = xhat ? xhat[3 * p + a] : nullptr;
            x2[p].p[a] = w;
            c2r[2 * p + 1].p[a] = s_out[3 * p + a];
        }
        c2r[2 * p] = x2[p];
        x1[p].alpha = alpha ? alpha[p] : nullptr;
        x1[p].mu = mu ? mu[p] : 0.0;
    }
    ar.upload(s);
    const FieldPtrs none{};
    launch_x1_krylov<T, KP_DIR>(g, KrylovPtrs{}, krylov_const<T>(g, sp), (T)0, flags, tw.t[0], s, nullptr, d_x1, np);
    launch_x2<T, +1>(g, none, 3, tw.t[1], s, d_x2, np);
    launch_c2r<T>(g, none, none, 3, tw.t[2], s, d_c2r, np);
    return true;
}

// ---- Two-level preconditioner on Krylov spectra (fine grid n, coarse n/2) ----
// Mode (w1, w2, w3) of a half spectrum [n1][n2][n3/2+1] at linear index j.
__device__ __forceinline__ void half_mode(unsigned j, int n1, int n2, int k3, int &w1, int &w2, int &w3) {
    const unsigned i3 = j % (unsigned)k3, row = j / (unsigned)k3;
    w1 = wavenumber((int)(row / (unsigned)n2), n1);
    w2 = wavenumber((int)(row % (unsigned)n2), n2);
    w3 = (int)i3;
}
template <typename T>
__device__ __forceinline__ void tl_symbols(int w1, int w2, int w3, int reg, T beta_v, T &sigma, T &c) {
    const T ks = (T)w1 * (T)w1 + (T)w2 * (T)w2 + (T)w3 * (T)w3;
    const T a = reg == 2 ? ks * ks : ks;
    sigma = ks == (T)0 ? (T)1 : (T)1 / (beta_v * a);
    c = ks == (T)0 ? (T)1 : (T)1 / sqrt(beta_v * a);
}

// Coarse right-hand side of the nested CG: rc = pc = Q_R c r for every coarse
// mode, i.e. (Nc/Nf) c(k) rf(k) on the modes below the coarse Nyquist, 0 on
// the coarse Nyquist planes.  Component blockIdx.y.
template <typename T>
__global__ __launch_bounds__(256) void k_tl_restrict(int n1f, int n2f, int k3f, int n1c, int n2c, int n3c, int k3c,
                                                     unsigned NSc, int reg, T beta_v, T factor, KrylovSet<T> v) {
    const unsigned j = blockIdx.x * 256u + threadIdx.x;
    if (j >= NSc) return;
    const int a = blockIdx.y;
    int w1, w2, w3;
    half_mode(j, n1c, n2c, k3c, w1, w2, w3);
    cx<T> val = make_cx<T>(0, 0);
    if (2 * abs(w1) < n1c && 2 * abs(w2) < n2c && 2 * w3 < n3c) {
        T sigma, c;
        tl_symbols<T>(w1, w2, w3, reg, beta_v, sigma, c);
        const int s1 = w1 >= 0 ? w1 : w1 + n1f, s2 = w2 >= 0 ? w2 : w2 + n2f;
        val = scale(v.p[a][((long long)s1 * n2f + s2) * k3f + w3], factor * c);
    }
    v.p[3 + a][j] = val;
    v.p[6 + a][j] = val;
}

// Fine preconditioned residual z = c (F_H c r + Q_P u): on the modes below
// n_a/4 on every axis c(k) (Nf/Nc) u(k), elsewhere sigma(k) r(k); partials
// of sum_x r . z (part[b], fixed grid of kRedBlocks workgroups).  u is
// u + alpha p (the nested CG's last update, pending) when palpha is given.
template <typename T>
__global__ __launch_bounds__(256) void k_tl_combine(int n1f, int n2f, int n3f, int k3f, int n2c, int k3c, unsigned NSf,
                                                    int reg, T beta_v, T factor, const double *palpha,
                                                    double norm, KrylovSet<T> v, double *__restrict__ part) {
    cx<T> *const *rf = v.p, *const *uc = v.p + 3, *const *zf = v.p + 6;
    const cx<T> *const *pc = v.p + 9;
    const T alpha = palpha ? (T)*palpha : (T)0;
    const int n1c = n1f / 2;
    double acc = 0;
    for (unsigned j = blockIdx.x * 256u + threadIdx.x; j < NSf; j += gridDim.x * 256u) {
        int w1, w2, w3;
        half_mode(j, n1f, n2f, k3f, w1, w2, w3);
        T sigma, c;
        tl_symbols<T>(w1, w2, w3, reg, beta_v, sigma, c);
        const bool low = 4 * abs(w1) < n1f && 4 * abs(w2) < n2f && 4 * w3 < n3f;
        const long long jc = low ? ((long long)(w1 >= 0 ? w1 : w1 + n1c) * n2c + (w2 >= 0 ? w2 : w2 + n2c)) * k3c + w3 : 0;
        const double wk3 = (w3 == 0 || 2 * w3 == n3f) ? 1.0 : 2.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<T> r = rf[a][j];
            cx<T> u = low ? uc[a][jc] : make_cx<T>(0, 0);
            if (low && alpha != (T)0) u = u + scale(pc[a][jc], alpha);
            const cx<T> z = low ? scale(u, factor * c) : scale(r, sigma);
            zf[a][j] = z;
            acc += wk3 * ((double)r.re * (double)z.re + (double)r.im * (double)z.im);
        }
    }
    __shared__ double sh[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) * norm;
}

template <typename T>
void twolevel_restrict(const Grid &gf, const Grid &gc, const cx<T> *const *rf, cx<T> *const *rc, cx<T> *const *pc,
                       const SpecParams &sp, hipStream_t s) {
    KrylovSet<T> v{};
    for (int a = 0; a < 3; ++a) {
        v.p[a] = const_cast<cx<T> *>(rf[a]);
        v.p[3 + a] = rc[a];
        v.p[6 + a] = pc[a];
    }
    HookScope hs(K_VECTOR, 9.0 * sizeof(cx<T>) * gc.NS);
    const T factor = (T)((double)gc.N / (double)gf.N);
    dim3 grid((unsigned)((gc.NS + 255) / 256), 3);
    hipLaunchKernelGGL((k_tl_restrict<T>), grid, dim3(256), 0, s, gf.n1, gf.n2, gf.k3, gc.n1, gc.n2, gc.n3, gc.k3,
                       (unsigned)gc.NS, sp.reg, (T)sp.beta_v, factor, v);
}

template <typename T>
void twolevel_combine(const Grid &gf, const Grid &gc, const cx<T> *const *rf, const cx<T> *const *uc,
                      const cx<T> *const *pc, const double *alpha, cx<T> *const *zf, const SpecParams &sp,
                      double *partials, double *out, hipStream_t s) {
    KrylovSet<T> v{};
    for (int a = 0; a < 3; ++a) {
        v.p[a] = const_cast<cx<T> *>(rf[a]);
        v.p[3 + a] = const_cast<cx<T> *>(uc[a]);
        v.p[6 + a] = zf[a];
        v.p[9 + a] = const_cast<cx<T> *>(pc[a]);
    }
    const T factor = (T)((double)gf.N / (double)gc.N);
    {
        HookScope hs(K_VECTOR, 6.0 * sizeof(cx<T>) * gf.NS);
        hipLaunchKernelGGL((k_tl_combine<T>), dim3(kRedBlocks), dim3(256), 0, s, gf.n1, gf.n2, gf.n3, gf.k3, gc.n2,
                           gc.k3, (unsigned)gf.NS, sp.reg, (T)sp.beta_v, factor, alpha, 1.0 / (double)gf.N, v,
                           partials);
    }
    HookScope hs(K_REDUCE, 8.0 * kRedBlocks);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, kRedBlocks, partials, out, nullptr);
}

#define MIREG_KRYLOV(T)                                                                                          \
    template void krylov_forward<T>(const Grid &, const T *const *, cx<T> *const *, cx<T> *, const Twiddles<T> &, \
                                    hipStream_t);                                                                \
    template void krylov_hessian<T>(const Grid &, const T *const *, const cx<T> *const *, cx<T> *const *,         \
                                    cx<T> *, const Twiddles<T> &, const SpecParams &, int, hipStream_t);         \
    template void krylov_direction<T>(const Grid &, const cx<T> *const *, cx<T> *const *, double, int,           \
                                      cx<T> *const *, const double *, T *const *, cx<T> *, const Twiddles<T> &,  \
                                      const SpecParams &, hipStream_t);                                          \
    template void twolevel_restrict<T>(const Grid &, const Grid &, const cx<T> *const *, cx<T> *const *,          \
                                       cx<T> *const *, const SpecParams &, hipStream_t);                          \
    template void twolevel_combine<T>(const Grid &, const Grid &, const cx<T> *const *, const cx<T> *const *,     \
                                      const cx<T> *const *, const double *, cx<T> *const *, const SpecParams &,   \
                                      double *, double *, hipStream_t);                                          \
    template void krylov_inverse<T>(const Grid &, const cx<T> *const *, const cx<T> *const *, const double *,     \
                                    T *const *, cx<T> *, const Twiddles<T> &, hipStream_t);                      \
    template void krylov_update<T>(const Grid &, bool, int, double *, cx<T> *const *, const cx<T> *const *,      \
                                   const SpecParams &, double *, hipStream_t);                                  \
    template bool krylov_hessian_multi<T>(const Grid &, int, const T *const *, const cx<T> *const *,              \
                                          cx<T> *const *, cx<T> *const *, double *const *, double *const *,       \
                                          const Twiddles<T> &, const SpecParams &, TabArena &, hipStream_t);      \
    template bool krylov_update_multi<T>(const Grid &, int, bool, int, double *const *, cx<T> *const *,            \
                                         const cx<T> *const *, double *const *, const SpecParams &, TabArena &,   \
                                         hipStream_t);                                                            \
    template bool krylov_direction_multi<T>(const Grid &, int, const cx<T> *const *, cx<T> *const *,               \
                                            const double *, int, cx<T> *const *, const double *const *,            \
                                            T *const *, cx<T> *const *, const Twiddles<T> &, const SpecParams &,   \
                                            TabArena &, hipStream_t);
MIREG_KRYLOV(float)
MIREG_KRYLOV(double)
#undef MIREG_KRYLOV

template void spectral_apply<float>(const Grid &, int, int, int, const void *const *, float *const *,
                                    cx<float> *, const Twiddles<float> &, const SpecParams &,
                                    hipStream_t);
template void spectral_apply<double>(const Grid &, int, int, int, const void *const *,
                                     double *const *, cx<double> *, const Twiddles<double> &,
                                     const SpecParams &, hipStream_t);

}  // namespace mireg
