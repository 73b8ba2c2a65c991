// Semi-Lagrangian transport kernels (Sec. 2.3.1, Sec. 3.4) for gfx950.
//
// Every kernel is one sweep over the grid, one thread per point, 256
// consecutive points of an x3 line per workgroup.  Off-grid values are
// gathered with third-degree Lagrange polynomials on a 4x4x4 stencil (or
// trilinear on 2x2x2), periodic wrap by masking (power-of-two sizes).
// Departure points are stored as displacements in cell units, so the local
// coordinate t = d - floor(d) keeps full precision in FP32 far from the
// origin.  The time integrals of the gradient and the Hessian matvec are
// accumulated inside the adjoint steps (Sec. 3.5, memory-reduced
// Gauss-Newton), so only the state history is stored.
#include "kernels.hpp"

namespace mireg {

struct PGrid {
    int n1, n2, n3;
    int s3, s23;  // log2(n3), log2(n2 n3)
    long long N;
};

static PGrid pgrid(const Grid &g) {
    PGrid p;
    p.n1 = g.n1;
    p.n2 = g.n2;
    p.n3 = g.n3;
    p.s3 = __builtin_ctz((unsigned)g.n3);
    p.s23 = p.s3 + __builtin_ctz((unsigned)g.n2);
    p.N = g.N;
    return p;
}

template <typename T, int ORDER>
struct Stencil {
    static constexpr int NP = ORDER == 3 ? 4 : 2;
    int o1[NP], o2[NP], o3[NP];  // offsets i1 n2 n3, i2 n3, i3 of the nodes
    T w1[NP], w2[NP], w3[NP];
};

template <typename T, int ORDER>
using NodeIdx = int[Stencil<T, ORDER>::NP];
template <typename T, int ORDER>
using NodeW = T[Stencil<T, ORDER>::NP];

template <typename T, int ORDER>
__device__ __forceinline__ void axis_nodes(int i, T d, int n, int mult, NodeIdx<T, ORDER> &o,
                                           NodeW<T, ORDER> &w) {
    const T fl = floor(d);
    const T t = d - fl;
    const int base = i + (int)fl;
    if constexpr (ORDER == 3) {
        // cubic Lagrange basis on the nodes -1, 0, 1, 2
        const T tm1 = t - (T)1, tm2 = t - (T)2, tp1 = t + (T)1;
        w[0] = -t * tm1 * tm2 * (T)(1.0 / 6.0);
        w[1] = tp1 * tm1 * tm2 * (T)0.5;
        w[2] = -tp1 * t * tm2 * (T)0.5;
        w[3] = tp1 * t * tm1 * (T)(1.0 / 6.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = ((base - 1 + k) & (n - 1)) * mult;
    } else {
        w[0] = (T)1 - t;
        w[1] = t;
#pragma unroll
        for (int k = 0; k < 2; ++k) o[k] = ((base + k) & (n - 1)) * mult;
    }
}

template <typename T, int ORDER>
__device__ __forceinline__ Stencil<T, ORDER> make_stencil(const PGrid &g, int i1, int i2, int i3, T d1,
                                                          T d2, T d3) {
    Stencil<T, ORDER> st;
    axis_nodes<T, ORDER>(i1, d1, g.n1, g.n2 * g.n3, st.o1, st.w1);
    axis_nodes<T, ORDER>(i2, d2, g.n2, g.n3, st.o2, st.w2);
    axis_nodes<T, ORDER>(i3, d3, g.n3, 1, st.o3, st.w3);
    return st;
}

template <typename T, int ORDER>
__device__ __forceinline__ T gather(const T *__restrict__ f, const Stencil<T, ORDER> &st) {
    constexpr int NP = Stencil<T, ORDER>::NP;
    T acc = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T ap = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const T *row = f + st.o1[p] + st.o2[q];
            T s = 0;
#pragma unroll
            for (int r = 0; r < NP; ++r) s += st.w3[r] * row[st.o3[r]];
            ap += st.w2[q] * s;
        }
        acc += st.w1[p] * ap;
    }
    return acc;
}

// I[f](y) and I[f d](y) from one stencil (the product is formed per node).
template <typename T, int ORDER>
__device__ __forceinline__ void gather_pair(const T *__restrict__ f, const T *__restrict__ d,
                                            const Stencil<T, ORDER> &st, T &If, T &Ifd) {
    constexpr int NP = Stencil<T, ORDER>::NP;
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T b0 = 0, b1 = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int row = st.o1[p] + st.o2[q];
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                const T fv = f[row + st.o3[r]];
                const T dv = d[row + st.o3[r]];
                s0 += st.w3[r] * fv;
                s1 += st.w3[r] * (fv * dv);
            }
            b0 += st.w2[q] * s0;
            b1 += st.w2[q] * s1;
        }
        a0 += st.w1[p] * b0;
        a1 += st.w1[p] * b1;
    }
    If = a0;
    Ifd = a1;
}

__device__ __forceinline__ void point_index(const PGrid &g, long long idx, int &i1, int &i2, int &i3) {
    i3 = (int)(idx & (g.n3 - 1));
    i2 = (int)((idx >> g.s3) & (g.n2 - 1));
    i1 = (int)(idx >> g.s23);
}

constexpr int kPtThreads = 256;

// ---------------------------------------------------------------------------
template <typename T, int ORDER>
__global__ __launch_bounds__(kPtThreads) void k_departure(PGrid g, T sdt, T ih1, T ih2, T ih3,
                                                          const T *__restrict__ v,
                                                          T *__restrict__ disp) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= g.N) return;
    int i1, i2, i3;
    point_index(g, idx, i1, i2, i3);
    const T v1 = v[idx], v2 = v[g.N + idx], v3 = v[2 * g.N + idx];
    // predictor x + sign dt v(x), in cells
    const Stencil<T, ORDER> st = make_stencil<T, ORDER>(g, i1, i2, i3, sdt * v1 * ih1, sdt * v2 * ih2,
                                                        sdt * v3 * ih3);
    const T p1 = gather<T, ORDER>(v, st);
    const T p2 = gather<T, ORDER>(v + g.N, st);
    const T p3 = gather<T, ORDER>(v + 2 * g.N, st);
    const T h = (T)0.5 * sdt;
    disp[idx] = h * (v1 + p1) * ih1;
    disp[g.N + idx] = h * (v2 + p2) * ih2;
    disp[2 * g.N + idx] = h * (v3 + p3) * ih3;
}

template <typename T, int ORDER>
__global__ __launch_bounds__(kPtThreads) void k_interp(PGrid g, const T *__restrict__ f,
                                                       const T *__restrict__ disp, T *__restrict__ out) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= g.N) return;
    int i1, i2, i3;
    point_index(g, idx, i1, i2, i3);
    const Stencil<T, ORDER> st =
        make_stencil<T, ORDER>(g, i1, i2, i3, disp[idx], disp[g.N + idx], disp[2 * g.N + idx]);
    out[idx] = gather<T, ORDER>(f, st);
}

template <typename T>
__global__ __launch_bounds__(kPtThreads) void k_adjoint_init(long long N, T a_nt, const T *__restrict__ mR,
                                                             const T *__restrict__ m,
                                                             const T *__restrict__ gm, T *__restrict__ lam,
                                                             T *__restrict__ b) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= N) return;
    const T l = mR[idx] - m[idx];  // final condition lambda(1) = mR - m(1)
    lam[idx] = l;
    const T al = a_nt * l;
    b[idx] = al * gm[idx];
    b[N + idx] = al * gm[N + idx];
    b[2 * N + idx] = al * gm[2 * N + idx];
}

// lambda^j = L + dt/2 (S + (L + dt S) d), L = I[lambda^{j+1}](Y), S = I[lambda^{j+1} d](Y)
template <typename T, int ORDER>
__global__ __launch_bounds__(kPtThreads) void k_adjoint_step(PGrid g, T dt, T aj, const T *__restrict__ lin,
                                                             const T *__restrict__ d,
                                                             const T *__restrict__ Y,
                                                             const T *__restrict__ gm,
                                                             T *__restrict__ lout, T *__restrict__ b) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= g.N) return;
    int i1, i2, i3;
    point_index(g, idx, i1, i2, i3);
    const Stencil<T, ORDER> st =
        make_stencil<T, ORDER>(g, i1, i2, i3, Y[idx], Y[g.N + idx], Y[2 * g.N + idx]);
    T L, S;
    gather_pair<T, ORDER>(lin, d, st, L, S);
    const T lam = L + (T)0.5 * dt * (S + (L + dt * S) * d[idx]);
    if (lout) lout[idx] = lam;
    const T al = aj * lam;
    b[idx] += al * gm[idx];
    b[g.N + idx] += al * gm[g.N + idx];
    b[2 * g.N + idx] += al * gm[2 * g.N + idx];
}

template <typename T>
__global__ __launch_bounds__(kPtThreads) void k_incstate_init(long long N, T hdt, const T *__restrict__ gm,
                                                              const T *__restrict__ vt, T *__restrict__ q) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= N) return;
    const T f = -(gm[idx] * vt[idx] + gm[N + idx] * vt[N + idx] + gm[2 * N + idx] * vt[2 * N + idx]);
    q[idx] = hdt * f;
}

template <typename T, int ORDER>
__global__ __launch_bounds__(kPtThreads) void k_incstate_step(PGrid g, T coef, const T *__restrict__ qin,
                                                              const T *__restrict__ X,
                                                              const T *__restrict__ gm,
                                                              const T *__restrict__ vt,
                                                              T *__restrict__ qout, T a_nt,
                                                              T *__restrict__ lt, T *__restrict__ b) {
    const long long idx = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    if (idx >= g.N) return;
    int i1, i2, i3;
    point_index(g, idx, i1, i2, i3);
    const Stencil<T, ORDER> st =
        make_stencil<T, ORDER>(g, i1, i2, i3, X[idx], X[g.N + idx], X[2 * g.N + idx]);
    const T Iq = gather<T, ORDER>(qin, st);
    const long long N = g.N;
    const T g1 = gm[idx], g2 = gm[N + idx], g3 = gm[2 * N + idx];
    const T f = -(g1 * vt[idx] + g2 * vt[N + idx] + g3 * vt[2 * N + idx]);
    if (lt == nullptr) {
        qout[idx] = Iq + coef * f;
    } else {
        // last step: mt(1) = I[q](X) + dt/2 f^nt; incremental adjoint starts at -mt(1)
        const T l = -(Iq + coef * f);
        lt[idx] = l;
        const T al = a_nt * l;
        b[idx] = al * g1;
        b[N + idx] = al * g2;
        b[2 * N + idx] = al * g3;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + kPtThreads - 1) / kPtThreads); }

template <typename T>
void departure(const Grid &gg, int order, int sign, double dt, const T *v, T *disp, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_DEPARTURE, 6.0 * g.N * sizeof(T));
    const double two_pi = 6.283185307179586476925;
    const T sdt = (T)(sign * dt);
    const T ih1 = (T)(g.n1 / two_pi), ih2 = (T)(g.n2 / two_pi), ih3 = (T)(g.n3 / two_pi);
    if (order == 3)
        hipLaunchKernelGGL((k_departure<T, 3>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, sdt, ih1,
                           ih2, ih3, v, disp);
    else
        hipLaunchKernelGGL((k_departure<T, 1>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, sdt, ih1,
                           ih2, ih3, v, disp);
}

template <typename T>
void interp_field(const Grid &gg, int order, const T *f, const T *disp, T *out, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INTERP, 5.0 * g.N * sizeof(T));
    if (order == 3)
        hipLaunchKernelGGL((k_interp<T, 3>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, f, disp, out);
    else
        hipLaunchKernelGGL((k_interp<T, 1>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, f, disp, out);
}

template <typename T>
void adjoint_init(const Grid &g, double a_nt, const T *mR, const T *m, const T *gradm, T *lam, T *b,
                  hipStream_t s) {
    HookScope hs(K_ADJ_INIT, 9.0 * g.N * sizeof(T));
    hipLaunchKernelGGL((k_adjoint_init<T>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g.N, (T)a_nt, mR,
                       m, gradm, lam, b);
}

template <typename T>
void adjoint_step(const Grid &gg, int order, double dt, double aj, const T *lam_in, const T *d,
                  const T *Y, const T *gradm_j, T *lam_out, T *b, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_ADJ_STEP, (lam_out ? 15.0 : 14.0) * g.N * sizeof(T));
    if (order == 3)
        hipLaunchKernelGGL((k_adjoint_step<T, 3>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, (T)dt,
                           (T)aj, lam_in, d, Y, gradm_j, lam_out, b);
    else
        hipLaunchKernelGGL((k_adjoint_step<T, 1>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, (T)dt,
                           (T)aj, lam_in, d, Y, gradm_j, lam_out, b);
}

template <typename T>
void incstate_init(const Grid &g, double dt, const T *gradm0, const T *vt, T *q, hipStream_t s) {
    HookScope hs(K_INC_INIT, 7.0 * g.N * sizeof(T));
    hipLaunchKernelGGL((k_incstate_init<T>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g.N,
                       (T)(0.5 * dt), gradm0, vt, q);
}

template <typename T>
void incstate_step(const Grid &gg, int order, double coef, const T *q_in, const T *X, const T *gradm_next,
                   const T *vt, T *q_out, double a_nt, T *lt_out, T *b_out, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INC_STEP, (lt_out ? 14.0 : 11.0) * g.N * sizeof(T));
    if (order == 3)
        hipLaunchKernelGGL((k_incstate_step<T, 3>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, (T)coef,
                           q_in, X, gradm_next, vt, q_out, (T)a_nt, lt_out, b_out);
    else
        hipLaunchKernelGGL((k_incstate_step<T, 1>), dim3(blocks_for(g.N)), dim3(kPtThreads), 0, s, g, (T)coef,
                           q_in, X, gradm_next, vt, q_out, (T)a_nt, lt_out, b_out);
}

#define MIREG_INST(T)                                                                                   \
    template void departure<T>(const Grid &, int, int, double, const T *, T *, hipStream_t);            \
    template void interp_field<T>(const Grid &, int, const T *, const T *, T *, hipStream_t);           \
    template void adjoint_init<T>(const Grid &, double, const T *, const T *, const T *, T *, T *,      \
                                  hipStream_t);                                                         \
    template void adjoint_step<T>(const Grid &, int, double, double, const T *, const T *, const T *,   \
                                  const T *, T *, T *, hipStream_t);                                    \
    template void incstate_init<T>(const Grid &, double, const T *, const T *, T *, hipStream_t);      \
    template void incstate_step<T>(const Grid &, int, double, const T *, const T *, const T *,          \
                                   const T *, T *, double, T *, T *, hipStream_t);
MIREG_INST(float)
MIREG_INST(double)
#undef MIREG_INST

}  // namespace mireg
