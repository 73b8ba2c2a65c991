// Semi-Lagrangian transport kernels (Sec. 2.3.1, Sec. 3.4) for gfx950.
//
// Off-grid values are third-degree Lagrange polynomials on a 4x4x4 stencil
// (trilinear on 2x2x2), periodic on power-of-two grids.  Departure points are
// stored as displacements in cell units, so t = d - floor(d) keeps full
// precision in FP32 anywhere on the grid.
//
// Every step is one kernel over tiles of points (16 x3 x 8 x2 x 8 x1 by
// default; 32 x 8 x 4 and 16 x 16 x 8 selectable), 256 threads:
//   1. each thread reads the displacement of its points (coalesced rows of
//      along x3) and the block reduces the bounding box of all stencils;
//   2. if the box fits the LDS budget, the block copies the box of the
//      gathered field(s) from HBM/L2 into LDS once (rows along x3, periodic
//      wrap applied here) and every 64-node stencil is read from LDS;
//      otherwise the tile gathers straight from global memory;
//   3. each point finishes its step (sources, time quadrature) and writes.
// Tiles are assigned XCD by XCD, so neighbouring tiles -- whose boxes
// overlap -- are served by the same L2.
// The adjoint sweeps store the adjoint history; the time integrals of the
// gradient and the Hessian matvec are then formed in one streaming pass
// (Sec. 3.5: only time histories are kept, no full space-time Newton).
#include <limits.h>

#include "kernels.hpp"

namespace mireg {

struct PGrid {
    int n1, n2, n3;
    int s3, s23;  // log2(n3), log2(n2 n3)
    long long N;
    int tx, ty, tz;  // tiles per axis
    int lds_cap;     // largest box (points) staged in LDS; 0 disables staging
    int shape;       // tile shape (SlTile)
};

// Tile shapes (x1 x x2 x x3 points) of the semi-Lagrangian kernels.
enum SlTile { TILE_4x8x32 = 0, TILE_8x8x16 = 1, TILE_8x16x16 = 2 };
template <int S>
struct TileDims;
template <>
struct TileDims<TILE_4x8x32> {
    static constexpr int TZ = 4, TY = 8, TX = 32;
};
template <>
struct TileDims<TILE_8x8x16> {
    static constexpr int TZ = 8, TY = 8, TX = 16;
};
template <>
struct TileDims<TILE_8x16x16> {
    static constexpr int TZ = 8, TY = 16, TX = 16;
};

constexpr int kSlThreads = 256;
constexpr int kBoxCap = 6144;                       // LDS box capacity in points
constexpr int kStageU = 8;                          // staging loads in flight per thread

// Box capacity of one instantiation: at most 64 KB of LDS per workgroup.
template <typename T, int NF>
constexpr int box_cap() {
    return (int)(65536 / (NF * sizeof(T))) < kBoxCap ? (int)(65536 / (NF * sizeof(T))) : kBoxCap;
}

static PGrid pgrid(const Grid &g) {
    PGrid p;
    p.n1 = g.n1;
    p.n2 = g.n2;
    p.n3 = g.n3;
    p.s3 = __builtin_ctz((unsigned)g.n3);
    p.s23 = p.s3 + __builtin_ctz((unsigned)g.n2);
    p.N = g.N;
    p.shape = g.sl_tile;
    const int TZ = p.shape == TILE_4x8x32 ? 4 : 8, TY = p.shape == TILE_8x16x16 ? 16 : 8,
              TX = p.shape == TILE_4x8x32 ? 32 : 16;
    p.tx = (g.n3 + TX - 1) / TX;
    p.ty = (g.n2 + TY - 1) / TY;
    p.tz = (g.n1 + TZ - 1) / TZ;
    p.lds_cap = g.lds_cap < kBoxCap ? g.lds_cap : kBoxCap;
    return p;
}

// Node weights of one axis and the node below the position.
template <typename T, int ORDER>
struct AxisW {
    static constexpr int NP = ORDER == 3 ? 4 : 2;
    static constexpr int FIRST = ORDER == 3 ? -1 : 0;
    int base;  // i + floor(d)
    T w[NP];
};

template <typename T, int ORDER>
__device__ __forceinline__ AxisW<T, ORDER> axis_weights(int i, T d) {
    AxisW<T, ORDER> a;
    const T fl = floor(d);
    const T t = d - fl;
    a.base = i + (int)fl;
    if constexpr (ORDER == 3) {
        // cubic Lagrange basis on the nodes -1, 0, 1, 2
        const T tm1 = t - (T)1, tm2 = t - (T)2, tp1 = t + (T)1;
        a.w[0] = -t * tm1 * tm2 * (T)(1.0 / 6.0);
        a.w[1] = tp1 * tm1 * tm2 * (T)0.5;
        a.w[2] = -tp1 * t * tm2 * (T)0.5;
        a.w[3] = tp1 * t * tm1 * (T)(1.0 / 6.0);
    } else {
        a.w[0] = (T)1 - t;
        a.w[1] = t;
    }
    return a;
}

template <int NP>
using NodeOff = int[NP];

// Tensor-product contraction of NF quantities; get(offset, v) reads the NF
// values at the combined node offset o1[p] + o2[q] + o3[r].
template <typename T, int ORDER, int NF, class Get>
__device__ __forceinline__ void contract(const AxisW<T, ORDER> &a1, const AxisW<T, ORDER> &a2,
                                         const AxisW<T, ORDER> &a3, const NodeOff<AxisW<T, ORDER>::NP> &o1,
                                         const NodeOff<AxisW<T, ORDER>::NP> &o2,
                                         const NodeOff<AxisW<T, ORDER>::NP> &o3, const Get &get, T *acc) {
    constexpr int NP = AxisW<T, ORDER>::NP;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T ap[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) ap[f] = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int row = o1[p] + o2[q];
            T s[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) s[f] = 0;
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                T v[NF];
                get(row + o3[r], v);
#pragma unroll
                for (int f = 0; f < NF; ++f) s[f] += a3.w[r] * v[f];
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) ap[f] += a2.w[q] * s[f];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] += a1.w[p] * ap[f];
    }
}

// Same contraction over an unwrapped box: node (p, q, r) at
// base + p s1 + q s2 + r, so the r taps of a row use immediate offsets.  All
// taps of a plane p are read before any arithmetic, so a wave keeps 16
// (NF = 1) or 32 (NF = 2) LDS words in flight instead of waiting row by row.
template <typename T, int ORDER, int NF, class Get>
__device__ __forceinline__ void contract_box(const AxisW<T, ORDER> &a1, const AxisW<T, ORDER> &a2,
                                             const AxisW<T, ORDER> &a3, int base, int s1, int s2,
                                             const Get &get, T *acc) {
    constexpr int NP = AxisW<T, ORDER>::NP;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T v[NP][NP][NF];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int row = base + p * s1 + q * s2;
#pragma unroll
            for (int r = 0; r < NP; ++r) get(row, r, v[q][r]);
        }
        T ap[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) ap[f] = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            T sr[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) sr[f] = 0;
#pragma unroll
            for (int r = 0; r < NP; ++r) {
#pragma unroll
                for (int f = 0; f < NF; ++f) sr[f] += a3.w[r] * v[q][r][f];
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) ap[f] += a2.w[q] * sr[f];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] += a1.w[p] * ap[f];
    }
}

// LDS layout of the staged box: NF <= 2 interleaved (the NF values of a node
// are adjacent, one 4/8/16-byte read), NF = 3 one array per quantity.
template <int NF>
struct BoxLayout {
    static constexpr bool AOS = NF <= 2;
    template <int CAP>
    static __device__ __forceinline__ int at(int k, int f) {
        return AOS ? k * NF + f : f * CAP + k;
    }
};

// Workgroup index -> tile index, contiguous runs of tiles per XCD (workgroups
// are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int x = bid % 8, j = bid / 8;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Generic tiled semi-Lagrangian sweep.  Op provides:
//   void disp(int idx, T *d)            displacement of point idx (cells, 3 values)
//   void stage(int gidx, T *v)          the NF gathered quantities at grid index gidx
//   Pre pre(int idx)                    operands of the point update, loaded early
//   void finish(int idx, const Pre &, const T *acc)  output of point idx
template <typename T, int ORDER, int NF, int SHAPE, class Op>
__global__ __launch_bounds__(kSlThreads) void k_sl(PGrid g, Op op) {
    constexpr int kTZ = TileDims<SHAPE>::TZ, kTY = TileDims<SHAPE>::TY, kTX = TileDims<SHAPE>::TX;
    constexpr int kPPT = kTX * kTY * kTZ / kSlThreads;  // points per thread
    using A = AxisW<T, ORDER>;
    constexpr int NP = A::NP, FIRST = A::FIRST;
    constexpr int CAP = box_cap<T, NF>();
    __shared__ __align__(16) T lds[NF * CAP];
    __shared__ int box[6];
    const int nb = g.tx * g.ty * g.tz;
    const int tile = xcd_tile(blockIdx.x, nb);
    const int bx = tile % g.tx, by = (tile / g.tx) % g.ty, bz = tile / (g.tx * g.ty);
    // point p of this thread: tile-local linear index tid + 256 p, x3 fastest
    const int lx = threadIdx.x % kTX, ly = (threadIdx.x / kTX) % kTY, lz0 = threadIdx.x / (kTX * kTY);
    constexpr int kZStep = kSlThreads / (kTX * kTY);
    const int i3 = bx * kTX + lx, i2 = by * kTY + ly;
    if (threadIdx.x == 0) {
        box[0] = box[1] = box[2] = INT_MAX;
        box[3] = box[4] = box[5] = INT_MIN;
    }
    // 1. displacements and weights of this thread's points; the operands of
    //    the point update are loaded now so their latency hides under staging
    A a1[kPPT], a2[kPPT], a3[kPPT];
    typename Op::Pre pre[kPPT];
    bool ok[kPPT];
    int mn1 = INT_MAX, mn2 = INT_MAX, mn3 = INT_MAX, mx1 = INT_MIN, mx2 = INT_MIN, mx3 = INT_MIN;
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
        const int i1 = bz * kTZ + lz0 + p * kZStep;
        ok[p] = (i1 < g.n1) && (i2 < g.n2) && (i3 < g.n3);
        if (ok[p]) {
            const int idx = (i1 << g.s23) + (i2 << g.s3) + i3;
            T d[3];
            op.disp(idx, d);
            pre[p] = op.pre(idx);
            a1[p] = axis_weights<T, ORDER>(i1, d[0]);
            a2[p] = axis_weights<T, ORDER>(i2, d[1]);
            a3[p] = axis_weights<T, ORDER>(i3, d[2]);
            mn1 = min(mn1, a1[p].base);
            mx1 = max(mx1, a1[p].base);
            mn2 = min(mn2, a2[p].base);
            mx2 = max(mx2, a2[p].base);
            mn3 = min(mn3, a3[p].base);
            mx3 = max(mx3, a3[p].base);
        }
    }
    __syncthreads();  // box initialised
    mn1 = wave_min(mn1);
    mn2 = wave_min(mn2);
    mn3 = wave_min(mn3);
    mx1 = wave_max(mx1);
    mx2 = wave_max(mx2);
    mx3 = wave_max(mx3);
    if ((threadIdx.x & 63) == 0 && mn1 != INT_MAX) {
        atomicMin(&box[0], mn1);
        atomicMin(&box[1], mn2);
        atomicMin(&box[2], mn3);
        atomicMax(&box[3], mx1);
        atomicMax(&box[4], mx2);
        atomicMax(&box[5], mx3);
    }
    __syncthreads();
    if (box[0] == INT_MAX) return;  // tile outside the grid (uniform across the block)
    // box of every stencil node, in unwrapped grid coordinates
    const int lo1 = box[0] + FIRST, lo2 = box[1] + FIRST, lo3 = box[2] + FIRST;
    const long long e1 = (long long)box[3] - box[0] + NP, e2 = (long long)box[4] - box[1] + NP,
                    e3 = (long long)box[5] - box[2] + NP;
    const long long vol = e1 * e2 * e3;
    const bool staged = vol <= (long long)(g.lds_cap < CAP ? g.lds_cap : CAP);  // uniform across the block
    if (staged) {
        // 2. copy the box into LDS: flat index k = (z E2 + y) E3 + x; each thread
        //    walks k = tid, tid + 256, ... with (z, y, x) carried incrementally,
        //    kStageU loads in flight before the LDS stores
        const int E2 = (int)e2, E3 = (int)e3, E23 = E2 * E3, V = (int)vol;
        const int dz = kSlThreads / E23, rest = kSlThreads - dz * E23, dy = rest / E3, dx = rest - dy * E3;
        int z = (int)threadIdx.x / E23, y = ((int)threadIdx.x - z * E23) / E3;
        int x = (int)threadIdx.x - z * E23 - y * E3;
        const int m1 = g.n1 - 1, m2 = g.n2 - 1, m3 = g.n3 - 1;
        for (int k0 = threadIdx.x; k0 < V; k0 += kSlThreads * kStageU) {
            T v[kStageU][NF];
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
                if (k0 + u * kSlThreads < V) {
                    const int gi = (((lo1 + z) & m1) << g.s23) + (((lo2 + y) & m2) << g.s3) + ((lo3 + x) & m3);
                    op.stage(gi, v[u]);
                }
                // advance (z, y, x) by kSlThreads elements
                x += dx;
                y += dy;
                z += dz;
                if (x >= E3) {
                    x -= E3;
                    ++y;
                }
                if (y >= E2) {
                    y -= E2;
                    ++z;
                }
            }
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
                const int k = k0 + u * kSlThreads;
                if (k < V) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) lds[BoxLayout<NF>::template at<CAP>(k, f)] = v[u][f];
                }
            }
        }
        __syncthreads();
        // 3. stencils from LDS
#pragma unroll
        for (int p = 0; p < kPPT; ++p) {
            if (!ok[p]) continue;
            const int base = ((a1[p].base + FIRST - lo1) * E2 + (a2[p].base + FIRST - lo2)) * E3 +
                             (a3[p].base + FIRST - lo3);
            T acc[NF];
            contract_box<T, ORDER, NF>(
                a1[p], a2[p], a3[p], base, E23, E3,
                [&](int row, int r, T *v) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) v[f] = lds[BoxLayout<NF>::template at<CAP>(row + r, f)];
                },
                acc);
            const int idx = ((bz * kTZ + lz0 + p * kZStep) << g.s23) + (i2 << g.s3) + i3;
            op.finish(idx, pre[p], acc);
        }
    } else {
        // 3'. box too large for LDS: stencils straight from global memory
#pragma unroll
        for (int p = 0; p < kPPT; ++p) {
            if (!ok[p]) continue;
            int o1[NP], o2[NP], o3[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                o1[k] = ((a1[p].base + FIRST + k) & (g.n1 - 1)) << g.s23;
                o2[k] = ((a2[p].base + FIRST + k) & (g.n2 - 1)) << g.s3;
                o3[k] = (a3[p].base + FIRST + k) & (g.n3 - 1);
            }
            T acc[NF];
            contract<T, ORDER, NF>(
                a1[p], a2[p], a3[p], o1, o2, o3, [&](int off, T *v) { op.stage(off, v); }, acc);
            const int idx = ((bz * kTZ + lz0 + p * kZStep) << g.s23) + (i2 << g.s3) + i3;
            op.finish(idx, pre[p], acc);
        }
    }
}

// ---------------------------------------------------------------------------
// Step operators
// ---------------------------------------------------------------------------

// Characteristic foot: predictor x + sign dt v(x), then
// disp = sign dt/2 (v(x) + v(predictor)) / h.
template <typename T>
struct DepartureOp {
    const T *__restrict__ v;
    T *__restrict__ out;
    int N;
    T sdt, ih1, ih2, ih3;
    __device__ void disp(int i, T *d) const {
        d[0] = sdt * v[i] * ih1;
        d[1] = sdt * v[N + i] * ih2;
        d[2] = sdt * v[2 * N + i] * ih3;
    }
    __device__ void stage(int i, T *x) const {
        x[0] = v[i];
        x[1] = v[N + i];
        x[2] = v[2 * N + i];
    }
    struct Pre {
        T v1, v2, v3;
    };
    __device__ Pre pre(int i) const { return Pre{v[i], v[N + i], v[2 * N + i]}; }
    __device__ void finish(int i, const Pre &p, const T *a) const {
        const T h = (T)0.5 * sdt;
        out[i] = h * (p.v1 + a[0]) * ih1;
        out[N + i] = h * (p.v2 + a[1]) * ih2;
        out[2 * N + i] = h * (p.v3 + a[2]) * ih3;
    }
};

// out = I[f](x + disp); f and out in storage types SI, SO
template <typename T, typename SI, typename SO>
struct InterpOp {
    const SI *__restrict__ f;
    const T *__restrict__ D;
    SO *__restrict__ out;
    int N;
    __device__ void disp(int i, T *d) const {
        d[0] = D[i];
        d[1] = D[N + i];
        d[2] = D[2 * N + i];
    }
    __device__ void stage(int i, T *x) const { x[0] = load_as<T>(f, i); }
    struct Pre {};
    __device__ Pre pre(int) const { return Pre{}; }
    __device__ void finish(int i, const Pre &, const T *a) const { store_as(out, i, a[0]); }
};

// Adjoint step: lambda^j = L + dt/2 (S + (L + dt S) d), L = I[lambda^{j+1}](Y),
// S = I[lambda^{j+1} d](Y).
template <typename T, typename SL>
struct AdjointOp {
    const SL *__restrict__ lin;
    const T *__restrict__ dv;
    const T *__restrict__ Y;
    SL *__restrict__ lout;
    int N;
    T dt;
    __device__ void disp(int i, T *d) const {
        d[0] = Y[i];
        d[1] = Y[N + i];
        d[2] = Y[2 * N + i];
    }
    __device__ void stage(int i, T *x) const {
        const T l = load_as<T>(lin, i);
        x[0] = l;
        x[1] = l * dv[i];
    }
    struct Pre {
        T d;
    };
    __device__ Pre pre(int i) const { return Pre{dv[i]}; }
    __device__ void finish(int i, const Pre &p, const T *a) const {
        const T L = a[0], S = a[1];
        store_as(lout, i, L + (T)0.5 * dt * (S + (L + dt * S) * p.d));
    }
};

// Last adjoint step (j = 0) fused with the time integral: lambda^0 as above,
// then b = sum_j a_j lambda^j grad m^j from lambda^0 (in registers) and the
// stored lambda^1..nt; the history reads overlap the gather-bound step.
template <typename T, typename SL>
struct AdjointAccumOp {
    AdjointOp<T, SL> step;
    const SL *__restrict__ lam;  // history [nt+1][N]
    const T *__restrict__ gm;   // [nt+1][3][N]
    T *__restrict__ b;
    int nt;
    T a_end, a_mid;
    __device__ void disp(int i, T *d) const { step.disp(i, d); }
    __device__ void stage(int i, T *x) const { step.stage(i, x); }
    using Pre = typename AdjointOp<T, SL>::Pre;
    __device__ Pre pre(int i) const { return step.pre(i); }
    __device__ void finish(int i, const Pre &p, const T *a) const {
        const int N = step.N;
        const T L = a[0], S = a[1];
        const T l0 = L + (T)0.5 * step.dt * (S + (L + step.dt * S) * p.d);
        T al = a_end * l0;
        T b1 = al * gm[i], b2 = al * gm[N + i], b3 = al * gm[2 * N + i];
        for (int j = 1; j <= nt; ++j) {
            al = (j == nt ? a_end : a_mid) * load_as<T>(lam, (long long)j * N + i);
            const T *g = gm + 3 * j * N;
            b1 += al * g[i];
            b2 += al * g[N + i];
            b3 += al * g[2 * N + i];
        }
        b[i] = b1;
        b[N + i] = b2;
        b[2 * N + i] = b3;
    }
};

// Incremental state: q^{j+1} = I[q^j](X) + coef f^{j+1}, f = -grad m^{j+1} . vt;
// on the last step (coef = dt/2) the output is -mt(1), the final condition
// of the incremental adjoint.
template <typename T, typename SQ>
struct IncStateOp {
    const SQ *__restrict__ qin;
    const T *__restrict__ X;
    const T *__restrict__ gm;
    const T *__restrict__ vt;
    SQ *__restrict__ qout;
    int N;
    T coef, sign;
    __device__ void disp(int i, T *d) const {
        d[0] = X[i];
        d[1] = X[N + i];
        d[2] = X[2 * N + i];
    }
    __device__ void stage(int i, T *x) const { x[0] = load_as<T>(qin, i); }
    struct Pre {
        T f;
    };
    __device__ Pre pre(int i) const {
        return Pre{-(gm[i] * vt[i] + gm[N + i] * vt[N + i] + gm[2 * N + i] * vt[2 * N + i])};
    }
    __device__ void finish(int i, const Pre &p, const T *a) const { store_as(qout, i, sign * (a[0] + coef * p.f)); }
};

// Final condition of the adjoint: lambda(1) = mR - m(1).
template <typename T, typename S>
__global__ __launch_bounds__(kSlThreads) void k_adjoint_init(long long N, const T *__restrict__ mR,
                                                             const T *__restrict__ m, S *__restrict__ lam) {
    const long long idx = (long long)blockIdx.x * kSlThreads + threadIdx.x;
    if (idx >= N) return;
    store_as(lam, idx, mR[idx] - m[idx]);
}

template <typename T, typename S>
__global__ __launch_bounds__(kSlThreads) void k_incstate_init(long long N, T hdt, const T *__restrict__ gm,
                                                              const T *__restrict__ vt, S *__restrict__ q) {
    const long long idx = (long long)blockIdx.x * kSlThreads + threadIdx.x;
    if (idx >= N) return;
    const T f = -(gm[idx] * vt[idx] + gm[N + idx] * vt[N + idx] + gm[2 * N + idx] * vt[2 * N + idx]);
    store_as(q, idx, hdt * f);
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + kSlThreads - 1) / kSlThreads); }

template <typename T, int NF, int SHAPE, class Op>
static void launch_sl_shape(const PGrid &g, int order, const Op &op, hipStream_t s) {
    const unsigned nb = (unsigned)(g.tx * g.ty * g.tz);
    if (order == 3)
        hipLaunchKernelGGL((k_sl<T, 3, NF, SHAPE, Op>), dim3(nb), dim3(kSlThreads), 0, s, g, op);
    else
        hipLaunchKernelGGL((k_sl<T, 1, NF, SHAPE, Op>), dim3(nb), dim3(kSlThreads), 0, s, g, op);
}

template <typename T, int NF, class Op>
static void launch_sl(const PGrid &g, int order, const Op &op, hipStream_t s) {
    switch (g.shape) {
        case TILE_8x8x16: launch_sl_shape<T, NF, TILE_8x8x16>(g, order, op, s); break;
        case TILE_8x16x16: launch_sl_shape<T, NF, TILE_8x16x16>(g, order, op, s); break;
        default: launch_sl_shape<T, NF, TILE_4x8x32>(g, order, op, s); break;
    }
}

template <typename T>
void departure(const Grid &gg, int order, int sign, double dt, const T *v, T *disp, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_DEPARTURE, 6.0 * g.N * sizeof(T));
    const double two_pi = 6.283185307179586476925;
    DepartureOp<T> op{v, disp, (int)g.N, (T)(sign * dt), (T)(g.n1 / two_pi), (T)(g.n2 / two_pi), (T)(g.n3 / two_pi)};
    launch_sl<T, 3>(g, order, op, s);
}

template <typename T, typename SI, typename SO>
void interp_field(const Grid &gg, int order, const SI *f, const T *disp, SO *out, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INTERP, (3.0 * sizeof(T) + sizeof(SI) + sizeof(SO)) * g.N);
    InterpOp<T, SI, SO> op{f, disp, out, (int)g.N};
    launch_sl<T, 1>(g, order, op, s);
}

template <typename T, typename S>
void adjoint_init(const Grid &g, const T *mR, const T *m, S *lam, hipStream_t s) {
    HookScope hs(K_ADJ_INIT, (2.0 * sizeof(T) + sizeof(S)) * g.N);
    hipLaunchKernelGGL((k_adjoint_init<T, S>), dim3(blocks_for(g.N)), dim3(kSlThreads), 0, s, g.N, mR, m, lam);
}

template <typename T, typename S>
void adjoint_step(const Grid &gg, int order, double dt, const S *lam_in, const T *d, const T *Y, S *lam_out,
                  hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_ADJ_STEP, (4.0 * sizeof(T) + 2.0 * sizeof(S)) * g.N);
    AdjointOp<T, S> op{lam_in, d, Y, lam_out, (int)g.N, (T)dt};
    launch_sl<T, 2>(g, order, op, s);
}

template <typename T, typename S>
void adjoint_step_accumulate(const Grid &gg, int order, double dt, int nt, const S *lam, const T *d,
                             const T *Y, const T *gradm, T *b, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_ADJ_ACC, ((4.0 + 3.0 * (nt + 1) + 3.0) * sizeof(T) + (double)nt * sizeof(S)) * g.N);
    const long long N = g.N;
    AdjointOp<T, S> step{lam + N, d, Y, nullptr, (int)N, (T)dt};
    AdjointAccumOp<T, S> op{step, lam, gradm, b, nt, (T)(0.5 * dt), (T)dt};
    launch_sl<T, 2>(g, order, op, s);
}

template <typename T, typename S>
void incstate_init(const Grid &g, double dt, const T *gradm0, const T *vt, S *q, hipStream_t s) {
    HookScope hs(K_INC_INIT, 6.0 * sizeof(T) * g.N + sizeof(S) * g.N);
    hipLaunchKernelGGL((k_incstate_init<T, S>), dim3(blocks_for(g.N)), dim3(kSlThreads), 0, s, g.N,
                       (T)(0.5 * dt), gradm0, vt, q);
}

template <typename T, typename S>
void incstate_step(const Grid &gg, int order, double coef, double sign, const S *q_in, const T *X,
                   const T *gradm_next, const T *vt, S *q_out, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INC_STEP, 9.0 * sizeof(T) * g.N + 2.0 * sizeof(S) * g.N);
    IncStateOp<T, S> op{q_in, X, gradm_next, vt, q_out, (int)g.N, (T)coef, (T)sign};
    launch_sl<T, 1>(g, order, op, s);
}

template void departure<float>(const Grid &, int, int, double, const float *, float *, hipStream_t);
template void departure<double>(const Grid &, int, int, double, const double *, double *, hipStream_t);
#define MIREG_INST(T, S)                                                                                  \
    template void interp_field<T, S, S>(const Grid &, int, const S *, const T *, S *, hipStream_t);       \
    template void adjoint_init<T, S>(const Grid &, const T *, const T *, S *, hipStream_t);              \
    template void adjoint_step<T, S>(const Grid &, int, double, const S *, const T *, const T *, S *,    \
                                     hipStream_t);                                                        \
    template void adjoint_step_accumulate<T, S>(const Grid &, int, double, int, const S *, const T *,    \
                                                const T *, const T *, T *, hipStream_t);                 \
    template void incstate_init<T, S>(const Grid &, double, const T *, const T *, S *, hipStream_t);     \
    template void incstate_step<T, S>(const Grid &, int, double, double, const S *, const T *, const T *, \
                                      const T *, S *, hipStream_t);
MIREG_INST(float, float)
MIREG_INST(double, double)
MIREG_INST(float, __half)
#undef MIREG_INST

}  // namespace mireg
