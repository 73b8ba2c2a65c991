// Semi-Lagrangian transport kernels (Sec. 2.3.1, Sec. 3.4) for gfx950.
//
// Off-grid values are third-degree Lagrange polynomials on a 4x4x4 stencil
// (trilinear on 2x2x2), periodic.  Departure points are
// stored as displacements in cell units, so t = d - floor(d) keeps full
// precision in FP32 anywhere on the grid.
//
// Every step is one kernel over tiles of points (16 x3 x 8 x2 x 8 x1 by
// default; 32 x 8 x 4 and 16 x 16 x 8 selectable), 256 threads:
//   1. each thread reads the displacement of its points (coalesced rows
//      along x3) and the block reads its tile's bounding box of all
//      stencils, measured once per displacement field (k_box; without the
//      stored boxes the block reduces it from the displacements);
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

#include <mutex>
#include <string>
#include <type_traits>

#include "kernels.hpp"
#include "mireg.h"

namespace mireg {

struct PGrid {
    int n1, n2, n3;
    int n23;      // n2 n3
    unsigned m1, m2, m3;  // n_a - 1 on power-of-two axes, 0 on the others
    long long N;
    int tx, ty, tz;  // tiles per axis
    int ltx, lty;    // log2(tx), log2(ty) when both are powers of two, else -1
    int lds_cap;     // largest box (nodes) staged in LDS in this launch; 0 disables staging
    int shape;       // tile shape (SlTile)
    const int *tbox; // every tile's stencil box (8 ints per tile), or null: reduce it in the kernel
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
constexpr int kStageU = 8;        // staging loads in flight per thread (wide planes)
constexpr int kStageZ = 4;        // planes per staging batch
constexpr int kStageCols = 2;     // plane positions per thread (planes of up to 512 nodes)
static_assert(kStageCols == 2, "the plane staging instantiates one and two positions");
constexpr int kLdsBytes = 65536;  // largest LDS allocation of one workgroup

// Cells per unit length on axis a (the grid spans 2 pi).
static double departure_ih(const Grid &g, int a) {
    const double two_pi = 6.283185307179586476925;
    return (a == 0 ? g.n1 : a == 1 ? g.n2 : g.n3) / two_pi;
}

static PGrid pgrid(const Grid &g) {
    PGrid p;
    p.n1 = g.n1;
    p.n2 = g.n2;
    p.n3 = g.n3;
    p.n23 = g.n2 * g.n3;
    auto mask = [](int n) { return (n & (n - 1)) == 0 ? (unsigned)(n - 1) : 0u; };
    p.m1 = mask(g.n1);
    p.m2 = mask(g.n2);
    p.m3 = mask(g.n3);
    p.N = g.N;
    p.shape = g.sl_tile;
    int TZ = 8, TY = 8, TX = 16;
    switch (p.shape) {
        case TILE_4x8x32: TZ = 4, TY = 8, TX = 32; break;
        case TILE_8x16x16: TZ = 8, TY = 16, TX = 16; break;
        default: break;
    }
    p.tx = (g.n3 + TX - 1) / TX;
    p.ty = (g.n2 + TY - 1) / TY;
    p.tz = (g.n1 + TZ - 1) / TZ;
    const bool pow2_tiles = (p.tx & (p.tx - 1)) == 0 && (p.ty & (p.ty - 1)) == 0;
    p.ltx = pow2_tiles ? __builtin_ctz((unsigned)p.tx) : -1;
    p.lty = pow2_tiles ? __builtin_ctz((unsigned)p.ty) : -1;
    p.lds_cap = g.lds_cap;
    p.tbox = nullptr;
    return p;
}

// Node weights of one axis (from the fractional position t in [0, 1)) and
// the node below the position.
template <typename T, int ORDER>
struct AxisW {
    static constexpr int NP = ORDER == 3 ? 4 : 2;
    static constexpr int FIRST = ORDER == 3 ? -1 : 0;
    int base;  // i + floor(d)
    T w[NP];
};

template <typename T, int ORDER>
__device__ __forceinline__ AxisW<T, ORDER> axis_weights(int base, T t) {
    AxisW<T, ORDER> a;
    a.base = base;
    if constexpr (ORDER == 3) {
        // cubic Lagrange basis on the nodes -1, 0, 1, 2
        const T tm1 = t - (T)1, tm2 = t - (T)2, tp1 = t + (T)1;
        const T u = t * tm1, w = tp1 * tm2;
        a.w[0] = u * (tm2 * (T)(-1.0 / 6.0));
        a.w[1] = w * (tm1 * (T)0.5);
        a.w[2] = w * (t * (T)(-0.5));
        a.w[3] = u * (tp1 * (T)(1.0 / 6.0));
    } else {
        a.w[0] = (T)1 - t;
        a.w[1] = t;
    }
    return a;
}

// t = d - floor(d) as a separately rounded subtraction.  Contracted with the
// product that formed d into one fused operation, t would describe the
// unrounded displacement, could leave [0, 1), and an integer displacement
// would no longer give exact 0/1 weights.
template <typename T>
__device__ __forceinline__ T frac_part(T d, T fl) {
#pragma clang fp contract(off)
    return d - fl;
}

// Element i of an array through a 32-bit unsigned byte offset (every field
// here is below 4 GiB), so loads and stores take the scalar-base plus
// vector-offset address form; S is the storage type, T the arithmetic type.
template <typename T, typename S>
__device__ __forceinline__ T ld(const S *p, unsigned i) {
    return load_as<T>(reinterpret_cast<const S *>(reinterpret_cast<const char *>(p) + i * (unsigned)sizeof(S)), 0);
}
template <typename S, typename T>
__device__ __forceinline__ void st(S *p, unsigned i, T v) {
    store_as(reinterpret_cast<S *>(reinterpret_cast<char *>(p) + i * (unsigned)sizeof(S)), 0, v);
}

template <int NP>
using NodeOff = unsigned[NP];

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
            const unsigned row = o1[p] + o2[q];
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

// Same contraction over an unwrapped box: row (p, q) at base + p s1 + q s2
// (byte offsets: one add per row, the r taps of a row at immediate
// offsets).  All taps of a plane p are read before any arithmetic, so a wave
// keeps 16 (NF = 1) or 32 (NF = 2) LDS words in flight instead of waiting row
// by row.
template <typename T, int ORDER, int NF, class Get>
__device__ __forceinline__ void contract_box(const AxisW<T, ORDER> &a1, const AxisW<T, ORDER> &a2,
                                             const AxisW<T, ORDER> &a3, unsigned base, unsigned s1,
                                             unsigned s2, const Get &get, T *acc) {
    constexpr int NP = AxisW<T, ORDER>::NP;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        T v[NP][NP][NF];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const unsigned row = base + (unsigned)p * s1 + (unsigned)q * s2;
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
// are adjacent, one 4/8/16-byte read), NF = 3 one array of `stride` nodes per
// quantity.
template <int NF>
__device__ __forceinline__ int box_at(int k, int f, int stride) {
    return NF <= 2 ? k * NF + f : f * stride + k;
}

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

// a mod n (Euclidean) for any a; mask = n - 1 when n is a power of two, else 0.
__device__ __forceinline__ unsigned wrap(int a, int n, unsigned mask) {
    if (mask) return (unsigned)a & mask;
    const int r = a % n;
    return (unsigned)(r < 0 ? r + n : r);
}

// Point p of a thread in its tile: tile-local linear index tid + 256 p, x3
// fastest.  Shared by the transport kernels and the box measurement, so both
// see the same tiles.
template <int SHAPE>
struct TilePoints {
    static constexpr int TZ = TileDims<SHAPE>::TZ, TY = TileDims<SHAPE>::TY, TX = TileDims<SHAPE>::TX;
    static constexpr int PPT = TX * TY * TZ / kSlThreads;  // points per thread
    static constexpr int ZSTEP = kSlThreads / (TX * TY);
    int i1_0, i2, i3;  // grid index of point 0 (i1 advances by ZSTEP per point)
    __device__ TilePoints(const PGrid &g, int tile) {
        int bx, by, bz;
        if (g.ltx >= 0) {
            bx = tile & (g.tx - 1);
            by = (tile >> g.ltx) & (g.ty - 1);
            bz = tile >> (g.ltx + g.lty);
        } else {
            bx = tile % g.tx;
            by = (tile / g.tx) % g.ty;
            bz = tile / (g.tx * g.ty);
        }
        i3 = bx * TX + (int)threadIdx.x % TX;
        i2 = by * TY + ((int)threadIdx.x / TX) % TY;
        i1_0 = bz * TZ + (int)threadIdx.x / (TX * TY);
    }
    __device__ int i1(int p) const { return i1_0 + p * ZSTEP; }
    __device__ bool ok(const PGrid &g, int p) const { return i1(p) < g.n1 && i2 < g.n2 && i3 < g.n3; }
    __device__ unsigned idx(const PGrid &g, int p) const {
        return __umul24((unsigned)i1(p), (unsigned)g.n23) + __umul24((unsigned)i2, (unsigned)g.n3) + (unsigned)i3;
    }
};

// q = a / b and r = a - q b for 0 <= a, 0 < b, both below 2^16, from the
// float estimate a (1/b) (relative error below 2^-22, so off by at most
// one) and one correction step.
__device__ __forceinline__ int small_div(int a, int b, float rb, int &r) {
    int q = (int)((float)a * rb);
    r = a - q * b;
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    return q;
}

// Block-wide bounding box of the base nodes (min, max per axis) into box[6];
// returns false when the tile has no point inside the grid (uniform).
__device__ __forceinline__ bool block_box(int *box, int mn1, int mn2, int mn3, int mx1, int mx2, int mx3) {
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
    return box[0] != INT_MAX;
}

// One-field FP32 ops whose staged value is the loaded value (the state and
// incremental-state steps): their box goes from global memory straight into
// LDS (global_load_lds_dword), without passing through registers.
template <class Op>
struct DirectStage {
    static constexpr bool value = false;
};

// Generic tiled semi-Lagrangian sweep.  Op provides:
//   void disp(unsigned idx, T *d)       displacement of point idx (cells, 3 values)
//   void stage(unsigned plane, unsigned rc, T *v)
//                                       loads behind the NF gathered quantities at grid index
//                                       plane + rc (plane: x1 offset, block-uniform)
//   void staged(T *v)                   turns those loads into the NF quantities (no loads)
//   Pre pre(unsigned idx)               operands of the point update, loaded early
//   void finish(unsigned idx, const Pre &, const T *acc)  output of point idx
// g.lds_cap is the dynamic LDS size of the launch in box nodes: tiles whose
// stencil box is larger gather from global memory.  Only the fractional
// positions and base nodes live across the staging phase; the weights are
// formed point by point afterwards, which keeps the register count low.
//
// MULTI: one launch for several problems.  Their tiles are numbered one after
// the other (problem p owns tiles tab[p].start .. tab[p].start + its tile
// count - 1), each workgroup finds its problem in the table (a block-uniform
// scan of at most a few dozen entries) and runs the single-problem tile code
// on that problem's grid and operands, so every problem's results are those
// of its own launch; every entry's lds_cap is at most the launch's dynamic
// LDS.  (A flag on this kernel rather than a shared device function: with
// the tile code outside the kernel body the compiler keeps the operands of
// the single-problem launches in more registers.)
template <class Op>
struct SlEntry {
    PGrid g;
    Op op;
    int start;
};

template <typename T, int ORDER, int NF, int SHAPE, class Op, bool MULTI = false>
__global__ __launch_bounds__(kSlThreads) void k_sl(PGrid g0, Op op0, const SlEntry<Op> *__restrict__ tab, int nprob,
                                                   int total) {
    int pm = 0;
    if constexpr (MULTI) {
        const int t = xcd_tile(blockIdx.x, total);
        while (pm + 1 < nprob && tab[pm + 1].start <= t) ++pm;
    }
    const PGrid &g = MULTI ? tab[pm].g : g0;
    const Op &op = MULTI ? tab[pm].op : op0;
    using TP = TilePoints<SHAPE>;
    constexpr int kPPT = TP::PPT;
    using A = AxisW<T, ORDER>;
    constexpr int NP = A::NP, FIRST = A::FIRST;
    extern __shared__ __align__(16) unsigned char sl_smem[];
    T *lds = reinterpret_cast<T *>(sl_smem);
    __shared__ int box[6];
    const int tile = MULTI ? xcd_tile(blockIdx.x, total) - tab[pm].start : xcd_tile(blockIdx.x, g.tx * g.ty * g.tz);
    const TP tp(g, tile);
    // box of the base nodes (lowest, highest per axis) in unwrapped grid
    // coordinates (block-uniform): the stored one, or reduced over the
    // block.  The stored box is one vector load per wave (lane l reads word
    // l & 7), issued with the displacement loads and waited for with them.
    const bool stored = g.tbox != nullptr;  // uniform
    int tbw = 0;
    if (stored) {
        tbw = g.tbox[8 * tile + ((int)threadIdx.x & 7)];
    } else if (threadIdx.x == 0) {
        box[0] = box[1] = box[2] = INT_MAX;
        box[3] = box[4] = box[5] = INT_MIN;
    }
    // 1. displacements -> base node and fractional position per axis
    T t1[kPPT], t2[kPPT], t3[kPPT];
    int b1[kPPT], b2[kPPT], b3[kPPT];
    typename Op::Pre pre[kPPT];
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
        if (tp.ok(g, p)) {
            const unsigned idx = tp.idx(g, p);
            T d[3];
            op.disp(idx, d);
            const T f1 = floor(d[0]), f2 = floor(d[1]), f3 = floor(d[2]);
            t1[p] = frac_part(d[0], f1);
            t2[p] = frac_part(d[1], f2);
            t3[p] = frac_part(d[2], f3);
            b1[p] = tp.i1(p) + (int)f1;
            b2[p] = tp.i2 + (int)f2;
            b3[p] = tp.i3 + (int)f3;
        }
    }
    int c0, c1, c2, c3, c4, c5;
    if (stored) {
        c0 = __builtin_amdgcn_readlane(tbw, 0);
        c1 = __builtin_amdgcn_readlane(tbw, 1);
        c2 = __builtin_amdgcn_readlane(tbw, 2);
        c3 = __builtin_amdgcn_readlane(tbw, 3);
        c4 = __builtin_amdgcn_readlane(tbw, 4);
        c5 = __builtin_amdgcn_readlane(tbw, 5);
        if (c0 == INT_MAX) return;  // no point of the grid in this tile
    } else {
        int mn1 = INT_MAX, mn2 = INT_MAX, mn3 = INT_MAX, mx1 = INT_MIN, mx2 = INT_MIN, mx3 = INT_MIN;
#pragma unroll
        for (int p = 0; p < kPPT; ++p) {
            if (tp.ok(g, p)) {
                mn1 = min(mn1, b1[p]);
                mx1 = max(mx1, b1[p]);
                mn2 = min(mn2, b2[p]);
                mx2 = max(mx2, b2[p]);
                mn3 = min(mn3, b3[p]);
                mx3 = max(mx3, b3[p]);
            }
        }
        __syncthreads();  // box initialised
        if (!block_box(box, mn1, mn2, mn3, mx1, mx2, mx3)) return;
        c0 = __builtin_amdgcn_readfirstlane(box[0]);
        c1 = __builtin_amdgcn_readfirstlane(box[1]);
        c2 = __builtin_amdgcn_readfirstlane(box[2]);
        c3 = __builtin_amdgcn_readfirstlane(box[3]);
        c4 = __builtin_amdgcn_readfirstlane(box[4]);
        c5 = __builtin_amdgcn_readfirstlane(box[5]);
    }
    // the operands of the point update, loaded now so that their latency
    // hides under the staging
#pragma unroll
    for (int p = 0; p < kPPT; ++p)
        if (tp.ok(g, p)) pre[p] = op.pre(tp.idx(g, p));
    const int lo1 = c0 + FIRST, lo2 = c1 + FIRST, lo3 = c2 + FIRST;
    const long long e1 = (long long)c3 - c0 + NP, e2 = (long long)c4 - c1 + NP, e3 = (long long)c5 - c2 + NP;
    const long long vol = e1 * e2 * e3;
    // LDS holds cap + 1 nodes: the box (at most cap) and one spare node;
    // NF = 3 keeps one array of cap + 1 per quantity
    const int cap = g.lds_cap, stride = cap + 1;
    if (vol <= (long long)cap) {  // uniform across the block
        // 2. copy the box into LDS, node (z, y, x) at k = z E23 + r, r = y E3 + x
        //    (vol <= cap < 2^16).
        const int E1 = (int)e1, E2 = (int)e2, E3 = (int)e3, E23 = E2 * E3, V = (int)vol;
        const float rE3 = 1.0f / (float)E3;
        const unsigned n23 = (unsigned)g.n23, n3 = (unsigned)g.n3;
        if (E23 <= kStageCols * kSlThreads) {  // uniform
            // Plane by plane: thread tid copies the plane positions r = tid +
            // 256 j, whose wrapped (x2, x3) offsets are formed once; the plane
            // offset is block-uniform.  A batch of kStageZ planes is straight-
            // line code, all its loads in flight before the LDS stores: lanes
            // past the plane or planes past the box load a duplicate node and
            // store it to the spare node `cap`.
            unsigned rc[kStageCols];
            int rk[kStageCols];
#pragma unroll
            for (int j = 0; j < kStageCols; ++j) {
                const int r = (int)threadIdx.x + j * kSlThreads;
                int x;
                const int y = small_div(r, E3, rE3, x);
                rc[j] = __umul24(wrap(lo2 + y, g.n2, g.m2), n3) + wrap(lo3 + x, g.n3, g.m3);
                rk[j] = r < E23 ? r : -1;
            }
            auto planes = [&](auto cols) {
                constexpr int JJ = decltype(cols)::value;
                if constexpr (DirectStage<Op>::value) {
                    // lane l of a wave writes the LDS word at a wave-uniform base + l: the
                    // wave's 64 consecutive plane positions; lanes past the plane are
                    // masked off (no spare node), the loads complete before the barrier
                    const int wave = (int)threadIdx.x >> 6;
                    for (int z = 0; z < E1; ++z) {
                        const unsigned plane = __umul24(wrap(lo1 + z, g.n1, g.m1), n23);
                        const float *srcp = op.direct_src(plane);
#pragma unroll
                        for (int j = 0; j < JJ; ++j) {
                            const int base = z * E23 + 64 * wave + kSlThreads * j;
                            if (rk[j] >= 0)
                                __builtin_amdgcn_global_load_lds(srcp + rc[j], lds + base, 4, 0, 0);
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0);
                    return;
                }
                unsigned src[JJ];
#pragma unroll
                for (int j = 0; j < JJ; ++j) src[j] = rk[j] >= 0 ? rc[j] : rc[0];
                for (int z0 = 0; z0 < E1; z0 += kStageZ) {
                    T v[kStageZ][JJ][NF];
#pragma unroll
                    for (int zz = 0; zz < kStageZ; ++zz) {
                        const int z = z0 + zz < E1 ? z0 + zz : E1 - 1;
                        const unsigned plane = __umul24(wrap(lo1 + z, g.n1, g.m1), n23);
#pragma unroll
                        for (int j = 0; j < JJ; ++j) op.stage(plane, src[j], v[zz][j]);
                    }
#pragma unroll
                    for (int zz = 0; zz < kStageZ; ++zz) {
                        const int kz = z0 + zz < E1 ? (z0 + zz) * E23 : -1;
#pragma unroll
                        for (int j = 0; j < JJ; ++j) {
                            op.staged(v[zz][j]);
                            const int k = (kz >= 0 && rk[j] >= 0) ? kz + rk[j] : cap;
#pragma unroll
                            for (int f = 0; f < NF; ++f) lds[box_at<NF>(k, f, stride)] = v[zz][j][f];
                        }
                    }
                }
            };
            if (E23 > kSlThreads)
                planes(std::integral_constant<int, 2>{});
            else
                planes(std::integral_constant<int, 1>{});
        } else {
            // Wide planes: thread tid walks k = tid, tid + 256, ... with (z, y, x)
            // carried incrementally (unwrapped as lo + (z, y, x)).
            const float rE23 = 1.0f / (float)E23;
            int rest, dx;
            const int dz = small_div(kSlThreads, E23, rE23, rest), dy = small_div(rest, E3, rE3, dx);
            int r0, x;
            const int z = small_div((int)threadIdx.x, E23, rE23, r0), y = small_div(r0, E3, rE3, x);
            int uz = lo1 + z, uy = lo2 + y, ux = lo3 + x;
            const int hi2 = lo2 + E2, hi3 = lo3 + E3;
            for (int k0 = threadIdx.x; k0 < V; k0 += kSlThreads * kStageU) {
                T v[kStageU][NF];
#pragma unroll
                for (int u = 0; u < kStageU; ++u) {
                    if (k0 + u * kSlThreads < V)
                        op.stage(__umul24(wrap(uz, g.n1, g.m1), n23),
                                 __umul24(wrap(uy, g.n2, g.m2), n3) + wrap(ux, g.n3, g.m3), v[u]);
                    ux += dx;
                    uy += dy;
                    uz += dz;
                    if (ux >= hi3) {
                        ux -= E3;
                        ++uy;
                    }
                    if (uy >= hi2) {
                        uy -= E2;
                        ++uz;
                    }
                }
#pragma unroll
                for (int u = 0; u < kStageU; ++u) {
                    const int k = k0 + u * kSlThreads;
                    if (k < V) {
                        op.staged(v[u]);
#pragma unroll
                        for (int f = 0; f < NF; ++f) lds[box_at<NF>(k, f, stride)] = v[u][f];
                    }
                }
            }
        }
        __syncthreads();
        // 3. stencils from LDS
#pragma unroll
        for (int p = 0; p < kPPT; ++p) {
            if (!tp.ok(g, p)) continue;
            const A a1 = axis_weights<T, ORDER>(b1[p], t1[p]);
            const A a2 = axis_weights<T, ORDER>(b2[p], t2[p]);
            const A a3 = axis_weights<T, ORDER>(b3[p], t3[p]);
            // byte offsets into the box: U bytes per node of the interleaved
            // layout (NF <= 2), one quantity's array at a time for NF = 3
            constexpr unsigned U = NF <= 2 ? NF * sizeof(T) : sizeof(T);
            const unsigned node =
                __umul24(__umul24((unsigned)(b1[p] + FIRST - lo1), (unsigned)E2) + (unsigned)(b2[p] + FIRST - lo2),
                         (unsigned)E3) +
                (unsigned)(b3[p] + FIRST - lo3);
            T acc[NF];
            contract_box<T, ORDER, NF>(
                a1, a2, a3, node * U, (unsigned)E23 * U, (unsigned)E3 * U,
                [&](unsigned row, int r, T *v) {
                    const char *at = reinterpret_cast<const char *>(lds) + row + r * U;
#pragma unroll
                    for (int f = 0; f < NF; ++f)
                        v[f] = *reinterpret_cast<const T *>(at + box_at<NF>(0, f, stride) * sizeof(T));
                },
                acc);
            op.finish(tp.idx(g, p), pre[p], acc);
        }
    } else {
        // 3'. box larger than the launch's LDS: stencils straight from global memory
#pragma unroll
        for (int p = 0; p < kPPT; ++p) {
            if (!tp.ok(g, p)) continue;
            const A a1 = axis_weights<T, ORDER>(b1[p], t1[p]);
            const A a2 = axis_weights<T, ORDER>(b2[p], t2[p]);
            const A a3 = axis_weights<T, ORDER>(b3[p], t3[p]);
            unsigned o1[NP], o2[NP], o3[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                o1[k] = __umul24(wrap(b1[p] + FIRST + k, g.n1, g.m1), (unsigned)g.n23);
                o2[k] = __umul24(wrap(b2[p] + FIRST + k, g.n2, g.m2), (unsigned)g.n3);
                o3[k] = wrap(b3[p] + FIRST + k, g.n3, g.m3);
            }
            T acc[NF];
            contract<T, ORDER, NF>(
                a1, a2, a3, o1, o2, o3,
                [&](unsigned off, T *v) {
                    op.stage(0u, off, v);
                    op.staged(v);
                },
                acc);
            op.finish(tp.idx(g, p), pre[p], acc);
        }
    }
}

// Largest stencil box (nodes) over the tiles of k_sl for the displacement
// d_a = (a_a D_a) b_a, the same expression the step operators evaluate:
// one block per tile, atomic maximum into one of kBoxSlots slots (so that
// the blocks do not all serialise on one address), then k_max_slots.  With
// `tiles`, also each tile's box of base nodes, as k_sl would reduce it.
constexpr int kBoxSlots = 1024;
template <typename T, int ORDER, int SHAPE>
__global__ __launch_bounds__(kSlThreads) void k_box(PGrid g, const T *__restrict__ D, T a, T b1, T b2, T b3,
                                                    unsigned *__restrict__ slots, int *__restrict__ tiles) {
    using TP = TilePoints<SHAPE>;
    constexpr int NP = AxisW<T, ORDER>::NP;
    __shared__ int box[6];
    const int tile = xcd_tile(blockIdx.x, g.tx * g.ty * g.tz);
    const TP tp(g, tile);
    if (threadIdx.x == 0) {
        box[0] = box[1] = box[2] = INT_MAX;
        box[3] = box[4] = box[5] = INT_MIN;
    }
    const unsigned N = (unsigned)g.N;
    int mn1 = INT_MAX, mn2 = INT_MAX, mn3 = INT_MAX, mx1 = INT_MIN, mx2 = INT_MIN, mx3 = INT_MIN;
#pragma unroll
    for (int p = 0; p < TP::PPT; ++p) {
        if (tp.ok(g, p)) {
            const unsigned idx = tp.idx(g, p);
            const int c1 = tp.i1(p) + (int)floor(a * ld<T>(D, idx) * b1);
            const int c2 = tp.i2 + (int)floor(a * ld<T>(D, N + idx) * b2);
            const int c3 = tp.i3 + (int)floor(a * ld<T>(D, 2 * N + idx) * b3);
            mn1 = min(mn1, c1);
            mx1 = max(mx1, c1);
            mn2 = min(mn2, c2);
            mx2 = max(mx2, c2);
            mn3 = min(mn3, c3);
            mx3 = max(mx3, c3);
        }
    }
    __syncthreads();
    const bool any = block_box(box, mn1, mn2, mn3, mx1, mx2, mx3);
    if (tiles && threadIdx.x < 8) tiles[8 * tile + (int)threadIdx.x] = threadIdx.x < 6 ? box[threadIdx.x] : 0;
    if (!any) return;
    if (threadIdx.x == 0) {
        const long long vol = ((long long)box[3] - box[0] + NP) * ((long long)box[4] - box[1] + NP) *
                              ((long long)box[5] - box[2] + NP);
        atomicMax(&slots[blockIdx.x & (kBoxSlots - 1)], (unsigned)(vol < (long long)UINT_MAX ? vol : (long long)UINT_MAX));
    }
}

__global__ __launch_bounds__(256) void k_zero_slots(unsigned *slots) {
    slots[blockIdx.x * 256 + threadIdx.x] = 0u;
}

// out[0] = max of the kBoxSlots slots (one workgroup)
__global__ __launch_bounds__(256) void k_max_slots(const unsigned *__restrict__ slots, unsigned *__restrict__ out) {
    __shared__ unsigned sh[4];
    unsigned m = 0;
    for (int i = threadIdx.x; i < kBoxSlots; i += 256) m = max(m, slots[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
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
    unsigned N;
    T sdt, ih1, ih2, ih3;
    __device__ void disp(unsigned i, T *d) const {
        d[0] = sdt * ld<T>(v, i) * ih1;
        d[1] = sdt * ld<T>(v, N + i) * ih2;
        d[2] = sdt * ld<T>(v, 2 * N + i) * ih3;
    }
    __device__ void stage(unsigned pl, unsigned i, T *x) const {
        x[0] = ld<T>(v + pl, i);
        x[1] = ld<T>(v + N + pl, i);
        x[2] = ld<T>(v + 2 * N + pl, i);
    }
    __device__ void staged(T *) const {}
    struct Pre {
        T v1, v2, v3;
    };
    __device__ Pre pre(unsigned i) const { return Pre{ld<T>(v, i), ld<T>(v, N + i), ld<T>(v, 2 * N + i)}; }
    __device__ void finish(unsigned i, const Pre &p, const T *a) const {
        const T h = (T)0.5 * sdt;
        st(out, i, h * (p.v1 + a[0]) * ih1);
        st(out, N + i, h * (p.v2 + a[1]) * ih2);
        st(out, 2 * N + i, h * (p.v3 + a[2]) * ih3);
    }
};

// out = I[f](x + disp); f and out in storage types SI, SO
template <typename T, typename SI, typename SO>
struct InterpOp {
    const SI *__restrict__ f;
    const T *__restrict__ D;
    SO *__restrict__ out;
    unsigned N;
    __device__ void disp(unsigned i, T *d) const {
        d[0] = ld<T>(D, i);
        d[1] = ld<T>(D, N + i);
        d[2] = ld<T>(D, 2 * N + i);
    }
    __device__ void stage(unsigned pl, unsigned i, T *x) const { x[0] = ld<T>(f + pl, i); }
    __device__ void staged(T *) const {}
    __device__ const SI *direct_src(unsigned pl) const { return f + pl; }
    struct Pre {};
    __device__ Pre pre(unsigned) const { return Pre{}; }
    __device__ void finish(unsigned i, const Pre &, const T *a) const { st(out, i, a[0]); }
};

// Adjoint step: lambda^j = L + dt/2 (S + (L + dt S) d), L = I[lambda^{j+1}](Y),
// S = I[lambda^{j+1} d](Y).
template <typename T, typename SL>
struct AdjointOp {
    const SL *__restrict__ lin;
    const T *__restrict__ dv;
    const T *__restrict__ Y;
    SL *__restrict__ lout;
    unsigned N;
    T dt;
    __device__ void disp(unsigned i, T *d) const {
        d[0] = ld<T>(Y, i);
        d[1] = ld<T>(Y, N + i);
        d[2] = ld<T>(Y, 2 * N + i);
    }
    // stage loads lambda and div v; staged forms the pair (lambda, lambda div v)
    __device__ void stage(unsigned pl, unsigned i, T *x) const {
        x[0] = ld<T>(lin + pl, i);
        x[1] = ld<T>(dv + pl, i);
    }
    __device__ void staged(T *x) const { x[1] = x[0] * x[1]; }
    struct Pre {
        T d;
    };
    __device__ Pre pre(unsigned i) const { return Pre{ld<T>(dv, i)}; }
    __device__ T value(const Pre &p, const T *a) const {
        const T L = a[0], S = a[1];
        return L + (T)0.5 * dt * (S + (L + dt * S) * p.d);
    }
    __device__ void finish(unsigned i, const Pre &p, const T *a) const { st(lout, i, value(p, a)); }
};

// Last adjoint step (j = 0) fused with the time integral: lambda^0 as above,
// then b = sum_j a_j lambda^j grad m^j from lambda^0 (in registers) and the
// stored lambda^1..nt; the history reads overlap the gather-bound step.
// lam and gm point at slice 0; slice j starts j N (j 3N) elements further.
template <typename T, typename SL>
struct AdjointAccumOp {
    AdjointOp<T, SL> step;
    const SL *__restrict__ lam;  // history [nt+1][N]
    const T *__restrict__ gm;   // [nt+1][3][N]
    T *__restrict__ b;
    int nt;
    T a_end, a_mid;
    __device__ void disp(unsigned i, T *d) const { step.disp(i, d); }
    __device__ void stage(unsigned pl, unsigned i, T *x) const { step.stage(pl, i, x); }
    __device__ void staged(T *x) const { step.staged(x); }
    using Pre = typename AdjointOp<T, SL>::Pre;
    __device__ Pre pre(unsigned i) const { return step.pre(i); }
    __device__ void finish(unsigned i, const Pre &p, const T *a) const {
        const unsigned N = step.N;
        T al = a_end * step.value(p, a);
        T b1 = al * ld<T>(gm, i), b2 = al * ld<T>(gm, N + i), b3 = al * ld<T>(gm, 2 * N + i);
        const SL *l = lam;
        const T *g = gm;
        for (int j = 1; j <= nt; ++j) {
            l += N;
            g += 3 * (size_t)N;
            al = (j == nt ? a_end : a_mid) * ld<T>(l, i);
            b1 += al * ld<T>(g, i);
            b2 += al * ld<T>(g, N + i);
            b3 += al * ld<T>(g, 2 * N + i);
        }
        st(b, i, b1);
        st(b, N + i, b2);
        st(b, 2 * N + i, b3);
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
    unsigned N;
    T coef, sign;
    __device__ void disp(unsigned i, T *d) const {
        d[0] = ld<T>(X, i);
        d[1] = ld<T>(X, N + i);
        d[2] = ld<T>(X, 2 * N + i);
    }
    __device__ void stage(unsigned pl, unsigned i, T *x) const { x[0] = ld<T>(qin + pl, i); }
    __device__ void staged(T *) const {}
    __device__ const SQ *direct_src(unsigned pl) const { return qin + pl; }
    struct Pre {
        T f;
    };
    __device__ Pre pre(unsigned i) const {
        return Pre{-(ld<T>(gm, i) * ld<T>(vt, i) + ld<T>(gm, N + i) * ld<T>(vt, N + i) +
                     ld<T>(gm, 2 * N + i) * ld<T>(vt, 2 * N + i))};
    }
    __device__ void finish(unsigned i, const Pre &p, const T *a) const { st(qout, i, sign * (a[0] + coef * p.f)); }
};

template <>
struct DirectStage<InterpOp<float, float, float>> {
    static constexpr bool value = true;
};
template <>
struct DirectStage<IncStateOp<float, float>> {
    static constexpr bool value = true;
};

// Final condition of the adjoint: lambda(1) = mR - m(1).
template <typename T, typename S>
__global__ __launch_bounds__(kSlThreads) void k_adjoint_init(long long N, const T *__restrict__ mR,
                                                             const T *__restrict__ m, S *__restrict__ lam) {
    const long long idx = (long long)blockIdx.x * kSlThreads + threadIdx.x;
    if (idx >= N) return;
    store_as(lam, idx, mR[idx] - m[idx]);
}

// out = in, converted between storage types (FP16 storage <-> the boundary type)
template <typename T, typename SI, typename SO>
__global__ __launch_bounds__(kSlThreads) void k_convert(long long N, const SI *__restrict__ in, SO *__restrict__ out) {
    const long long idx = (long long)blockIdx.x * kSlThreads + threadIdx.x;
    if (idx >= N) return;
    store_as(out, idx, load_as<T>(in, idx));
}

template <typename T, typename S>
__global__ __launch_bounds__(kSlThreads) void k_incstate_init(long long N, T hdt, const T *__restrict__ gm,
                                                              const T *__restrict__ vt, S *__restrict__ q) {
    const long long idx = (long long)blockIdx.x * kSlThreads + threadIdx.x;
    if (idx >= N) return;
    const T f = -(gm[idx] * vt[idx] + gm[N + idx] * vt[N + idx] + gm[2 * N + idx] * vt[2 * N + idx]);
    store_as(q, idx, hdt * f);
}

// The incremental state's first source for several problems in one launch
// (problem p owns blocks start .. start + its block count - 1).
template <typename T, typename S>
struct InitEntry {
    long long N;
    T hdt;
    const T *gm, *vt;
    S *q;
    int start;
};
template <typename T, typename S>
__global__ __launch_bounds__(kSlThreads) void k_incstate_init_multi(const InitEntry<T, S> *__restrict__ tab,
                                                                    int nprob) {
    int p = 0;
    while (p + 1 < nprob && tab[p + 1].start <= (int)blockIdx.x) ++p;
    const InitEntry<T, S> e = tab[p];
    const long long idx = (long long)((int)blockIdx.x - e.start) * kSlThreads + threadIdx.x;
    if (idx >= e.N) return;
    const long long N = e.N;
    const T f = -(e.gm[idx] * e.vt[idx] + e.gm[N + idx] * e.vt[N + idx] + e.gm[2 * N + idx] * e.vt[2 * N + idx]);
    store_as(e.q, idx, e.hdt * f);
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n) { return (unsigned)((n + kSlThreads - 1) / kSlThreads); }

// LDS nodes of one launch: the largest box of the displacement field (box),
// at most 64 KB, and none when staging is switched off (g.lds_cap = 0).
template <typename T, int NF>
static int launch_cap(const PGrid &g, int box) {
    const int hard = kLdsBytes / (NF * (int)sizeof(T)) - 1;  // and the spare node
    int cap = box < hard ? box : hard;
    return cap < g.lds_cap ? cap : g.lds_cap;
}

template <typename T, int NF, int SHAPE, class Op>
static void launch_sl_shape(const PGrid &g, int order, const Op &op, hipStream_t s) {
    const unsigned nb = (unsigned)(g.tx * g.ty * g.tz);
    const size_t lds = g.lds_cap > 0 ? (size_t)(g.lds_cap + 1) * NF * sizeof(T) : 0;
    if (order == 3)
        hipLaunchKernelGGL((k_sl<T, 3, NF, SHAPE, Op>), dim3(nb), dim3(kSlThreads), lds, s, g, op,
                           (const SlEntry<Op> *)nullptr, 0, 0);
    else
        hipLaunchKernelGGL((k_sl<T, 1, NF, SHAPE, Op>), dim3(nb), dim3(kSlThreads), lds, s, g, op,
                           (const SlEntry<Op> *)nullptr, 0, 0);
}

template <typename T, int NF, class Op>
static void launch_sl(PGrid g, int order, SlBox box, const Op &op, hipStream_t s) {
    g.lds_cap = launch_cap<T, NF>(g, box.cap);
    g.tbox = box.tiles;
    switch (g.shape) {
        case TILE_8x8x16: launch_sl_shape<T, NF, TILE_8x8x16>(g, order, op, s); break;
        case TILE_8x16x16: launch_sl_shape<T, NF, TILE_8x16x16>(g, order, op, s); break;
        default: launch_sl_shape<T, NF, TILE_4x8x32>(g, order, op, s); break;
    }
}

long long sl_box_words(const Grid &g) {
    const int dims[3][3] = {{4, 8, 32}, {8, 8, 16}, {8, 16, 16}};
    long long most = 0;
    for (const auto &d : dims) {
        const long long t = (long long)((g.n1 + d[0] - 1) / d[0]) * ((g.n2 + d[1] - 1) / d[1]) *
                            ((g.n3 + d[2] - 1) / d[2]);
        most = t > most ? t : most;
    }
    return 8 * most;
}

template <typename T>
void sl_box_volume(const Grid &gg, int order, const T *D, double a, const double b[3], unsigned *out,
                   unsigned *slots, int *tiles, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_VECTOR, 3.0 * sizeof(T) * g.N);
    const unsigned nb = (unsigned)(g.tx * g.ty * g.tz);
    hipLaunchKernelGGL(k_zero_slots, dim3(kBoxSlots / 256), dim3(256), 0, s, slots);
#define MIREG_BOX(ORD, SH)                                                                                     \
    hipLaunchKernelGGL((k_box<T, ORD, SH>), dim3(nb), dim3(kSlThreads), 0, s, g, D, (T)a, (T)b[0], (T)b[1], \
                       (T)b[2], slots, tiles)
    if (order == 3) {
        switch (g.shape) {
            case TILE_8x8x16: MIREG_BOX(3, TILE_8x8x16); break;
            case TILE_8x16x16: MIREG_BOX(3, TILE_8x16x16); break;
            default: MIREG_BOX(3, TILE_4x8x32); break;
        }
    } else {
        switch (g.shape) {
            case TILE_8x8x16: MIREG_BOX(1, TILE_8x8x16); break;
            case TILE_8x16x16: MIREG_BOX(1, TILE_8x16x16); break;
            default: MIREG_BOX(1, TILE_4x8x32); break;
        }
    }
#undef MIREG_BOX
    hipLaunchKernelGGL(k_max_slots, dim3(1), dim3(256), 0, s, slots, out);
}

template <typename T>
void departure(const Grid &gg, int order, int sign, double dt, const T *v, T *disp, SlBox box, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_DEPARTURE, 6.0 * g.N * sizeof(T));
    DepartureOp<T> op{v, disp, (unsigned)g.N, (T)(sign * dt), (T)departure_ih(gg, 0), (T)departure_ih(gg, 1),
                      (T)departure_ih(gg, 2)};
    launch_sl<T, 3>(g, order, box, op, s);
}

template <typename T, typename SI, typename SO>
void interp_field(const Grid &gg, int order, const SI *f, const T *disp, SO *out, SlBox box, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INTERP, (3.0 * sizeof(T) + sizeof(SI) + sizeof(SO)) * g.N);
    InterpOp<T, SI, SO> op{f, disp, out, (unsigned)g.N};
    launch_sl<T, 1>(g, order, box, op, s);
}

template <typename T, typename S>
void adjoint_init(const Grid &g, const T *mR, const T *m, S *lam, hipStream_t s) {
    HookScope hs(K_ADJ_INIT, (2.0 * sizeof(T) + sizeof(S)) * g.N);
    hipLaunchKernelGGL((k_adjoint_init<T, S>), dim3(blocks_for(g.N)), dim3(kSlThreads), 0, s, g.N, mR, m, lam);
}

template <typename T, typename SI, typename SO>
void convert_field(long long n, const SI *in, SO *out, hipStream_t s) {
    HookScope hs(K_VECTOR, (double)(sizeof(SI) + sizeof(SO)) * n);
    hipLaunchKernelGGL((k_convert<T, SI, SO>), dim3(blocks_for(n)), dim3(kSlThreads), 0, s, n, in, out);
}

template <typename T, typename S>
void adjoint_step(const Grid &gg, int order, double dt, const S *lam_in, const T *d, const T *Y, S *lam_out,
                  SlBox box, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_ADJ_STEP, (4.0 * sizeof(T) + 2.0 * sizeof(S)) * g.N);
    AdjointOp<T, S> op{lam_in, d, Y, lam_out, (unsigned)g.N, (T)dt};
    launch_sl<T, 2>(g, order, box, op, s);
}

template <typename T, typename S>
void adjoint_step_accumulate(const Grid &gg, int order, double dt, int nt, const S *lam, const T *d,
                             const T *Y, const T *gradm, T *b, SlBox box, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_ADJ_ACC, ((4.0 + 3.0 * (nt + 1) + 3.0) * sizeof(T) + (double)nt * sizeof(S)) * g.N);
    const unsigned N = (unsigned)g.N;
    AdjointOp<T, S> step{lam + N, d, Y, nullptr, N, (T)dt};
    AdjointAccumOp<T, S> op{step, lam, gradm, b, nt, (T)(0.5 * dt), (T)dt};
    launch_sl<T, 2>(g, order, box, op, s);
}

template <typename T, typename S>
void incstate_init(const Grid &g, double dt, const T *gradm0, const T *vt, S *q, hipStream_t s) {
    HookScope hs(K_INC_INIT, 6.0 * sizeof(T) * g.N + sizeof(S) * g.N);
    hipLaunchKernelGGL((k_incstate_init<T, S>), dim3(blocks_for(g.N)), dim3(kSlThreads), 0, s, g.N,
                       (T)(0.5 * dt), gradm0, vt, q);
}

template <typename T, typename S>
void incstate_step(const Grid &gg, int order, double coef, double sign, const S *q_in, const T *X,
                   const T *gradm_next, const T *vt, S *q_out, SlBox box, hipStream_t s) {
    const PGrid g = pgrid(gg);
    HookScope hs(K_INC_STEP, 9.0 * sizeof(T) * g.N + 2.0 * sizeof(S) * g.N);
    IncStateOp<T, S> op{q_in, X, gradm_next, vt, q_out, (unsigned)g.N, (T)coef, (T)sign};
    launch_sl<T, 1>(g, order, box, op, s);
}

// ---- batched GN matvec transport: one launch per step across problems ----
// Table layout in device memory: init entries, then nt incremental-state
// step tables, nt - 1 adjoint step tables and one accumulate table, each
// nprob entries, every table 256-byte aligned.
namespace {
constexpr size_t kTabAlign = 256;
size_t tab_round(size_t b) { return (b + kTabAlign - 1) / kTabAlign * kTabAlign; }
template <typename T, typename S>
struct BatchLayout {
    size_t init, inc, adj, acc, total;
    BatchLayout(int nprob, int nt) {
        init = 0;
        inc = tab_round(sizeof(InitEntry<T, S>) * nprob);
        adj = inc + (size_t)nt * tab_round(sizeof(SlEntry<IncStateOp<T, S>>) * nprob);
        acc = adj + (size_t)(nt > 1 ? nt - 1 : 0) * tab_round(sizeof(SlEntry<AdjointOp<T, S>>) * nprob);
        total = acc + tab_round(sizeof(SlEntry<AdjointAccumOp<T, S>>) * nprob);
    }
    size_t inc_at(int j, int nprob) const { return inc + (size_t)j * tab_round(sizeof(SlEntry<IncStateOp<T, S>>) * nprob); }
    size_t adj_at(int j, int nprob) const {  // j = 1 .. nt-1 -> slot j - 1
        return adj + (size_t)(j - 1) * tab_round(sizeof(SlEntry<AdjointOp<T, S>>) * nprob);
    }
};

template <typename T, int NF>
PGrid entry_grid(const Grid &gg, SlBox box) {
    PGrid g = pgrid(gg);
    g.lds_cap = launch_cap<T, NF>(g, box.cap);
    g.tbox = box.tiles;
    return g;
}

template <typename T, int NF, int SHAPE, class Op>
void launch_multi_shape(const SlEntry<Op> *dtab, int nprob, int total, int order, size_t lds, hipStream_t s) {
    const PGrid none{};
    if (order == 3)
        hipLaunchKernelGGL((k_sl<T, 3, NF, SHAPE, Op, true>), dim3(total), dim3(kSlThreads), lds, s, none, Op{}, dtab,
                           nprob, total);
    else
        hipLaunchKernelGGL((k_sl<T, 1, NF, SHAPE, Op, true>), dim3(total), dim3(kSlThreads), lds, s, none, Op{}, dtab,
                           nprob, total);
}

// entries: the host copy (for the tile counts and the LDS size), dtab: the
// same entries in device memory
template <typename T, int NF, class Op>
void launch_multi(const SlEntry<Op> *entries, const SlEntry<Op> *dtab, int nprob, int order, int shape,
                  hipStream_t s) {
    int total = 0;
    size_t lds = 0;
    for (int p = 0; p < nprob; ++p) {
        const PGrid &g = entries[p].g;
        total += g.tx * g.ty * g.tz;
        const size_t l = g.lds_cap > 0 ? (size_t)(g.lds_cap + 1) * NF * sizeof(T) : 0;
        lds = l > lds ? l : lds;
    }
    switch (shape) {
        case TILE_8x8x16: launch_multi_shape<T, NF, TILE_8x8x16>(dtab, nprob, total, order, lds, s); break;
        case TILE_8x16x16: launch_multi_shape<T, NF, TILE_8x16x16>(dtab, nprob, total, order, lds, s); break;
        default: launch_multi_shape<T, NF, TILE_4x8x32>(dtab, nprob, total, order, lds, s); break;
    }
}
}  // namespace

template <typename T, typename S>
size_t batch_table_bytes(int nprob, int nt) {
    return BatchLayout<T, S>(nprob, nt).total;
}

template <typename T, typename S>
void matvec_transport_tables(const SlProblem *pr, int nprob, int nt, void *htab, void *dtab, hipStream_t s) {
    const BatchLayout<T, S> L(nprob, nt);
    char *h = static_cast<char *>(htab);
    const double dt = 1.0 / nt;
    int start = 0, bstart = 0;
    for (int p = 0; p < nprob; ++p) {
        const SlProblem &q = pr[p];
        const unsigned N = (unsigned)q.g.N;
        const T *gm = static_cast<const T *>(q.gradm), *vt = static_cast<const T *>(q.vt);
        const T *X = static_cast<const T *>(q.X), *Y = static_cast<const T *>(q.Y), *d = static_cast<const T *>(q.d);
        S *q0 = static_cast<S *>(q.q), *q1 = q0 + N, *lam = static_cast<S *>(q.lam);
        InitEntry<T, S> *ie = reinterpret_cast<InitEntry<T, S> *>(h + L.init);
        ie[p] = InitEntry<T, S>{q.g.N, (T)(0.5 * dt), gm, vt, q0, bstart};
        bstart += (int)blocks_for(q.g.N);
        const PGrid gx1 = entry_grid<T, 1>(q.g, q.boxX), gy2 = entry_grid<T, 2>(q.g, q.boxY);
        const int tiles = gx1.tx * gx1.ty * gx1.tz;
        S *cur = q0, *nxt = q1;
        for (int j = 0; j < nt; ++j) {
            auto *te = reinterpret_cast<SlEntry<IncStateOp<T, S>> *>(h + L.inc_at(j, nprob));
            const bool last = j == nt - 1;
            te[p].g = gx1;
            te[p].op = IncStateOp<T, S>{cur, X, gm + 3 * (size_t)(j + 1) * N, vt, last ? lam + (size_t)nt * N : nxt, N,
                                        (T)(last ? 0.5 * dt : dt), (T)(last ? -1.0 : 1.0)};
            te[p].start = start;
            S *t = cur;
            cur = nxt;
            nxt = t;
        }
        for (int j = nt - 1; j >= 1; --j) {
            auto *ae = reinterpret_cast<SlEntry<AdjointOp<T, S>> *>(h + L.adj_at(j, nprob));
            ae[p].g = gy2;
            ae[p].op = AdjointOp<T, S>{lam + (size_t)(j + 1) * N, d, Y, lam + (size_t)j * N, N, (T)dt};
            ae[p].start = start;
        }
        auto *ce = reinterpret_cast<SlEntry<AdjointAccumOp<T, S>> *>(h + L.acc);
        ce[p].g = gy2;
        ce[p].op = AdjointAccumOp<T, S>{AdjointOp<T, S>{lam + N, d, Y, nullptr, N, (T)dt}, lam, gm,
                                        static_cast<T *>(q.b), nt, (T)(0.5 * dt), (T)dt};
        ce[p].start = start;
        start += tiles;
    }
    hipMemcpyAsync(dtab, htab, L.total, hipMemcpyHostToDevice, s);
}

template <typename T, typename S>
void matvec_transport_batch(const SlProblem *pr, int nprob, int order, int nt, const void *htab, const void *dtab,
                            hipStream_t s) {
    const BatchLayout<T, S> L(nprob, nt);
    const char *h = static_cast<const char *>(htab), *dv = static_cast<const char *>(dtab);
    const int shape = pr[0].g.sl_tile;
    double Ntot = 0;
    int blocks = 0;
    for (int p = 0; p < nprob; ++p) {
        Ntot += (double)pr[p].g.N;
        blocks += (int)blocks_for(pr[p].g.N);
    }
    {
        HookScope hs(K_INC_INIT, (6.0 * sizeof(T) + sizeof(S)) * Ntot);
        hipLaunchKernelGGL((k_incstate_init_multi<T, S>), dim3(blocks), dim3(kSlThreads), 0, s,
                           reinterpret_cast<const InitEntry<T, S> *>(dv + L.init), nprob);
    }
    for (int j = 0; j < nt; ++j) {
        HookScope hs(K_INC_STEP, (9.0 * sizeof(T) + 2.0 * sizeof(S)) * Ntot);
        launch_multi<T, 1>(reinterpret_cast<const SlEntry<IncStateOp<T, S>> *>(h + L.inc_at(j, nprob)),
                           reinterpret_cast<const SlEntry<IncStateOp<T, S>> *>(dv + L.inc_at(j, nprob)), nprob, order,
                           shape, s);
    }
    for (int j = nt - 1; j >= 1; --j) {
        HookScope hs(K_ADJ_STEP, (4.0 * sizeof(T) + 2.0 * sizeof(S)) * Ntot);
        launch_multi<T, 2>(reinterpret_cast<const SlEntry<AdjointOp<T, S>> *>(h + L.adj_at(j, nprob)),
                           reinterpret_cast<const SlEntry<AdjointOp<T, S>> *>(dv + L.adj_at(j, nprob)), nprob, order,
                           shape, s);
    }
    HookScope hs(K_ADJ_ACC, ((4.0 + 3.0 * (nt + 1) + 3.0) * sizeof(T) + (double)nt * sizeof(S)) * Ntot);
    launch_multi<T, 2>(reinterpret_cast<const SlEntry<AdjointAccumOp<T, S>> *>(h + L.acc),
                       reinterpret_cast<const SlEntry<AdjointAccumOp<T, S>> *>(dv + L.acc), nprob, order, shape, s);
}

#define MIREG_INST_T(T)                                                                                   \
    template void departure<T>(const Grid &, int, int, double, const T *, T *, SlBox, hipStream_t);      \
    template void interp_field<T, T, T>(const Grid &, int, const T *, const T *, T *, SlBox, hipStream_t); \
    template void sl_box_volume<T>(const Grid &, int, const T *, double, const double *, unsigned *,     \
                                   unsigned *, int *, hipStream_t);
#define MIREG_INST(T, S)                                                                                  \
    template void adjoint_init<T, S>(const Grid &, const T *, const T *, S *, hipStream_t);              \
    template void adjoint_step<T, S>(const Grid &, int, double, const S *, const T *, const T *, S *,    \
                                     SlBox, hipStream_t);                                                 \
    template void adjoint_step_accumulate<T, S>(const Grid &, int, double, int, const S *, const T *,    \
                                                const T *, const T *, T *, SlBox, hipStream_t);          \
    template void incstate_init<T, S>(const Grid &, double, const T *, const T *, S *, hipStream_t);     \
    template void incstate_step<T, S>(const Grid &, int, double, double, const S *, const T *, const T *, \
                                      const T *, S *, SlBox, hipStream_t);                               \
    template size_t batch_table_bytes<T, S>(int, int);                                                   \
    template void matvec_transport_tables<T, S>(const SlProblem *, int, int, void *, void *, hipStream_t); \
    template void matvec_transport_batch<T, S>(const SlProblem *, int, int, int, const void *, const void *, \
                                               hipStream_t);
MIREG_INST_T(float)
MIREG_INST_T(double)
MIREG_INST(float, float)
MIREG_INST(double, double)
MIREG_INST(float, __half)
template void convert_field<float, float, __half>(long long, const float *, __half *, hipStream_t);
template void convert_field<float, __half, float>(long long, const __half *, float *, hipStream_t);
#undef MIREG_INST
#undef MIREG_INST_T

// ---------------------------------------------------------------------------
// Allocation-free interpolation (mireg_interp_noalloc): the per-tile stencil
// boxes and the box-measurement slots live in one file-scope device array
// sized for the largest supported grid (512^3: 131072 tiles of 8 ints under
// any tile shape), so a call allocates nothing.  Host code reaches the array
// only through the device address hipGetSymbolAddress returns, taken once
// per device with that device current.
constexpr long long kNoAllocTileWords = 8LL * 131072;
constexpr long long kNoAllocWords = kNoAllocTileWords + kBoxSlots + 64;
static __device__ __align__(256) int scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int *g_scratch_ptr[kMaxDevices];
thread_local std::string g_noalloc_err;

int noalloc_fail(int code, const std::string &msg) {
    g_noalloc_err = msg;
    return code;
}

bool noalloc_axis(int n) {
    return (n >= 8 && n <= 512 && (n & (n - 1)) == 0) || n == 48 || n == 80 || n == 96 || n == 160;
}

// Device address of `scratch` on the current device (looked up once per device).
int scratch_ptr(int **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return noalloc_fail(MIREG_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return noalloc_fail(MIREG_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(MIREG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<int *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MIREG_OK;
}

template <typename T>
void interp_noalloc(const Grid &g, int order, const T *f, const T *disp, T *out, int *scr, hipStream_t s) {
    int *tiles = scr;
    unsigned *slots = reinterpret_cast<unsigned *>(scr + kNoAllocTileWords);
    unsigned *vol = slots + kBoxSlots;
    const double one[3] = {1.0, 1.0, 1.0};
    // every tile's box (written tile by tile, nothing to clear); the slots
    // are cleared by a kernel inside sl_box_volume
    sl_box_volume<T>(g, order, disp, 1.0, one, vol, slots, tiles, s);
    // LDS sized for the largest box the launch allows; larger tiles gather
    // from global memory, as in every transport launch
    interp_field<T, T, T>(g, order, f, disp, out, SlBox(INT_MAX, tiles), s);
}
}  // namespace

const char *noalloc_error() { return g_noalloc_err.c_str(); }

}  // namespace mireg

extern "C" int mireg_interp_noalloc(const int n[3], int order, int dtype, const void *f, const void *disp,
                                    void *out, void *stream) {
    using namespace mireg;
    if (!n || !f || !disp || !out) return noalloc_fail(MIREG_E_ARG, "null pointer");
    for (int a = 0; a < 3; ++a)
        if (!noalloc_axis(n[a]))
            return noalloc_fail(MIREG_E_SHAPE, "grid axis " + std::to_string(n[a]) +
                                                   " unsupported (powers of two 8..512, or 48, 80, 96, 160)");
    if (order != 1 && order != 3) return noalloc_fail(MIREG_E_ARG, "interpolation order must be 1 or 3");
    if (dtype != MIREG_F32 && dtype != MIREG_F64) return noalloc_fail(MIREG_E_ARG, "dtype must be F32 or F64");
    Grid g{};
    g.n1 = n[0];
    g.n2 = n[1];
    g.n3 = n[2];
    g.k3 = n[2] / 2 + 1;
    g.N = (long long)n[0] * n[1] * n[2];
    g.NS = (long long)n[0] * n[1] * g.k3;
    g.lds_cap = INT_MAX;
    g.sl_tile = TILE_8x8x16;
    const long long need = sl_box_words(g);
    if (need > kNoAllocTileWords)
        return noalloc_fail(MIREG_E_SHAPE, "grid needs " + std::to_string(need) + " box words, scratch holds " +
                                               std::to_string(kNoAllocTileWords));
    int *scr = nullptr;
    int rc = scratch_ptr(&scr);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == MIREG_F32)
        interp_noalloc<float>(g, order, static_cast<const float *>(f), static_cast<const float *>(disp),
                              static_cast<float *>(out), scr, s);
    else
        interp_noalloc<double>(g, order, static_cast<const double *>(f), static_cast<const double *>(disp),
                               static_cast<double *>(out), scr, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return noalloc_fail(MIREG_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return MIREG_OK;
}
