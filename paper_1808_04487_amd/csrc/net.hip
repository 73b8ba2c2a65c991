// Learned warm start: a periodic 3D convolutional encoder-decoder that maps
// an image pair to an initial velocity, with its training (not part of the
// paper; the solver's warm-start input is what it feeds, Sec. 3.6).
//
// Dense layers run on the matrix cores: every 3x3x3 convolution is an
// implicit GEMM (rows: 16 voxels, columns: output channels, reduction: 27
// taps x input channels) on v_mfma_f32_16x16x32_bf16 with BF16 operands and
// FP32 accumulation.  Activations are BF16, channels last ([voxel][channel]),
// so one lane's 8-value slice of the reduction is one 16-byte load.  The data
// adjoint of a convolution is the same kernel with transposed, tap-mirrored
// weights; the weight gradient is a second MFMA GEMM that reduces over voxels
// (tiles staged transposed in LDS, per-block partial sums added in a fixed
// order).  Pooling, masks, the pointwise heads and Adam are elementwise
// kernels; the spectral Gaussian and the Leray projection are the solver's
// own spectral operators (mireg_op).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mireg.h"
#include "mireg_net.h"

namespace mireg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetThreads = 256;

__device__ __forceinline__ f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Output grid (cubic, 2^lg per axis), input grid (2^lg_in; lg - 1 when the
// input is upsampled by 2 in the gather) and the number of output voxels.
struct ConvGeom {
    int lg, lg_in;
    unsigned V;
};

template <int CIN>
constexpr int conv_kpad() {
    return ((27 * CIN + 31) / 32) * 32;
}

// Input voxel read by tap (d1, d2, d3) of output voxel (i1, i2, i3):
// periodic neighbour on the output grid, halved when the input is the
// coarse grid of a nearest upsampling.
template <bool UP>
__device__ __forceinline__ unsigned tap_source(const ConvGeom &g, int i1, int i2, int i3, int tap) {
    const int m = (1 << g.lg) - 1;
    int j1 = (i1 + tap / 9 - 1) & m, j2 = (i2 + (tap / 3) % 3 - 1) & m, j3 = (i3 + tap % 3 - 1) & m;
    if (UP) {
        j1 >>= 1;
        j2 >>= 1;
        j3 >>= 1;
    }
    return ((unsigned)j1 << (2 * g.lg_in)) | ((unsigned)j2 << g.lg_in) | (unsigned)j3;
}

// out[v][co] = act(sum_{tap, ci} W[co][tap CIN + ci] in[src(v, tap)][ci] + bias[co] + res[v][co])
// W: [COUT][KPAD] BF16 (zero beyond 27 CIN).  One wave: 16 consecutive
// voxels x all COUT channels; lane l loads A rows (voxel l % 16) and the
// B columns (channel l % 16 of each 16-channel tile).
template <int CIN, int COUT, bool UP, typename OT>
__global__ __launch_bounds__(kNetThreads) void k_conv(ConvGeom g, const __bf16 *__restrict__ in,
                                                     const __bf16 *__restrict__ W, const float *__restrict__ bias,
                                                     const __bf16 *__restrict__ res, int relu, OT *__restrict__ out) {
    constexpr int KPAD = conv_kpad<CIN>();
    constexpr int NT = COUT / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned vbase = (blockIdx.x * (kNetThreads / 64) + wave) * 16u;
    if (vbase >= g.V) return;  // no barrier in this kernel
    const unsigned vrow = vbase + (lane & 15);
    const bool rowok = vrow < g.V;
    const int m = (1 << g.lg) - 1;
    const int i1 = (int)(vrow >> (2 * g.lg)), i2 = (int)(vrow >> g.lg) & m, i3 = (int)vrow & m;
    const int kq = 8 * (lane >> 4);
    f32x4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 *wrow = W + (size_t)(lane & 15) * KPAD + kq;
    for (int c = 0; c < KPAD / 32; ++c) {
        const int k0 = 32 * c + kq;
        const int tap = k0 / CIN, ci = k0 % CIN;
        bf16x8 a = {};
        if (rowok && tap < 27)
            a = *reinterpret_cast<const bf16x8 *>(in + (size_t)tap_source<UP>(g, i1, i2, i3, tap) * CIN + ci);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(wrow + (size_t)16 * j * KPAD + 32 * c);
            acc[j] = mfma16(a, b, acc[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + (lane & 15);
        const float bj = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned v = vbase + 4 * (lane >> 4) + i;
            if (v < g.V) {
                float x = acc[j][i] + bj;
                if (res) x += (float)res[(size_t)v * COUT + co];
                if (relu) x = fmaxf(x, 0.f);
                out[(size_t)v * COUT + co] = (OT)x;
            }
        }
    }
}

// Block-tiled variant of k_conv for grids of 64^3 and up: a workgroup owns a
// 4 x 4 x 16 (x1, x2, x3) tile of output voxels, stages the input it reads
// (the tile and a one-voxel halo, or the 4 x 4 x 10 coarse voxels behind it
// when the input is upsampled) once in LDS, and each wave computes four rows
// of 16 voxels (x1 = tile + wave, x2 = tile + row) x all COUT channels, so a
// B fragment serves four MFMAs and the A fragments are 16-byte LDS reads
// instead of per-tap global gathers.  Same reduction chunks in the same
// order as k_conv, hence the same results.
template <int CIN, bool UP>
struct ConvTile {
    static constexpr int E1 = UP ? 4 : 6, E2 = UP ? 4 : 6, E3 = UP ? 10 : 18;
    static constexpr int NVOX = E1 * E2 * E3;
    static constexpr int BYTES = NVOX * CIN * 2;
    // tile-relative fine index (0 .. extent + 1, halo included) -> staged index
    static __device__ __forceinline__ int at(int x) { return UP ? (x + 1) >> 1 : x; }
};
template <int CIN, int COUT, bool UP, typename OT>
__global__ __launch_bounds__(kNetThreads) void k_conv_tile(ConvGeom g, const __bf16 *__restrict__ in,
                                                          const __bf16 *__restrict__ W,
                                                          const float *__restrict__ bias,
                                                          const __bf16 *__restrict__ res, int relu,
                                                          OT *__restrict__ out) {
    using TL = ConvTile<CIN, UP>;
    constexpr int KPAD = conv_kpad<CIN>();
    constexpr int NT = COUT / 16;
    constexpr int CH = CIN / 8;  // 16-byte chunks per staged voxel
    __shared__ __align__(16) __bf16 tile[TL::NVOX * CIN];
    const int lg = g.lg, n = 1 << lg;
    const int tx3 = n >> 4, tx2 = n >> 2;
    const int b = (int)blockIdx.x;
    const int o3 = (b % tx3) << 4, o2 = ((b / tx3) % tx2) << 2, o1 = (b / (tx3 * tx2)) << 2;
    // 1. stage: staged voxel (z, y, x) is input voxel base + (z, y, x), wrapped
    {
        const int lgi = g.lg_in, mi = (1 << lgi) - 1;
        const int b1 = (UP ? o1 >> 1 : o1) - 1, b2 = (UP ? o2 >> 1 : o2) - 1, b3 = (UP ? o3 >> 1 : o3) - 1;
        for (int q = (int)threadIdx.x; q < TL::NVOX * CH; q += kNetThreads) {
            const int vox = q / CH, part = q % CH;
            const int z = vox / (TL::E2 * TL::E3), y = (vox / TL::E3) % TL::E2, x = vox % TL::E3;
            const unsigned src = ((unsigned)((b1 + z) & mi) << (2 * lgi)) | ((unsigned)((b2 + y) & mi) << lgi) |
                                 (unsigned)((b3 + x) & mi);
            *reinterpret_cast<bf16x8 *>(tile + vox * CIN + 8 * part) =
                *reinterpret_cast<const bf16x8 *>(in + (size_t)src * CIN + 8 * part);
        }
    }
    __syncthreads();
    // 2. implicit GEMM: lane l holds A rows of voxel x3 = l % 16, k-slice 8 (l / 16)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = 8 * (lane >> 4), x3 = lane & 15;
    f32x4 acc[4][NT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 *wrow = W + (size_t)(lane & 15) * KPAD + kq;
    for (int c = 0; c < KPAD / 32; ++c) {
        const int k0 = 32 * c + kq;
        const int tap = k0 / CIN, ci = k0 % CIN;
        const bool tapok = tap < 27;
        const int d1 = tap / 9, d2 = (tap / 3) % 3, d3 = tap % 3;
        bf16x8 bw[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) bw[j] = *reinterpret_cast<const bf16x8 *>(wrow + (size_t)16 * j * KPAD + 32 * c);
        const int zx = TL::at(wave + d1) * TL::E2;
        const int xx = TL::at(x3 + d3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bf16x8 a = {};
            if (tapok)
                a = *reinterpret_cast<const bf16x8 *>(tile + ((zx + TL::at(r + d2)) * TL::E3 + xx) * CIN + ci);
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[r][j] = mfma16(a, bw[j], acc[r][j]);
        }
    }
    // 3. bias, skip, ReLU; D row 4 (l / 16) + i is voxel x3 = that row
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const unsigned vrow = ((unsigned)(o1 + wave) << (2 * lg)) | ((unsigned)(o2 + r) << lg) | (unsigned)o3;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = 16 * j + (lane & 15);
            const float bj = bias ? bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned v = vrow + 4 * (lane >> 4) + i;
                float x = acc[r][j][i] + bj;
                if (res) x += (float)res[(size_t)v * COUT + co];
                if (relu) x = fmaxf(x, 0.f);
                out[(size_t)v * COUT + co] = (OT)x;
            }
        }
    }
}

// Weight gradient of k_conv: part[blk][co][tap CIN + ci] = sum over the
// block's voxels v of dz[v][co] in[src(v, tap)][ci].  Per tap, chunks of 64
// voxels of dz and of the gathered input are staged transposed in LDS
// ([channel][voxel]), so both MFMA operands are 16-byte LDS reads; each wave
// owns a set of 16x16 (co, ci) tiles.
template <int CIN, int COUT, bool UP>
__global__ __launch_bounds__(kNetThreads) void k_wgrad(ConvGeom g, const __bf16 *__restrict__ in,
                                                      const __bf16 *__restrict__ dz, unsigned vpb,
                                                      float *__restrict__ part) {
    constexpr int CINP = CIN < 16 ? 16 : CIN;
    constexpr int KPAD = conv_kpad<CIN>();
    constexpr int VB = 64, LP = VB + 8;
    constexpr int TC = CINP / 16, NTILE = (COUT / 16) * TC;
    constexpr int TPW = (NTILE + 3) / 4;
    __shared__ __align__(16) __bf16 xs[CINP * LP];
    __shared__ __align__(16) __bf16 zs[COUT * LP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned v0 = blockIdx.x * vpb;
    const unsigned v1 = v0 + vpb < g.V ? v0 + vpb : g.V;
    const int m = (1 << g.lg) - 1;
    float *out = part + (size_t)blockIdx.x * COUT * KPAD;
    for (int tap = 0; tap < 27; ++tap) {
        f32x4 acc[TPW];
#pragma unroll
        for (int s = 0; s < TPW; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (unsigned c0 = v0; c0 < v1; c0 += VB) {
            __syncthreads();  // the previous chunk's LDS reads are done
            for (int e = threadIdx.x; e < VB * (COUT / 8); e += kNetThreads) {
                const int vv = e / (COUT / 8), cg = e % (COUT / 8);
                const unsigned v = c0 + vv;
                bf16x8 val = {};
                if (v < v1) val = *reinterpret_cast<const bf16x8 *>(dz + (size_t)v * COUT + 8 * cg);
#pragma unroll
                for (int q = 0; q < 8; ++q) zs[(8 * cg + q) * LP + vv] = val[q];
            }
            for (int e = threadIdx.x; e < VB * (CINP / 8); e += kNetThreads) {
                const int vv = e / (CINP / 8), cg = e % (CINP / 8);
                const unsigned v = c0 + vv;
                bf16x8 val = {};
                if (v < v1 && 8 * cg < CIN) {
                    const int i1 = (int)(v >> (2 * g.lg)), i2 = (int)(v >> g.lg) & m, i3 = (int)v & m;
                    val = *reinterpret_cast<const bf16x8 *>(in + (size_t)tap_source<UP>(g, i1, i2, i3, tap) * CIN +
                                                            8 * cg);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) xs[(8 * cg + q) * LP + vv] = val[q];
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const int t = wave + 4 * s;
                if (t < NTILE) {
                    const int tr = t / TC, tc = t % TC;
#pragma unroll
                    for (int kk = 0; kk < VB; kk += 32) {
                        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(zs + (16 * tr + (lane & 15)) * LP + kk +
                                                                           8 * (lane >> 4));
                        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(xs + (16 * tc + (lane & 15)) * LP + kk +
                                                                           8 * (lane >> 4));
                        acc[s] = mfma16(a, b, acc[s]);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = wave + 4 * s;
            if (t < NTILE) {
                const int tr = t / TC, tc = t % TC;
                const int ci = 16 * tc + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = 16 * tr + 4 * (lane >> 4) + i;
                    if (ci < CIN) out[(size_t)co * KPAD + tap * CIN + ci] = acc[s][i];
                }
            }
        }
    }
}

// Block-tiled weight gradient for grids of 32^3 and up: the same partial
// sums as k_wgrad, reduced over the 4 x 4 x 16 voxel tiles of k_conv_tile.
// Input channels go in slices of up to 32 (blockIdx.y selects the slice).
// A workgroup walks a fixed set of tiles; per tile it stages
// dz transposed ([co][voxel]) and the input tile with its one-voxel halo
// transposed, in three copies shifted by 0, 1 and 2 voxels along x3
// ([d3][ci][z][y][x], 16 x positions per row), so that every MFMA operand of
// every tap is one aligned 16-byte LDS read and each staged value serves all
// 27 taps.  The taps are split over the waves (tap t on wave t mod 8); a
// wave's accumulators run over all tiles of its workgroup, which writes
// them once.  Reduction chunks of 32 voxels are two 16-voxel rows of a
// tile: lane group q = lane / 16 holds voxels 8 (q & 1) .. + 7 of row
// 2 chunk + q / 2.
template <int CIN, int COUT, bool UP>
struct WgradTile {
    static constexpr int CIH = CIN < 32 ? CIN : 32;     // input channels per workgroup
    static constexpr int CINP = CIH < 16 ? 16 : CIH;    // staged (zero padded)
    static constexpr int ZP = 256 + 8;       // dz row pitch (voxels)
    static constexpr int CP = 36 * 16 + 8;   // one channel of one copy: 6 x 6 rows of 16
    static constexpr int BYTES = 2 * (COUT * ZP + 3 * CINP * CP);
};
constexpr int kWgradThreads = 512;
template <int CIN, int COUT, bool UP>
__global__ __launch_bounds__(kWgradThreads) void k_wgrad_tile(ConvGeom g, const __bf16 *__restrict__ in,
                                                             const __bf16 *__restrict__ dz,
                                                             float *__restrict__ part) {
    using TL = WgradTile<CIN, COUT, UP>;
    constexpr int CIH = TL::CIH, CINP = TL::CINP, ZP = TL::ZP, CP = TL::CP;
    constexpr int KPAD = conv_kpad<CIN>();
    constexpr int NW = kWgradThreads / 64, TPW = (27 + NW - 1) / NW;
    constexpr int NR = COUT / 16, NC = CINP / 16;
    __shared__ __align__(16) __bf16 zs[COUT * ZP];
    __shared__ __align__(16) __bf16 xs[3 * CINP * CP];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lg = g.lg, lgi = g.lg_in, m = (1 << lg) - 1;
    const int tx3 = 1 << (lg - 4), tx2 = 1 << (lg - 2);
    const int ntiles = (int)(g.V >> 8);
    const int c0 = (int)blockIdx.y * CIH;  // first input channel of the slice
    // padded input channels stay zero in every copy
    if constexpr (CIH < CINP) {
        for (int q = tid; q < 3 * (CINP - CIH) * CP; q += kWgradThreads) {
            const int d = q / ((CINP - CIH) * CP), r = q % ((CINP - CIH) * CP);
            xs[(d * CINP + CIH) * CP + r] = (__bf16)0.f;
        }
    }
    f32x4 acc[TPW][NR][NC];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[i][r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tile = (int)blockIdx.x; tile < ntiles; tile += (int)gridDim.x) {
        const int o3 = (tile % tx3) << 4, o2 = ((tile / tx3) % tx2) << 2, o1 = (tile / (tx3 * tx2)) << 2;
        __syncthreads();  // the previous tile's LDS reads are done
        // 1. dz of the tile's voxel v = (z 4 + y) 16 + x, channel-major
        for (int q = tid; q < 256 * (COUT / 8); q += kWgradThreads) {
            const int v = q / (COUT / 8), cg = q % (COUT / 8);
            const unsigned src = ((unsigned)(o1 + (v >> 6)) << (2 * lg)) | ((unsigned)(o2 + ((v >> 4) & 3)) << lg) |
                                 (unsigned)(o3 + (v & 15));
            const bf16x8 val = *reinterpret_cast<const bf16x8 *>(dz + (size_t)src * COUT + 8 * cg);
#pragma unroll
            for (int k = 0; k < 8; ++k) zs[(8 * cg + k) * ZP + v] = val[k];
        }
        // 2. halo voxel (z, y, x), x < 18, is input voxel (o1, o2, o3) + (z, y, x) - 1
        //    (wrapped; its coarse parent when upsampled); copy d holds it at x - d
        for (int q = tid; q < 648 * (CIH / 8); q += kWgradThreads) {
            const int vox = q / (CIH / 8), cg = q % (CIH / 8);
            const int z = vox / 108, y = (vox / 18) % 6, x = vox % 18;
            int f1 = (o1 - 1 + z) & m, f2 = (o2 - 1 + y) & m, f3 = (o3 - 1 + x) & m;
            if (UP) {
                f1 >>= 1;
                f2 >>= 1;
                f3 >>= 1;
            }
            const unsigned src = ((unsigned)f1 << (2 * lgi)) | ((unsigned)f2 << lgi) | (unsigned)f3;
            const bf16x8 val = *reinterpret_cast<const bf16x8 *>(in + (size_t)src * CIN + c0 + 8 * cg);
            const int row = (z * 6 + y) * 16;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int xd = x - d;
                if (xd >= 0 && xd < 16) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) xs[(d * CINP + 8 * cg + k) * CP + row + xd] = val[k];
                }
            }
        }
        __syncthreads();
        // 3. per reduction chunk: the A fragments (dz) once, then every tap of the wave
        const int q4 = lane >> 4, l16 = lane & 15;
#pragma unroll 2
        for (int ch = 0; ch < 8; ++ch) {
            const int r = 2 * ch + (q4 >> 1), z = r >> 2, y = r & 3, xh = 8 * (q4 & 1);
            bf16x8 a[NR];
#pragma unroll
            for (int tr = 0; tr < NR; ++tr)
                a[tr] = *reinterpret_cast<const bf16x8 *>(zs + (16 * tr + l16) * ZP + 32 * ch + 8 * q4);
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                const int t = wave + NW * i;
                if (t < 27) {  // uniform per wave
                    const int d1 = t / 9, d2 = (t / 3) % 3, d3 = t % 3;
                    const __bf16 *xb = xs + (d3 * CINP + l16) * CP + ((z + d1) * 6 + (y + d2)) * 16 + xh;
#pragma unroll
                    for (int tc = 0; tc < NC; ++tc) {
                        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(xb + 16 * tc * CP);
#pragma unroll
                        for (int tr = 0; tr < NR; ++tr) acc[i][tr][tc] = mfma16(a[tr], b, acc[i][tr][tc]);
                    }
                }
            }
        }
    }
    // 4. partials of this workgroup: D row 4 (lane / 16) + k is co, column lane % 16 is ci
    float *out = part + (size_t)blockIdx.x * COUT * KPAD;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int t = wave + NW * i;
        if (t < 27) {
#pragma unroll
            for (int tr = 0; tr < NR; ++tr)
#pragma unroll
                for (int tc = 0; tc < NC; ++tc) {
                    const int ci = 16 * tc + (lane & 15);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int co = 16 * tr + 4 * (lane >> 4) + k;
                        if (ci < CIH) out[(size_t)co * KPAD + t * CIN + c0 + ci] = acc[i][tr][tc][k];
                    }
                }
        }
    }
}

// grad[co][tap][ci] (flat, ci < cin_f) += sum_b part[b][co][tap cin_k + ci]
// A workgroup takes 32 outputs; its 8 thread rows sum consecutive eighths
// of the partials, which are then added in row order.
__global__ __launch_bounds__(kNetThreads) void k_wgrad_finish(int nblk, int cin_k, int cin_f, int cout, int kpad,
                                                              const float *__restrict__ part,
                                                              float *__restrict__ grad) {
    __shared__ float red[kNetThreads];
    const int o = (int)threadIdx.x & 31, seg = (int)threadIdx.x >> 5;
    const int j = (int)blockIdx.x * 32 + o;
    const int per = 27 * cin_f;
    const int len = (nblk + 7) / 8, b0 = seg * len, b1 = b0 + len < nblk ? b0 + len : nblk;
    float s = 0.f;
    if (j < cout * per) {
        const int co = j / per, r = j % per, tap = r / cin_f, ci = r % cin_f;
        const size_t src = (size_t)co * kpad + tap * cin_k + ci;
        for (int b = b0; b < b1; ++b) s += part[(size_t)b * cout * kpad + src];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (seg == 0 && j < cout * per) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) t += red[32 * q + o];
        grad[j] += t;
    }
}

// Packed MFMA weights from the flat FP32 vector: W[co][tap cin_k + ci] (zero
// for ci >= cin_f and beyond 27 cin_k) and, for the data adjoint,
// WT[ci][t cout + co] = W[co][26 - t][ci] (tap t of the adjoint reads
// x - offset(26 - t) = x + offset(t)).
__global__ void k_pack_w(int cin_f, int cin_k, int cout, int kpad, const float *__restrict__ flat,
                         __bf16 *__restrict__ W) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cout * kpad) return;
    const int co = j / kpad, k = j % kpad, tap = k / cin_k, ci = k % cin_k;
    float x = 0.f;
    if (tap < 27 && ci < cin_f) x = flat[((size_t)co * 27 + tap) * cin_f + ci];
    W[j] = (__bf16)x;
}
__global__ void k_pack_wt(int cin, int cout, int kpad_t, const float *__restrict__ flat, __bf16 *__restrict__ WT) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cin * kpad_t) return;
    const int ci = j / kpad_t, k = j % kpad_t, t = k / cout, co = k % cout;
    float x = 0.f;
    if (t < 27) x = flat[((size_t)co * 27 + (26 - t)) * cin + ci];
    WT[j] = (__bf16)x;
}

// x[v] = (mT, mR, 0 x 6) in BF16
__global__ void k_pack_input(unsigned V, const float *__restrict__ mT, const float *__restrict__ mR,
                             __bf16 *__restrict__ x) {
    const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    bf16x8 val = {};
    val[0] = (__bf16)mT[v];
    val[1] = (__bf16)mR[v];
    *reinterpret_cast<bf16x8 *>(x + (size_t)v * 8) = val;
}

// out[u][c] = mean of the 8 children of coarse voxel u (fine grid 2^(lgc+1))
__global__ void k_pool2(int lgc, int C, const __bf16 *__restrict__ in, __bf16 *__restrict__ out) {
    const unsigned Vc = 1u << (3 * lgc);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Vc * (unsigned)(C / 8)) return;
    const unsigned u = j / (C / 8);
    const int cg = j % (C / 8);
    const int mc = (1 << lgc) - 1, lgf = lgc + 1;
    const int u1 = u >> (2 * lgc), u2 = (u >> lgc) & mc, u3 = u & mc;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 8; ++a) {
        const unsigned f = ((unsigned)(2 * u1 + (a >> 2)) << (2 * lgf)) | ((unsigned)(2 * u2 + ((a >> 1) & 1)) << lgf) |
                           (unsigned)(2 * u3 + (a & 1));
        const bf16x8 x = *reinterpret_cast<const bf16x8 *>(in + (size_t)f * C + 8 * cg);
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] += (float)x[q];
    }
    bf16x8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (__bf16)(s[q] * 0.125f);
    *reinterpret_cast<bf16x8 *>(out + (size_t)u * C + 8 * cg) = o;
}

// coarse[u][c] (= or +=) sum of the 8 children's fine[.][c]
__global__ void k_sumpool2(int lgc, int C, const float *__restrict__ fine, float *__restrict__ coarse, int add) {
    const unsigned Vc = 1u << (3 * lgc);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Vc * (unsigned)C) return;
    const unsigned u = j / C;
    const int c = j % C;
    const int mc = (1 << lgc) - 1, lgf = lgc + 1;
    const int u1 = u >> (2 * lgc), u2 = (u >> lgc) & mc, u3 = u & mc;
    float s = 0.f;
    for (int a = 0; a < 8; ++a) {
        const unsigned f = ((unsigned)(2 * u1 + (a >> 2)) << (2 * lgf)) | ((unsigned)(2 * u2 + ((a >> 1) & 1)) << lgf) |
                           (unsigned)(2 * u3 + (a & 1));
        s += fine[(size_t)f * C + c];
    }
    coarse[j] = add ? coarse[j] + s : s;
}

// fine[v][c] += coarse[parent(v)][c] / 8   (adjoint of the 2x2x2 mean)
__global__ void k_unpool_add(int lgf, int C, const float *__restrict__ coarse, float *__restrict__ fine) {
    const unsigned Vf = 1u << (3 * lgf);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Vf * (unsigned)C) return;
    const unsigned v = j / C;
    const int c = j % C;
    const int mf = (1 << lgf) - 1, lgc = lgf - 1;
    const unsigned u = ((unsigned)((v >> (2 * lgf)) >> 1) << (2 * lgc)) |
                       ((unsigned)(((v >> lgf) & mf) >> 1) << lgc) | (unsigned)((v & mf) >> 1);
    fine[j] += 0.125f * coarse[(size_t)u * C + c];
}

// g <- g [act > 0] (in place, FP32), dz = BF16(g); per-block sums of dz per
// channel for the bias gradient.  The grid stride is a multiple of C, so a
// thread always sees one channel.
__global__ __launch_bounds__(kNetThreads) void k_mask(unsigned total, int C, float *__restrict__ g,
                                                     const __bf16 *__restrict__ act, __bf16 *__restrict__ dz,
                                                     float *__restrict__ bpart) {
    __shared__ float red[kNetThreads];
    const unsigned stride = gridDim.x * kNetThreads;
    float s = 0.f;
    for (unsigned e = blockIdx.x * kNetThreads + threadIdx.x; e < total; e += stride) {
        const float x = (float)act[e] > 0.f ? g[e] : 0.f;
        g[e] = x;
        const __bf16 xb = (__bf16)x;
        dz[e] = xb;
        s += (float)xb;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < C) {
        float t = 0.f;
        for (int r = 0; r < kNetThreads / C; ++r) t += red[threadIdx.x + C * r];
        bpart[(size_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

// grad[c] += sum_b part[b][c]
// One workgroup per column c (kNetThreads threads): thread t sums rows
// t, t + 256, ..., then a fixed-order tree over the threads.
__global__ __launch_bounds__(kNetThreads) void k_rows_finish(int nblk, int C, const float *__restrict__ part,
                                                             float *__restrict__ grad) {
    __shared__ float red[kNetThreads];
    const int c = (int)blockIdx.x, t = (int)threadIdx.x;
    float s = 0.f;
    for (int b = t; b < nblk; b += kNetThreads) s += part[(size_t)b * C + c];
    red[t] = s;
    __syncthreads();
#pragma unroll
    for (int h = kNetThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) grad[c] += red[0];
}

// Pointwise head: out[c][v] = sum_k W[c][k] in[v][k] + b[c]   (3 outputs, FP32 weights)
__global__ void k_head_fwd(unsigned V, int C, const __bf16 *__restrict__ in, const float *__restrict__ W,
                           float *__restrict__ out) {
    const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float *b = W + 3 * C;
    float y0 = b[0], y1 = b[1], y2 = b[2];
    for (int k = 0; k < C; k += 8) {
        const bf16x8 x = *reinterpret_cast<const bf16x8 *>(in + (size_t)v * C + k);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float xv = (float)x[q];
            y0 += W[k + q] * xv;
            y1 += W[C + k + q] * xv;
            y2 += W[2 * C + k + q] * xv;
        }
    }
    out[v] = y0;
    out[V + v] = y1;
    out[2 * V + v] = y2;
}

// Adjoint of the head: dx[v][k] = sum_c W[c][k] dy[c][v]
__global__ void k_head_bwd(unsigned V, int C, const float *__restrict__ dy, const float *__restrict__ W,
                           float *__restrict__ dx) {
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= V * (unsigned)C) return;
    const unsigned v = j / C;
    const int k = j % C;
    dx[j] = W[k] * dy[v] + W[C + k] * dy[V + v] + W[2 * C + k] * dy[2 * V + v];
}

// Head weight gradient, per block over a voxel range: part[blk][p] for
// p < 3C: sum_v dy[p / C][v] in[v][p % C]; p = 3C + c: sum_v dy[c][v].
// Thread tid owns channel k = tid % C and the voxels v0 + tid / C + j (256 / C)
// of its workgroup's range; a fixed-order sum over the voxel lanes follows.
__global__ __launch_bounds__(kNetThreads) void k_head_wgrad(unsigned V, int C, unsigned vpb,
                                                            const float *__restrict__ dy,
                                                            const __bf16 *__restrict__ in,
                                                            float *__restrict__ part) {
    __shared__ float red[6][kNetThreads];
    const int tid = (int)threadIdx.x, k = tid % C, lanes = kNetThreads / C, vs = tid / C;
    const unsigned v0 = blockIdx.x * vpb, v1 = v0 + vpb < V ? v0 + vpb : V;
    float w0 = 0.f, w1 = 0.f, w2 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
    if (vs < lanes) {
        for (unsigned v = v0 + (unsigned)vs; v < v1; v += (unsigned)lanes) {
            const float a = (float)in[(size_t)v * C + k];
            const float y0 = dy[v], y1 = dy[(size_t)V + v], y2 = dy[2 * (size_t)V + v];
            w0 += y0 * a;
            w1 += y1 * a;
            w2 += y2 * a;
            b0 += y0;
            b1 += y1;
            b2 += y2;
        }
    }
    red[0][tid] = w0;
    red[1][tid] = w1;
    red[2][tid] = w2;
    red[3][tid] = b0;
    red[4][tid] = b1;
    red[5][tid] = b2;
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * (3 * C + 3);
    for (int p = tid; p < 3 * C + 3; p += kNetThreads) {
        // weights: (c, k) summed over the voxel lanes of channel k; biases:
        // output c summed over the voxel lanes of channel 0
        const int q = p < 3 * C ? p / C : 3 + (p - 3 * C), kk = p < 3 * C ? p % C : 0;
        float sum = 0.f;
        for (int l = 0; l < lanes; ++l) sum += red[q][l * C + kk];
        out[p] = sum;
    }
}

// out[c][v] = in[c][parent8(v)]  (nearest upsampling by 8, planar)
__global__ void k_up8(int lgf, const float *__restrict__ in, float *__restrict__ out) {
    const unsigned Vf = 1u << (3 * lgf);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 3 * Vf) return;
    const unsigned c = j / Vf, v = j % Vf;
    const int mf = (1 << lgf) - 1, lgc = lgf - 3;
    const unsigned u = ((unsigned)((v >> (2 * lgf)) >> 3) << (2 * lgc)) | ((unsigned)(((v >> lgf) & mf) >> 3) << lgc) |
                       (unsigned)((v & mf) >> 3);
    out[j] = in[(size_t)c * (1u << (3 * lgc)) + u];
}

// out[c][u] = sum of the 512 children of u (adjoint of k_up8)
__global__ void k_sumpool8(int lgc, const float *__restrict__ in, float *__restrict__ out) {
    const unsigned Vc = 1u << (3 * lgc);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 3 * Vc) return;
    const unsigned c = j / Vc, u = j % Vc;
    const int mc = (1 << lgc) - 1, lgf = lgc + 3;
    const unsigned Vf = 1u << (3 * lgf);
    const int u1 = u >> (2 * lgc), u2 = (u >> lgc) & mc, u3 = u & mc;
    float s = 0.f;
    for (int a = 0; a < 512; ++a) {
        const unsigned f = ((unsigned)(8 * u1 + (a >> 6)) << (2 * lgf)) | ((unsigned)(8 * u2 + ((a >> 3) & 7)) << lgf) |
                           (unsigned)(8 * u3 + (a & 7));
        s += in[(size_t)c * Vf + f];
    }
    out[j] = s;
}

__global__ void k_add(unsigned n, const float *__restrict__ x, float *__restrict__ y) {
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) y[j] += x[j];
}

// d = (v - vt) * scale
__global__ void k_scaled_diff(unsigned n, const float *__restrict__ v, const float *__restrict__ vt, float scale,
                              float *__restrict__ d) {
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) d[j] = (v[j] - vt[j]) * scale;
}

__global__ void k_adam(unsigned n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, float gscale, float lr, float c1, float c2) {
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j] * gscale;
    const float a = 0.9f * m1[j] + 0.1f * gj, b = 0.999f * m2[j] + 0.001f * gj * gj;
    m1[j] = a;
    m2[j] = b;
    p[j] -= lr * (a * c1) / (sqrtf(b * c2) + 1e-8f);
}

// Periodic Voronoi labels: value of the nearest seed (first index on ties).
__global__ void k_voronoi(int lg, int ns, const float *__restrict__ seeds, const float *__restrict__ values,
                          float *__restrict__ out) {
    const unsigned V = 1u << (3 * lg);
    const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int m = (1 << lg) - 1;
    const float two_pi = 6.283185307179586f, h = two_pi / (float)(1 << lg);
    const float x[3] = {h * (float)(v >> (2 * lg)), h * (float)((v >> lg) & m), h * (float)(v & m)};
    float best = 1e30f;
    int bi = 0;
    for (int s = 0; s < ns; ++s) {
        float d2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float d = fabsf(x[a] - seeds[3 * s + a]);
            d = fminf(d, two_pi - d);
            d2 += d * d;
        }
        if (d2 < best) {
            best = d2;
            bi = s;
        }
    }
    out[v] = values[bi];
}

inline unsigned nblocks(size_t n, int t = kNetThreads) { return (unsigned)((n + t - 1) / t); }

// ---- template dispatch over channel counts ----
// The block-tiled kernel on cubic grids of 32^3 and up whose staged input
// fits 64 KB of LDS (taking the 32^3 level too, 128 tiles, moved the 128^3
// forward pass from 0.756 to 0.737 ms, identical bits); k_conv otherwise, or always with
// MIREG_CONV_TILE=0 in the environment (the two give identical results).
inline bool conv_tile_enabled() {
    const char *e = getenv("MIREG_CONV_TILE");
    return !(e && e[0] == '0');
}
// Smallest grid (log2 of points per axis) that takes the block-tiled
// convolution; MIREG_CONV_TILE_MIN_LG overrides it (for measurements).
inline int conv_tile_min_lg() {
    const char *e = getenv("MIREG_CONV_TILE_MIN_LG");
    return e ? atoi(e) : 5;
}
template <int CIN, int COUT, bool UP, typename OT>
void conv_go(ConvGeom g, const __bf16 *in, const __bf16 *W, const float *b, const __bf16 *res, int relu, OT *out,
             hipStream_t s) {
    if constexpr (ConvTile<CIN, UP>::BYTES <= 65536) {
        if (g.lg >= conv_tile_min_lg() && g.lg >= 4 && conv_tile_enabled()) {
            const unsigned ntiles = g.V / 256u;
            hipLaunchKernelGGL((k_conv_tile<CIN, COUT, UP, OT>), dim3(ntiles), dim3(kNetThreads), 0, s, g, in, W, b,
                               res, relu, out);
            return;
        }
    }
    hipLaunchKernelGGL((k_conv<CIN, COUT, UP, OT>), dim3(nblocks(g.V, 64)), dim3(kNetThreads), 0, s, g, in, W, b, res,
                       relu, out);
}
template <int CIN, bool UP, typename OT>
bool conv_co(int cout, ConvGeom g, const __bf16 *in, const __bf16 *W, const float *b, const __bf16 *res, int relu,
             OT *out, hipStream_t s) {
    switch (cout) {
        case 16: conv_go<CIN, 16, UP, OT>(g, in, W, b, res, relu, out, s); return true;
        case 32: conv_go<CIN, 32, UP, OT>(g, in, W, b, res, relu, out, s); return true;
        case 64: conv_go<CIN, 64, UP, OT>(g, in, W, b, res, relu, out, s); return true;
        case 128: conv_go<CIN, 128, UP, OT>(g, in, W, b, res, relu, out, s); return true;
        default: return false;
    }
}
template <bool UP, typename OT>
bool conv(int cin, int cout, ConvGeom g, const __bf16 *in, const __bf16 *W, const float *b, const __bf16 *res,
          int relu, OT *out, hipStream_t s) {
    switch (cin) {
        case 8: return conv_co<8, UP, OT>(cout, g, in, W, b, res, relu, out, s);
        case 16: return conv_co<16, UP, OT>(cout, g, in, W, b, res, relu, out, s);
        case 32: return conv_co<32, UP, OT>(cout, g, in, W, b, res, relu, out, s);
        case 64: return conv_co<64, UP, OT>(cout, g, in, W, b, res, relu, out, s);
        case 128: return conv_co<128, UP, OT>(cout, g, in, W, b, res, relu, out, s);
        default: return false;
    }
}

constexpr int kWgradVB = 64;
inline void wgrad_blocks(unsigned V, int *nblk, unsigned *vpb) {
    const unsigned chunks = (V + kWgradVB - 1) / kWgradVB;
    const unsigned nb = chunks < 256 ? chunks : 256;
    const unsigned per = (chunks + nb - 1) / nb;
    *vpb = per * kWgradVB;
    *nblk = (int)((V + *vpb - 1) / *vpb);
}
// The block-tiled weight gradient on grids of 32^3 and up whose staging fits
// the LDS; k_wgrad otherwise, or always with MIREG_WGRAD_TILE=0 in the
// environment.  *nb: the number of partial rows written (the tiled kernel
// uses at most one row per tile).
inline bool wgrad_tile_enabled() {
    const char *e = getenv("MIREG_WGRAD_TILE");
    return !(e && e[0] == '0');
}
template <int CIN, int COUT, bool UP>
void wgrad_go(ConvGeom g, const __bf16 *in, const __bf16 *dz, float *part, hipStream_t s, int *nb) {
    unsigned vpb;
    wgrad_blocks(g.V, nb, &vpb);
    using TL = WgradTile<CIN, COUT, UP>;
    if constexpr (CIN % 8 == 0 && TL::BYTES <= 160 * 1024) {
        const unsigned tiles = g.V >> 8;
        if (g.lg >= 5 && wgrad_tile_enabled()) {
            if (tiles < (unsigned)*nb) *nb = (int)tiles;
            hipLaunchKernelGGL((k_wgrad_tile<CIN, COUT, UP>), dim3(*nb, CIN / TL::CIH), dim3(kWgradThreads), 0, s, g,
                               in, dz, part);
            return;
        }
    }
    hipLaunchKernelGGL((k_wgrad<CIN, COUT, UP>), dim3(*nb), dim3(kNetThreads), 0, s, g, in, dz, vpb, part);
}
template <int CIN, bool UP>
bool wgrad_co(int cout, ConvGeom g, const __bf16 *in, const __bf16 *dz, float *part, hipStream_t s, int *nb) {
    switch (cout) {
        case 16: wgrad_go<CIN, 16, UP>(g, in, dz, part, s, nb); return true;
        case 32: wgrad_go<CIN, 32, UP>(g, in, dz, part, s, nb); return true;
        case 64: wgrad_go<CIN, 64, UP>(g, in, dz, part, s, nb); return true;
        case 128: wgrad_go<CIN, 128, UP>(g, in, dz, part, s, nb); return true;
        default: return false;
    }
}
template <bool UP>
bool wgrad(int cin, int cout, ConvGeom g, const __bf16 *in, const __bf16 *dz, float *part, hipStream_t s, int *nb) {
    switch (cin) {
        case 8: return wgrad_co<8, UP>(cout, g, in, dz, part, s, nb);
        case 16: return wgrad_co<16, UP>(cout, g, in, dz, part, s, nb);
        case 32: return wgrad_co<32, UP>(cout, g, in, dz, part, s, nb);
        case 64: return wgrad_co<64, UP>(cout, g, in, dz, part, s, nb);
        case 128: return wgrad_co<128, UP>(cout, g, in, dz, part, s, nb);
        default: return false;
    }
}

inline int kpad_of(int cin) { return ((27 * cin + 31) / 32) * 32; }

}  // namespace
}  // namespace mireg

using namespace mireg;

// One 3x3x3 layer: flat offsets of W and b, channel counts (cin_k: the
// channel stride of its input activation, 8 for the padded image pair),
// packed weights for the forward pass and (except enc0) the data adjoint.
struct NetConv {
    int cin_f, cin_k, cout;
    size_t woff, boff;
    int kpad, kpad_t;
    __bf16 *W = nullptr, *WT = nullptr;
};

struct mireg_net {
    mireg_net_config cfg{};
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;
    mireg_ctx *spec = nullptr;  // spectral operators on the n^3 grid
    int lg = 0;
    int ch[4] = {0, 0, 0, 0};
    unsigned V[4] = {0, 0, 0, 0};
    long long np = 0;
    NetConv L[7];  // enc0, enc1, enc2, enc3, dec2, dec1, dec0
    size_t head_off = 0, head3_off = 0;
    float *P = nullptr, *G = nullptr, *M1 = nullptr, *M2 = nullptr;
    __bf16 *x8 = nullptr, *e[4] = {}, *p[3] = {}, *d[3] = {};
    float *w = nullptr, *vout = nullptr, *tmp = nullptr, *h3 = nullptr, *dh3 = nullptr;
    float *Gl[4] = {};
    float *du = nullptr;
    __bf16 *dz16 = nullptr;
    float *part = nullptr;
    double *partials = nullptr, *dres = nullptr, *hres = nullptr;
    int step = 0;
    bool packed = false;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    ConvGeom geom(int level, bool up) const {
        ConvGeom g;
        g.lg = lg - level;
        g.lg_in = up ? g.lg - 1 : g.lg;
        g.V = V[level];
        return g;
    }
};

namespace {

#define NET_OK(call)                                                                                          \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess) return net->fail(MIREG_E_HIP, "%s: %s", #call, hipGetErrorString(e_));          \
    } while (0)

template <typename T>
int net_alloc(mireg_net *net, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T) + 16) != hipSuccess)
        return net->fail(MIREG_E_NOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    net->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return MIREG_OK;
}

int net_check(mireg_net *net) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return net->fail(MIREG_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return MIREG_OK;
}

// Refresh the packed BF16 weights from the FP32 parameters.
int pack_weights(mireg_net *net) {
    for (int l = 0; l < 7; ++l) {
        NetConv &c = net->L[l];
        hipLaunchKernelGGL(k_pack_w, dim3(nblocks((size_t)c.cout * c.kpad)), dim3(kNetThreads), 0, net->stream,
                           c.cin_f, c.cin_k, c.cout, c.kpad, net->P + c.woff, c.W);
        if (c.WT)
            hipLaunchKernelGGL(k_pack_wt, dim3(nblocks((size_t)c.cin_f * c.kpad_t)), dim3(kNetThreads), 0,
                               net->stream, c.cin_f, c.cout, c.kpad_t, net->P + c.woff, c.WT);
    }
    net->packed = true;
    return net_check(net);
}

int conv_fwd(mireg_net *net, int l, int level, bool up, const __bf16 *in, const __bf16 *res, __bf16 *out) {
    const NetConv &c = net->L[l];
    const ConvGeom g = net->geom(level, up);
    const bool ok = up ? conv<true, __bf16>(c.cin_k, c.cout, g, in, c.W, net->P + c.boff, res, 1, out, net->stream)
                       : conv<false, __bf16>(c.cin_k, c.cout, g, in, c.W, net->P + c.boff, res, 1, out, net->stream);
    return ok ? MIREG_OK : net->fail(MIREG_E_ARG, "unsupported channels %d -> %d", c.cin_k, c.cout);
}

// Forward pass of one pair; leaves every activation in place for backward.
int forward(mireg_net *net, const float *mT, const float *mR) {
    int rc;
    if (!net->packed && (rc = pack_weights(net))) return rc;
    hipStream_t s = net->stream;
    const unsigned V0 = net->V[0], V3 = net->V[3];
    hipLaunchKernelGGL(k_pack_input, dim3(nblocks(V0)), dim3(kNetThreads), 0, s, V0, mT, mR, net->x8);
    if ((rc = conv_fwd(net, 0, 0, false, net->x8, nullptr, net->e[0]))) return rc;
    for (int l = 1; l <= 3; ++l) {
        const int C = net->ch[l - 1];
        hipLaunchKernelGGL(k_pool2, dim3(nblocks((size_t)net->V[l] * (C / 8))), dim3(kNetThreads), 0, s, net->lg - l, C,
                           net->e[l - 1], net->p[l - 1]);
        if ((rc = conv_fwd(net, l, l, false, net->p[l - 1], nullptr, net->e[l]))) return rc;
    }
    // decoder: layer 4 = dec2 (to level 2), 5 = dec1, 6 = dec0
    if ((rc = conv_fwd(net, 4, 2, true, net->e[3], net->e[2], net->d[2]))) return rc;
    if ((rc = conv_fwd(net, 5, 1, true, net->d[2], net->e[1], net->d[1]))) return rc;
    if ((rc = conv_fwd(net, 6, 0, true, net->d[1], net->e[0], net->d[0]))) return rc;
    // heads and the spectral skip
    hipLaunchKernelGGL(k_head_fwd, dim3(nblocks(V0)), dim3(kNetThreads), 0, s, V0, net->ch[0], net->d[0],
                       net->P + net->head_off, net->w);
    hipLaunchKernelGGL(k_head_fwd, dim3(nblocks(V3)), dim3(kNetThreads), 0, s, V3, net->ch[3], net->e[3],
                       net->P + net->head3_off, net->h3);
    hipLaunchKernelGGL(k_up8, dim3(nblocks((size_t)3 * V0)), dim3(kNetThreads), 0, s, net->lg, net->h3, net->tmp);
    for (int c = 0; c < 3; ++c) {
        if ((rc = mireg_op(net->spec, MIREG_OP_GAUSS, net->tmp + (size_t)c * V0, net->tmp + (size_t)c * V0,
                           net->cfg.skip_sigma)))
            return net->fail(rc, "spectral Gaussian: %s", mireg_last_error(net->spec));
    }
    hipLaunchKernelGGL(k_add, dim3(nblocks((size_t)3 * V0)), dim3(kNetThreads), 0, s, 3 * V0, net->tmp, net->w);
    if ((rc = mireg_op(net->spec, MIREG_OP_LERAY, net->w, net->vout, 0.0)))
        return net->fail(rc, "Leray projection: %s", mireg_last_error(net->spec));
    return net_check(net);
}

int mask(mireg_net *net, int level, int C, float *g, const __bf16 *act, float *bgrad) {
    const unsigned total = net->V[level] * (unsigned)C;
    unsigned nb = nblocks(total);
    if (nb > 1024) nb = 1024;
    // the bias partials reuse the weight-gradient partial buffer
    hipLaunchKernelGGL(k_mask, dim3(nb), dim3(kNetThreads), 0, net->stream, total, C, g, act, net->dz16, net->part);
    hipLaunchKernelGGL(k_rows_finish, dim3(C), dim3(kNetThreads), 0, net->stream, (int)nb, C, net->part, bgrad);
    return MIREG_OK;
}

int conv_wgrad(mireg_net *net, int l, int level, bool up, const __bf16 *in) {
    const NetConv &c = net->L[l];
    const ConvGeom g = net->geom(level, up);
    int nb = 0;
    const bool ok = up ? wgrad<true>(c.cin_k, c.cout, g, in, net->dz16, net->part, net->stream, &nb)
                       : wgrad<false>(c.cin_k, c.cout, g, in, net->dz16, net->part, net->stream, &nb);
    if (!ok) return net->fail(MIREG_E_ARG, "unsupported channels %d -> %d", c.cin_k, c.cout);
    const int n = c.cout * 27 * c.cin_f;
    hipLaunchKernelGGL(k_wgrad_finish, dim3((unsigned)(n + 31) / 32), dim3(kNetThreads), 0, net->stream, nb, c.cin_k,
                       c.cin_f, c.cout, c.kpad, net->part, net->G + c.woff);
    return MIREG_OK;
}

// du[v][ci] = data adjoint of layer l at level (stride-1 convolution with WT)
int conv_bwd_data(mireg_net *net, int l, int level) {
    const NetConv &c = net->L[l];
    const ConvGeom g = net->geom(level, false);
    const bool ok = conv<false, float>(c.cout, c.cin_f, g, net->dz16, c.WT, nullptr, nullptr, 0, net->du, net->stream);
    return ok ? MIREG_OK : net->fail(MIREG_E_ARG, "unsupported channels %d -> %d", c.cout, c.cin_f);
}

int head_backward(mireg_net *net, unsigned V, int C, const float *dy, const __bf16 *in, size_t off, float *dx) {
    hipStream_t s = net->stream;
    hipLaunchKernelGGL(k_head_bwd, dim3(nblocks((size_t)V * C)), dim3(kNetThreads), 0, s, V, C, dy, net->P + off, dx);
    unsigned nb = V / 64 < 1024 ? (V / 64 > 0 ? V / 64 : 1) : 1024;
    const unsigned vpb = (V + nb - 1) / nb;
    nb = (V + vpb - 1) / vpb;
    hipLaunchKernelGGL(k_head_wgrad, dim3(nb), dim3(kNetThreads), 0, s, V, C, vpb, dy, in, net->part);
    hipLaunchKernelGGL(k_rows_finish, dim3(3 * C + 3), dim3(kNetThreads), 0, s, (int)nb, 3 * C + 3, net->part,
                       net->G + off);
    return MIREG_OK;
}

// Loss of the last forward pass against vt; accumulates the parameter
// gradient into net->G.
int backward(mireg_net *net, const float *vt, double *loss) {
    int rc;
    hipStream_t s = net->stream;
    const unsigned V0 = net->V[0], V3 = net->V[3];
    const size_t n3 = (size_t)3 * V0;
    sumsq_diff<float, float>(net->vout, vt, (long long)n3, net->partials, net->dres, s);
    NET_OK(hipMemcpyAsync(net->hres, net->dres, sizeof(double), hipMemcpyDeviceToHost, s));
    // dv = (v - vt) / (3N); dw = Leray(dv)
    hipLaunchKernelGGL(k_scaled_diff, dim3(nblocks(n3)), dim3(kNetThreads), 0, s, (unsigned)n3, net->vout, vt,
                       (float)(1.0 / (3.0 * V0)), net->tmp);
    if ((rc = mireg_op(net->spec, MIREG_OP_LERAY, net->tmp, net->w, 0.0)))
        return net->fail(rc, "Leray projection: %s", mireg_last_error(net->spec));
    // heads
    if ((rc = head_backward(net, V0, net->ch[0], net->w, net->d[0], net->head_off, net->Gl[0]))) return rc;
    for (int c = 0; c < 3; ++c) {
        if ((rc = mireg_op(net->spec, MIREG_OP_GAUSS, net->w + (size_t)c * V0, net->tmp + (size_t)c * V0,
                           net->cfg.skip_sigma)))
            return net->fail(rc, "spectral Gaussian: %s", mireg_last_error(net->spec));
    }
    hipLaunchKernelGGL(k_sumpool8, dim3(nblocks((size_t)3 * V3)), dim3(kNetThreads), 0, s, net->lg - 3, net->tmp,
                       net->dh3);
    if ((rc = head_backward(net, V3, net->ch[3], net->dh3, net->e[3], net->head3_off, net->Gl[3]))) return rc;
    // decoder: layer l produces level lev from the level above (upsampled)
    const int dec_layer[3] = {6, 5, 4};  // dec0, dec1, dec2
    const __bf16 *dec_in[3] = {net->d[1], net->d[2], net->e[3]};
    for (int lev = 0; lev < 3; ++lev) {
        const int l = dec_layer[lev];
        const NetConv &c = net->L[l];
        if ((rc = mask(net, lev, c.cout, net->Gl[lev], net->d[lev], net->G + c.boff))) return rc;
        if ((rc = conv_wgrad(net, l, lev, true, dec_in[lev]))) return rc;
        if ((rc = conv_bwd_data(net, l, lev))) return rc;
        // d(input) at the coarse level = sum over the 8 children
        const int C = c.cin_f;
        hipLaunchKernelGGL(k_sumpool2, dim3(nblocks((size_t)net->V[lev + 1] * C)), dim3(kNetThreads), 0, s,
                           net->lg - lev - 1, C, net->du, net->Gl[lev + 1], lev + 1 == 3 ? 1 : 0);
    }
    // encoder: layer l (1..3) maps pooled level l-1 to level l
    for (int l = 3; l >= 1; --l) {
        const NetConv &c = net->L[l];
        if ((rc = mask(net, l, c.cout, net->Gl[l], net->e[l], net->G + c.boff))) return rc;
        if ((rc = conv_wgrad(net, l, l, false, net->p[l - 1]))) return rc;
        if ((rc = conv_bwd_data(net, l, l))) return rc;
        const int C = c.cin_f;
        hipLaunchKernelGGL(k_unpool_add, dim3(nblocks((size_t)net->V[l - 1] * C)), dim3(kNetThreads), 0, s,
                           net->lg - l + 1, C, net->du, net->Gl[l - 1]);
    }
    if ((rc = mask(net, 0, net->L[0].cout, net->Gl[0], net->e[0], net->G + net->L[0].boff))) return rc;
    if ((rc = conv_wgrad(net, 0, 0, false, net->x8))) return rc;
    NET_OK(hipStreamSynchronize(s));
    if (loss) *loss = 0.5 * net->hres[0] / (3.0 * V0);
    return net_check(net);
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

int mireg_net_create(const mireg_net_config *cfg, void *stream, mireg_net **out) {
    if (!cfg || !out) return MIREG_E_ARG;
    *out = nullptr;
    if (!pow2(cfg->n) || cfg->n < 16 || cfg->n > 256) return MIREG_E_SHAPE;
    for (int l = 0; l < 4; ++l) {
        const int c = cfg->channels[l];
        if (c != 16 && c != 32 && c != 64 && c != 128) return MIREG_E_ARG;
    }
    if (!(cfg->skip_sigma >= 0)) return MIREG_E_ARG;
    mireg_net *net = new (std::nothrow) mireg_net;
    if (!net) return MIREG_E_NOMEM;
    net->cfg = *cfg;
    net->stream = static_cast<hipStream_t>(stream);
    int lg = 0;
    while ((1 << lg) < cfg->n) ++lg;
    net->lg = lg;
    for (int l = 0; l < 4; ++l) {
        net->ch[l] = cfg->channels[l];
        net->V[l] = 1u << (3 * (lg - l));
    }
    const int *c = net->ch;
    // layer table in parameter order; heads after the seven 3x3x3 layers
    const int cin_f[7] = {2, c[0], c[1], c[2], c[3], c[2], c[1]};
    const int cout[7] = {c[0], c[1], c[2], c[3], c[2], c[1], c[0]};
    size_t off = 0;
    for (int l = 0; l < 7; ++l) {
        NetConv &L = net->L[l];
        L.cin_f = cin_f[l];
        L.cin_k = l == 0 ? 8 : cin_f[l];
        L.cout = cout[l];
        L.woff = off;
        off += (size_t)L.cout * 27 * L.cin_f;
        L.boff = off;
        off += L.cout;
        L.kpad = kpad_of(L.cin_k);
        L.kpad_t = kpad_of(L.cout);
    }
    net->head_off = off;
    off += 3 * c[0] + 3;
    net->head3_off = off;
    off += 3 * c[3] + 3;
    net->np = (long long)off;
    mireg_params p;
    mireg_default_params(&p);
    p.n[0] = p.n[1] = p.n[2] = cfg->n;
    p.nt = 1;
    p.dtype = MIREG_F32;
    int rc = mireg_create(&p, stream, &net->spec);
    if (rc) {
        delete net;
        return rc;
    }
    const size_t V0 = net->V[0];
    rc = net_alloc(net, &net->P, off);
    if (!rc) rc = net_alloc(net, &net->G, off);
    if (!rc) rc = net_alloc(net, &net->M1, off);
    if (!rc) rc = net_alloc(net, &net->M2, off);
    for (int l = 0; l < 7 && !rc; ++l) {
        NetConv &L = net->L[l];
        rc = net_alloc(net, &L.W, (size_t)L.cout * L.kpad);
        if (!rc && l > 0) rc = net_alloc(net, &L.WT, (size_t)L.cin_f * L.kpad_t);
    }
    if (!rc) rc = net_alloc(net, &net->x8, V0 * 8);
    for (int l = 0; l < 4 && !rc; ++l) rc = net_alloc(net, &net->e[l], (size_t)net->V[l] * c[l]);
    for (int l = 0; l < 3 && !rc; ++l) rc = net_alloc(net, &net->p[l], (size_t)net->V[l + 1] * c[l]);
    for (int l = 0; l < 3 && !rc; ++l) rc = net_alloc(net, &net->d[l], (size_t)net->V[l] * c[l]);
    for (int l = 0; l < 4 && !rc; ++l) rc = net_alloc(net, &net->Gl[l], (size_t)net->V[l] * c[l]);
    if (!rc) rc = net_alloc(net, &net->w, 3 * V0);
    if (!rc) rc = net_alloc(net, &net->vout, 3 * V0);
    if (!rc) rc = net_alloc(net, &net->tmp, 3 * V0);
    if (!rc) rc = net_alloc(net, &net->h3, 3 * (size_t)net->V[3]);
    if (!rc) rc = net_alloc(net, &net->dh3, 3 * (size_t)net->V[3]);
    // scratch sized for the largest user: data adjoints (V_l x cin), masked
    // gradients (V_l x c_l), weight-gradient and bias partials
    size_t du = 0, dz = 0, part = 0;
    for (int l = 0; l < 7; ++l) {
        const NetConv &L = net->L[l];
        const int lev = l <= 3 ? l : 6 - l;
        const size_t Vl = net->V[lev];
        if (l > 0) du = du > Vl * L.cin_f ? du : Vl * L.cin_f;
        dz = dz > Vl * L.cout ? dz : Vl * L.cout;
        int nb;
        unsigned vpb;
        wgrad_blocks((unsigned)Vl, &nb, &vpb);
        part = part > (size_t)nb * L.cout * L.kpad ? part : (size_t)nb * L.cout * L.kpad;
    }
    part = part > (size_t)1024 * 128 ? part : (size_t)1024 * 128;
    part = part > (size_t)1024 * (3 * 128 + 3) ? part : (size_t)1024 * (3 * 128 + 3);
    if (!rc) rc = net_alloc(net, &net->du, du);
    if (!rc) rc = net_alloc(net, &net->dz16, dz);
    if (!rc) rc = net_alloc(net, &net->part, part);
    if (!rc) rc = net_alloc(net, &net->partials, (size_t)kRedBlocks);
    if (!rc) rc = net_alloc(net, &net->dres, 4);
    if (!rc && hipHostMalloc((void **)&net->hres, 4 * sizeof(double)) != hipSuccess)
        rc = net->fail(MIREG_E_NOMEM, "pinned host allocation failed");
    if (!rc) {
        if (hipMemsetAsync(net->P, 0, off * sizeof(float), net->stream) != hipSuccess ||
            hipMemsetAsync(net->M1, 0, off * sizeof(float), net->stream) != hipSuccess ||
            hipMemsetAsync(net->M2, 0, off * sizeof(float), net->stream) != hipSuccess ||
            hipStreamSynchronize(net->stream) != hipSuccess)
            rc = net->fail(MIREG_E_HIP, "initialisation failed");
    }
    if (rc) {
        mireg_net_destroy(net);
        return rc;
    }
    *out = net;
    return MIREG_OK;
}

int mireg_net_destroy(mireg_net *net) {
    if (!net) return MIREG_OK;
    if (net->stream) hipStreamSynchronize(net->stream);
    for (void *p : net->allocs) hipFree(p);
    if (net->hres) hipHostFree(net->hres);
    if (net->spec) mireg_destroy(net->spec);
    delete net;
    return MIREG_OK;
}

const char *mireg_net_last_error(const mireg_net *net) { return net ? net->err.c_str() : "null network"; }

long long mireg_net_param_count(const mireg_net *net) { return net ? net->np : 0; }

int mireg_net_set_params(mireg_net *net, const float *params) {
    if (!net || !params) return MIREG_E_ARG;
    const size_t bytes = (size_t)net->np * sizeof(float);
    NET_OK(hipMemcpyAsync(net->P, params, bytes, hipMemcpyHostToDevice, net->stream));
    NET_OK(hipMemsetAsync(net->M1, 0, bytes, net->stream));
    NET_OK(hipMemsetAsync(net->M2, 0, bytes, net->stream));
    net->step = 0;
    int rc = pack_weights(net);
    if (rc) return rc;
    NET_OK(hipStreamSynchronize(net->stream));
    return MIREG_OK;
}

int mireg_net_get_params(const mireg_net *net_c, float *params) {
    mireg_net *net = const_cast<mireg_net *>(net_c);
    if (!net || !params) return MIREG_E_ARG;
    NET_OK(hipMemcpyAsync(params, net->P, (size_t)net->np * sizeof(float), hipMemcpyDeviceToHost, net->stream));
    NET_OK(hipStreamSynchronize(net->stream));
    return MIREG_OK;
}

int mireg_net_forward(mireg_net *net, const float *mT, const float *mR, float *v) {
    if (!net || !mT || !mR || !v) return MIREG_E_ARG;
    int rc = forward(net, mT, mR);
    if (rc) return rc;
    NET_OK(hipMemcpyAsync(v, net->vout, (size_t)3 * net->V[0] * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
    NET_OK(hipStreamSynchronize(net->stream));
    return net_check(net);
}

int mireg_net_loss_grad(mireg_net *net, const float *mT, const float *mR, const float *v_target, double *loss,
                        float *grad) {
    if (!net || !mT || !mR || !v_target) return MIREG_E_ARG;
    NET_OK(hipMemsetAsync(net->G, 0, (size_t)net->np * sizeof(float), net->stream));
    int rc = forward(net, mT, mR);
    if (!rc) rc = backward(net, v_target, loss);
    if (rc) return rc;
    if (grad) {
        NET_OK(hipMemcpyAsync(grad, net->G, (size_t)net->np * sizeof(float), hipMemcpyDeviceToHost, net->stream));
        NET_OK(hipStreamSynchronize(net->stream));
    }
    return MIREG_OK;
}

int mireg_net_train_step(mireg_net *net, int batch, const float *const *mT, const float *const *mR,
                         const float *const *v_target, double lr, double *loss) {
    if (!net || batch < 1 || !mT || !mR || !v_target || !(lr > 0)) return MIREG_E_ARG;
    NET_OK(hipMemsetAsync(net->G, 0, (size_t)net->np * sizeof(float), net->stream));
    double sum = 0;
    for (int i = 0; i < batch; ++i) {
        double li = 0;
        int rc = forward(net, mT[i], mR[i]);
        if (!rc) rc = backward(net, v_target[i], &li);
        if (rc) return rc;
        sum += li;
    }
    net->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, net->step)), c2 = 1.0 / (1.0 - std::pow(0.999, net->step));
    hipLaunchKernelGGL(k_adam, dim3(nblocks((size_t)net->np)), dim3(kNetThreads), 0, net->stream, (unsigned)net->np,
                       net->P, net->G, net->M1, net->M2, (float)(1.0 / batch), (float)lr, (float)c1, (float)c2);
    int rc = pack_weights(net);
    if (rc) return rc;
    NET_OK(hipStreamSynchronize(net->stream));
    if (loss) *loss = sum / batch;
    return net_check(net);
}

int mireg_net_voronoi(mireg_net *net, int ns, const float *seeds, const float *values, float *out) {
    if (!net || ns < 1 || ns > 4096 || !seeds || !values || !out) return MIREG_E_ARG;
    // seeds and values go through the weight-gradient scratch (>= 4 ns floats)
    float *dseeds = net->part, *dvalues = net->part + 3 * ns;
    NET_OK(hipMemcpyAsync(dseeds, seeds, 3 * ns * sizeof(float), hipMemcpyHostToDevice, net->stream));
    NET_OK(hipMemcpyAsync(dvalues, values, ns * sizeof(float), hipMemcpyHostToDevice, net->stream));
    hipLaunchKernelGGL(k_voronoi, dim3(nblocks(net->V[0])), dim3(kNetThreads), 0, net->stream, net->lg, ns, dseeds,
                       dvalues, out);
    NET_OK(hipStreamSynchronize(net->stream));
    return net_check(net);
}

}  // extern "C"
