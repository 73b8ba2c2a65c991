// Internal interface between the host solver and the HIP kernels.
#pragma once

#include "common.hpp"

namespace mireg {

// Kernel kinds for the per-launch statistics.
enum KernelId {
    K_R2C = 0, K_C2C_FWD, K_C2C_INV, K_X1_SCALE, K_X1_GRAD, K_X1_DIV, K_X1_PROJ, K_X1_TAIL, K_C2R,
    K_DEPARTURE, K_INTERP, K_ADJ_INIT, K_ADJ_STEP, K_ADJ_ACC, K_INC_INIT, K_INC_STEP, K_REDUCE, K_VECTOR,
    K_X1_KRYLOV, K_KRYLOV_UPDATE, K_COUNT
};
extern const char *const kKernelNames[K_COUNT];

// Optional observer of kernel launches (per-kernel event timing); set by the
// host for the duration of an entry point, null otherwise.
struct KernelHook {
    virtual void begin(int kid, double bytes) = 0;
    virtual void end() = 0;
    virtual ~KernelHook() {}
};
extern thread_local KernelHook *g_hook;
struct HookScope {
    explicit HookScope(int kid, double bytes) {
        if (g_hook) g_hook->begin(kid, bytes);
    }
    ~HookScope() {
        if (g_hook) g_hook->end();
    }
};

// Up to six field base pointers handed to one launch.
struct FieldPtrs {
    void *p[6];
};

// Spectral operators applied between the forward and inverse x1 passes.
enum SpecKind {
    SPEC_SCALE = 0,  // n -> n fields, one scalar symbol per mode
    SPEC_GRAD = 1,   // 1 -> 3
    SPEC_DIV = 2,    // 3 -> 1
    SPEC_PROJ = 3,   // 3 -> 3, K
    SPEC_TAIL = 4,   // 6 -> 3, alpha A u + K b (u in slots 0..2, b in 3..5)
    SPEC_REG = 5     // 3 -> 0, only the reduction: the regulariser of v
};
// SYM_AINV_SQRT: (alpha a(k))^(-1/2), 1 at k = 0; SYM_HIGHPASS: 0 on the modes
// a grid of half the size resolves below its Nyquist (|k_a| < n_a / 4 on every
// axis), 1 elsewhere.
// SYM_GRADSQ: |kt|^2 with the odd-symbol wavenumbers of the spectral
// gradient, so <u, SYM_GRADSQ u> = ||grad u||^2 by Parseval.
enum SymKind {
    SYM_ID = 0, SYM_A = 1, SYM_AINV = 2, SYM_LAP = 3, SYM_GAUSS = 4, SYM_AINV_SQRT = 5, SYM_HIGHPASS = 6,
    SYM_GRADSQ = 7
};

struct SpecParams {
    int sym;        // SymKind for SPEC_SCALE
    int nf;         // fields for SPEC_SCALE
    int reg;        // 1: |k|^2, 2: |k|^4
    int div;        // 0 none, 1 near-incompressible, 2 Leray
    double alpha;   // factor of A (SYM_A, SYM_AINV, SPEC_TAIL)
    double beta_v, beta_w;
    double sigma;   // Gaussian width in cells
    // Optional fused reduction (SPEC_SCALE, SPEC_TAIL): *red_out = sum_x in(x) out(x)
    // over all fields, from the spectra (Parseval); red holds one partial per
    // x1 workgroup (at most n2 (n3/2+1) / 8 + 1 doubles).
    double *red = nullptr, *red_out = nullptr;
};

// Device twiddle tables exp(-2 pi i j / n_a), j < n_a, for the three axes.
template <typename T>
struct Twiddles {
    const cx<T> *t[3];
};

// 3D pipeline: R2C(x3) -> C2C(x2) -> [x1 forward, operator, x1 inverse]
// -> C2C(x2 inverse) -> C2R(x3).  spec holds max(nin, nout) half spectra.
template <typename T>
void spectral_apply(const Grid &g, int kind, int nin, int nout, const void *const *in, T *const *out,
                    cx<T> *spec, const Twiddles<T> &tw, const SpecParams &sp, hipStream_t s);

// ---- PCG with Krylov vectors held as half spectra (all three axes
// transformed, unnormalised forward DFT; three arrays of NS modes per vector
// field).  work holds three half spectra.  The preconditioner is the
// spectral one, M^{-1}(k) = 1 / (beta_v a(k)), 1 at k = 0 (sp: reg, beta_v).
enum KrylovPass { KP_FWD = 0, KP_HESS = 1, KP_DIR = 2, KP_INV = 3 };
// KF_FIRST: the direction is z (no previous direction); KF_SQRT: the operator
// and the direction's grid field carry c = (beta_v a(k))^{-1/2} (the nested CG
// of the two-level preconditioner); KF_ZRAW: z is the given spectrum itself;
// KF_XUPD (set by the host functions below): the iterate takes alpha times
// the old direction in the pass that reads it.
enum KrylovFlags { KF_FIRST = 1, KF_SQRT = 2, KF_ZRAW = 4, KF_XUPD = 8 };
// hat = F u
template <typename T>
void krylov_forward(const Grid &g, const T *const *u, cx<T> *const *hat, cx<T> *work, const Twiddles<T> &tw,
                    hipStream_t s);
// hhat = beta_v a(k) shat + K F b (sp: reg, div, beta_v, beta_w); KF_SQRT:
// hhat = c (beta_v a(k) c shat + K F b); with sp.red / sp.red_out set,
// *red_out = sum_x s . Hs
template <typename T>
void krylov_hessian(const Grid &g, const T *const *b, const cx<T> *const *shat, cx<T> *const *hhat, cx<T> *work,
                    const Twiddles<T> &tw, const SpecParams &sp, int flags, hipStream_t s);
// The same two passes across precisions, for the tail beta_v A u + K b of an
// FP32 problem whose u spectrum must be accurate mode by mode: hat = F u
// with FP64 arithmetic from FP32 u (work: 3 FP64 half spectra), and
// hhat = beta_v a(k) shat + K F b in FP32 with the FP64 shat rounded at the
// load (no reduction).
void krylov_forward_wide(const Grid &g, const float *const *u, cx<double> *const *hat, cx<double> *work,
                         const Twiddles<double> &tw, hipStream_t s);
void krylov_hessian_wide(const Grid &g, const float *const *b, const cx<double> *const *shat,
                         cx<float> *const *hhat, cx<float> *work, const Twiddles<float> &tw, const SpecParams &sp,
                         hipStream_t s);
// xhat += alpha shat (when xhat and alpha are given and not KF_FIRST: the
// iterate's update of the previous iteration, from the old direction; alpha
// a device scalar), then shat = z + mu shat (shat not read with KF_FIRST),
// z = M^{-1} rhat (rhat itself with KF_ZRAW); s_out = F^{-1} shat
// (F^{-1} c shat with KF_SQRT)
template <typename T>
void krylov_direction(const Grid &g, const cx<T> *const *rhat, cx<T> *const *shat, double mu, int flags,
                      cx<T> *const *xhat, const double *alpha, T *const *s_out, cx<T> *work, const Twiddles<T> &tw,
                      const SpecParams &sp, hipStream_t s);
// Two-level preconditioner on spectra: rc = pc = Q_R c rf (coarse grid gc =
// gf / 2); zf = c (F_H c rf + Q_P (uc + alpha pc)) (alpha a device scalar,
// none when null) and *out = sum_x r . z (partials: kRedBlocks)
template <typename T>
void twolevel_restrict(const Grid &gf, const Grid &gc, const cx<T> *const *rf, cx<T> *const *rc, cx<T> *const *pc,
                       const SpecParams &sp, hipStream_t s);
template <typename T>
void twolevel_combine(const Grid &gf, const Grid &gc, const cx<T> *const *rf, const cx<T> *const *uc,
                      const cx<T> *const *pc, const double *alpha, cx<T> *const *zf, const SpecParams &sp,
                      double *partials, double *out, hipStream_t s);
// u = F^{-1} hat, or F^{-1} (hat + alpha shat) when shat and the device
// scalar alpha are given
template <typename T>
void krylov_inverse(const Grid &g, const cx<T> *const *hat, const cx<T> *const *shat, const double *alpha,
                    T *const *u, cx<T> *work, const Twiddles<T> &tw, hipStream_t s);
// res: device doubles.  With update: alpha = res[num] / res[0] and, when
// res[0] > 0, rhat -= alpha hhat, res[3] = alpha (0 when res[0] <= 0; the
// iterate is updated by the next krylov_direction or the final
// krylov_inverse).  Then res[1] = sum_x r . M^{-1} r and res[2] = sum_x r . r.
// partials holds 2 kRedBlocks doubles.
template <typename T>
void krylov_update(const Grid &g, bool update, int num, double *res, cx<T> *const *rhat, const cx<T> *const *hhat,
                   const SpecParams &sp, double *partials, hipStream_t s);

// ---- the Krylov passes of several problems of one grid size ----
// Pinned host and device staging for the launches' per-problem pointer
// tables: alloc() hands out a chunk (host pointer; *dev its device twin),
// upload() copies everything allocated since the last upload in one copy on
// the stream.  The owner calls reset() only when every copy it issued has
// completed (after a synchronisation of that stream).
struct TabArena {
    char *h = nullptr, *d = nullptr;
    size_t cap = 0, off = 0, sent = 0;
    bool overflow = false;
    template <class E>
    E *alloc(int n, const E **dev) {
        const size_t a = (off + 255) / 256 * 256, b = a + sizeof(E) * (size_t)n;
        if (b > cap) {
            overflow = true;
            return nullptr;
        }
        off = b;
        *dev = reinterpret_cast<const E *>(d + a);
        return reinterpret_cast<E *>(h + a);
    }
    void upload(hipStream_t s) {
        if (off > sent) hipMemcpyAsync(d + sent, h + sent, off - sent, hipMemcpyHostToDevice, s);
        sent = off;
    }
    void reset() { off = sent = 0; }
};
// For problems p < np (arrays of per-problem operands, three components each
// where a vector is meant: index 3 p + a), exactly krylov_hessian (flags 0,
// reduction into red[p] / red_out[p]), krylov_update and krylov_direction of
// each problem, in one launch per pass.  tw: the grid's twiddles.
template <typename T>
bool krylov_hessian_multi(const Grid &g, int np, const T *const *b, const cx<T> *const *shat, cx<T> *const *hhat,
                          cx<T> *const *work, double *const *red, double *const *red_out, const Twiddles<T> &tw,
                          const SpecParams &sp, TabArena &ar, hipStream_t s);
template <typename T>
bool krylov_update_multi(const Grid &g, int np, bool update, int num, double *const *res, cx<T> *const *rhat,
                         const cx<T> *const *hhat, double *const *partials, const SpecParams &sp, TabArena &ar,
                         hipStream_t s);
template <typename T>
bool krylov_direction_multi(const Grid &g, int np, const cx<T> *const *rhat, cx<T> *const *shat, const double *mu,
                            int flags, cx<T> *const *xhat, const double *const *alpha, T *const *s_out,
                            cx<T> *const *work, const Twiddles<T> &tw, const SpecParams &sp, TabArena &ar,
                            hipStream_t s);

// Spectral resampling between two grids (each axis the same or half/double
// the size): out = the trigonometric interpolant of in, truncated to the
// modes both grids resolve below their Nyquist (|k_a| < min(n_a, m_a) / 2),
// sampled on the destination grid.  spec_s / spec_d hold nf half spectra of
// the source / destination grid; tws / twd are their twiddle tables.
template <typename T>
void spectral_resample(const Grid &gs, const Grid &gd, int nf, const T *const *in, T *const *out, cx<T> *spec_s,
                       cx<T> *spec_d, const Twiddles<T> &tws, const Twiddles<T> &twd, hipStream_t s);

// ---- semi-Lagrangian transport (transport.hip) ----
// Every step kernel takes `box`: box.cap is the largest stencil box (nodes)
// of its displacement field, as sl_box_volume measures it; the launch sizes
// its LDS for that box (at most 64 KB), and tiles with a larger box gather
// from global memory, so any cap is correct and only the speed depends on
// it.  box.tiles, when not null, holds every tile's box as sl_box_volume
// wrote it for this displacement field and the current tile shape (the
// kernel then reads its box instead of reducing it); it must be exactly
// that, since a smaller box would leave stencil nodes outside the staged
// copy.
struct SlBox {
    int cap;
    const int *tiles;
    SlBox(int c = 0, const int *t = nullptr) : cap(c), tiles(t) {}
};
// Words of per-tile box storage for a grid under any tile shape.
long long sl_box_words(const Grid &g);
// Message of the last failed mireg_interp_noalloc call in this thread.
const char *noalloc_error();

// *out (device) = largest stencil box over the transport tiles for the
// displacement (a D_a) b_a in cell units; slots: 1024 device words of
// scratch; tiles (device, sl_box_words(g) ints, or null): every tile's box,
// 8 ints per tile (lowest base node per axis, highest base node per axis, 2
// unused).
template <typename T>
void sl_box_volume(const Grid &g, int order, const T *D, double a, const double b[3], unsigned *out,
                   unsigned *slots, int *tiles, hipStream_t s);
// disp = sign dt/2 (v + I[v](x + sign dt v)) / h  (cell units); the
// predictor displacement is (sign dt v_a) n_a / (2 pi)
template <typename T>
void departure(const Grid &g, int order, int sign, double dt, const T *v, T *disp, SlBox box, hipStream_t s);
// out = I[f](x + disp); f and out in storage types SI, SO (arithmetic in T)
template <typename T, typename SI, typename SO>
void interp_field(const Grid &g, int order, const SI *f, const T *disp, SO *out, SlBox box, hipStream_t s);
// Adjoint final condition: lam = mR - m(1)   (lam in storage type S)
template <typename T, typename S>
void adjoint_init(const Grid &g, const T *mR, const T *m, S *lam, hipStream_t s);
// out[i] = in[i] for i < n, converted from type SI to SO (through T)
template <typename T, typename SI, typename SO>
void convert_field(long long n, const SI *in, SO *out, hipStream_t s);
// One adjoint step: lam_out = L + dt/2 (S + (L + dt S) d), L = I[lam_in](Y), S = I[lam_in d](Y)
template <typename T, typename S>
void adjoint_step(const Grid &g, int order, double dt, const S *lam_in, const T *d, const T *Y,
                  S *lam_out, SlBox box, hipStream_t s);
// Last adjoint step fused with the time integral: lam^0 from lam^1 (in the
// history), then b = sum_j a_j lam^j grad m^j (lam^0 is not stored)
template <typename T, typename S>
void adjoint_step_accumulate(const Grid &g, int order, double dt, int nt, const S *lam, const T *d,
                             const T *Y, const T *gradm, T *b, SlBox box, hipStream_t s);
// ---- batched GN matvec transport (several problems, one launch per step) ----
// One problem's operands, as its context holds them: T fields gradm
// ([nt+1][3][N]), vt, X, Y ([3][N]) and d; q (2 N) and lam ((nt+1) N) in the
// storage type S; b ([3][N], T).  Every problem of a batch shares nt, the
// interpolation order and the tile shape g.sl_tile.
struct SlProblem {
    Grid g;
    const void *gradm, *vt, *X, *Y, *d;
    void *q, *lam, *b;
    SlBox boxX, boxY;
};
// Bytes of the step tables of a batch of nprob problems.
template <typename T, typename S>
size_t batch_table_bytes(int nprob, int nt);
// Writes the step tables into htab (host, pinned) and copies them to dtab
// (device) on s; htab must stay untouched until that copy has completed.
template <typename T, typename S>
void matvec_transport_tables(const SlProblem *pr, int nprob, int nt, void *htab, void *dtab, hipStream_t s);
// The incremental state and adjoint sweeps of every problem (what
// matvec_transport does for one): one launch per step across the problems,
// each problem's results those of its own launches.  htab/dtab: the tables
// above, for the same problems.
template <typename T, typename S>
void matvec_transport_batch(const SlProblem *pr, int nprob, int order, int nt, const void *htab, const void *dtab,
                            hipStream_t s);
// Incremental state: q0 = -dt/2 grad m^0 . vt
template <typename T, typename S>
void incstate_init(const Grid &g, double dt, const T *gradm0, const T *vt, S *q, hipStream_t s);
// q_out = sign (I[q_in](X) + coef f^{j+1}), f = -grad m^{j+1} . vt
template <typename T, typename S>
void incstate_step(const Grid &g, int order, double coef, double sign, const S *q_in, const T *X,
                   const T *gradm_next, const T *vt, S *q_out, SlBox box, hipStream_t s);

// ---- vector kernels and FP64 reductions (vec.hip) ----
// result[k] (device doubles) for k < nres; see the individual descriptions.
template <typename T>
void dot(const T *a, const T *b, long long n, double *partials, double *result, hipStream_t s);
template <typename TA, typename TB>
void sumsq_diff(const TA *a, const TB *b, long long n, double *partials, double *result,
                hipStream_t s);
// y = a x + b y
template <typename T>
void axpby(long long n, double a, const T *x, double b, T *y, hipStream_t s);
// z = x + a y  (z may alias x or y)
template <typename T>
void xpay(long long n, const T *x, double a, const T *y, T *z, hipStream_t s);
// PCG update: x += k s; r -= k Hs; result[0] = <r, r> (unweighted)
template <typename T>
void pcg_update(long long n, double k, const T *sdir, const T *Hs, T *x, T *r, double *partials,
                double *result, hipStream_t s);
// result[0] = min, result[1] = max, result[2] = count of non-finite values
template <typename T>
void minmax_nonfinite(const T *a, long long n, double *partials, double *result, hipStream_t s);
// result[0] = max_x sum_c v_c(x)^2 over a vector field of N points
template <typename T>
void max_norm2(const T *v, long long N, double *partials, double *result, hipStream_t s);
template <typename T>
void affine(long long n, const T *x, double a, double b, T *y, hipStream_t s);  // y = a x + b
template <typename T>
void fill(long long n, T val, T *y, hipStream_t s);
// Number of partial sums the reductions use.
constexpr int kRedBlocks = 1024;

}  // namespace mireg
