// Host side of the mireg C-ABI: context and workspace, the velocity-dependent
// caches, the reduced gradient and Gauss-Newton Hessian matvec (Sec. 2.2),
// PCG (Algorithm "inner iteration") and the inexact Gauss-Newton-Krylov
// loop with Armijo line search (Algorithm "outer iteration").  Every field
// operation runs in the HIP kernels of fft.hip, transport.hip and vec.hip;
// the host only sequences launches on the context stream and reads back
// FP64 scalars.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <new>
#include <tuple>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/mireg.h"
#include "kernels.hpp"

using namespace mireg;

namespace {

// Axis lengths the FFT passes and transport kernels support: powers of two
// in [8, 512] and 48, 80, 96, 160 (3 and 5 times a power of two).
bool supported_axis(int n) {
    return (n >= 8 && n <= 512 && (n & (n - 1)) == 0) || n == 48 || n == 80 || n == 96 || n == 160;
}

struct Timers {
    bool on = false;
    double fft_ms = 0, interp_ms = 0, other_ms = 0;
    long launches = 0;
};

// Per-kernel HIP-event timing: each launch is bracketed by two events on the
// context stream; elapsed times are harvested lazily (pool of event pairs).
struct StatsHook : mireg::KernelHook {
    hipStream_t stream = nullptr;
    struct Pending {
        int kid;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> free_ev;
    std::vector<Pending> pending;
    Pending cur{};
    int depth = 0;
    struct Acc {
        long n = 0;
        double ms = 0, bytes = 0;
    } acc[mireg::K_COUNT];

    hipEvent_t take() {
        if (free_ev.empty()) {
            hipEvent_t e;
            hipEventCreate(&e);
            return e;
        }
        hipEvent_t e = free_ev.back();
        free_ev.pop_back();
        return e;
    }
    void begin(int kid, double bytes) override {
        if (depth++ > 0) return;
        if (pending.size() >= 4096) harvest();
        cur.kid = kid;
        cur.bytes = bytes;
        cur.a = take();
        cur.b = take();
        hipEventRecord(cur.a, stream);
    }
    void end() override {
        if (--depth > 0) return;
        hipEventRecord(cur.b, stream);
        pending.push_back(cur);
    }
    void harvest() {
        for (auto &p : pending) {
            hipEventSynchronize(p.b);
            float ms = 0;
            hipEventElapsedTime(&ms, p.a, p.b);
            acc[p.kid].n += 1;
            acc[p.kid].ms += ms;
            acc[p.kid].bytes += p.bytes;
            free_ev.push_back(p.a);
            free_ev.push_back(p.b);
        }
        pending.clear();
    }
    void reset() {
        harvest();
        for (auto &a : acc) a = Acc{};
    }
    ~StatsHook() override {
        harvest();
        for (hipEvent_t e : free_ev) hipEventDestroy(e);
    }
};

}  // namespace

// Krylov spectra of the spectral PCG (mireg_ctx::kspec)
enum KrylovVec { KV_X = 0, KV_R = 1, KV_S = 2, KV_H = 3, KV_Z = 4 };

struct mireg_ctx {
    mireg_params p{};
    hipStream_t stream = nullptr;
    Grid g{};
    size_t elem = 4;
    std::vector<void *> allocs;
    size_t bytes = 0;
    std::string err;

    // fields (typed at use)
    void *mT = nullptr, *mR = nullptr, *v = nullptr, *X = nullptr, *Y = nullptr;
    void *m = nullptr;      // (nt+1) N  state history
    void *gradm = nullptr;  // (nt+1) 3N
    void *d = nullptr;      // N, div v
    void *lam = nullptr;    // (nt+1) N, adjoint / incremental adjoint history
    void *q = nullptr;      // 2N, ping-pong of the incremental state
    void *b = nullptr;      // 3N, time integral of the gradient / matvec
    void *vecs = nullptr;   // kVecs x 3N work vectors
    void *spec = nullptr;   // 6 half spectra
    void *kspec = nullptr;  // 15 half spectra: x, r, s, Hs, z of the spectral PCG
    void *tw[3] = {nullptr, nullptr, nullptr};
    // FP32 contexts: FP64 twiddles and 6 FP64 half spectra for the accurate
    // spectrum of u in beta_v A u + K b, allocated on first use
    void *tw64[3] = {nullptr, nullptr, nullptr};
    cx<double> *spec64 = nullptr;
    double *partials = nullptr, *dres = nullptr;  // device reduction buffers
    double *xpart = nullptr;                      // partials of the fused spectral dot products
    double *hres = nullptr;                       // pinned host mirror of dres

    bool have_images = false;
    bool have_X = false, have_Y = false, have_state = false, have_gradm = false, have_d = false;
    // grad m^0 = grad mT does not depend on the velocity: kept until the images change
    bool have_gradm0 = false;
    SlBox box_X, box_Y;                    // stencil boxes of X and Y (largest, per tile)
    int *tbox_X = nullptr, *tbox_Y = nullptr;  // per-tile box storage of X and Y
    bool tile_boxes = true;  // hand the per-tile boxes to the transport kernels
    // two-level preconditioner: the n/2 context, its freshness, counters
    int pc_kind = MIREG_PC_SPECTRAL;
    double pc_kappa = 0.1;
    int pc_max_inner = 50;
    mireg_ctx *coarse = nullptr;
    long long vel_version = 0, coarse_vel_version = -1;
    bool coarse_images = false;
    long long coarse_matvecs = 0;
    // JSON-lines log of the GN iterations (mireg_set_log_jsonl), or null
    FILE *jlog = nullptr;
    // PCG's matvec replayed from a captured graph (per velocity and buffers)
    bool use_graphs = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t mv_exec = nullptr;
    const void *mv_in = nullptr;
    void *mv_out = nullptr;
    bool mv_spectral = false;
    int mv_flags = 0;
    long long mv_version = -1;
    Timers tm;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool stats_on = false;
    StatsHook stats;

    static constexpr int kVecs = 8;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    // every change of the velocity goes through here (the coarse problem of
    // the two-level preconditioner follows the version)
    void invalidate() {
        have_X = have_Y = have_state = have_gradm = have_d = false;
        vel_version += 1;
    }
    long long N() const { return g.N; }
    double cell() const {
        const double two_pi = 6.283185307179586476925;
        return (two_pi / g.n1) * (two_pi / g.n2) * (two_pi / g.n3);
    }
    template <typename T>
    T *f(void *p) const {
        return static_cast<T *>(p);
    }
    template <typename T>
    T *vec(int i) const {
        return static_cast<T *>(vecs) + (long long)i * 3 * g.N;
    }
    // component a of Krylov spectrum v (KV_X, KV_R, KV_S, KV_H, KV_Z)
    template <typename T>
    cx<T> *khat(int v, int a) const {
        return static_cast<cx<T> *>(kspec) + (long long)(3 * v + a) * g.NS;
    }
};

namespace {

#define HIP_OK(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return ctx->fail(MIREG_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Phase timing (only when enabled): events around a phase, synchronised.
struct Phase {
    mireg_ctx *ctx;
    int kind;  // 0 fft, 1 interp, 2 other
    Phase(mireg_ctx *c, int k) : ctx(c), kind(k) {
        if (ctx->tm.on) hipEventRecord(ctx->ev0, ctx->stream);
    }
    ~Phase() {
        if (!ctx->tm.on) return;
        hipEventRecord(ctx->ev1, ctx->stream);
        hipEventSynchronize(ctx->ev1);
        float ms = 0;
        hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        (kind == 0 ? ctx->tm.fft_ms : kind == 1 ? ctx->tm.interp_ms : ctx->tm.other_ms) += ms;
        ctx->tm.launches++;
    }
};

int check_launch(mireg_ctx *ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx->fail(MIREG_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return MIREG_OK;
}

// Read nres FP64 results back (synchronises the stream).
int readback(mireg_ctx *ctx, int nres) {
    HIP_OK(hipMemcpyAsync(ctx->hres, ctx->dres, nres * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return MIREG_OK;
}

template <typename T, typename S = T>
SpecParams spec_params(const mireg_ctx *ctx) {
    SpecParams sp{};
    sp.reg = ctx->p.reg;
    sp.div = ctx->p.div;
    sp.beta_v = ctx->p.beta_v;
    sp.beta_w = ctx->p.beta_w;
    sp.alpha = 1.0;
    sp.nf = 1;
    return sp;
}

template <typename T, typename S = T>
Twiddles<T> twiddles(const mireg_ctx *ctx) {
    Twiddles<T> t;
    for (int a = 0; a < 3; ++a) t.t[a] = static_cast<const cx<T> *>(ctx->tw[a]);
    return t;
}

template <typename T, typename S = T>
void spec(mireg_ctx *ctx, int kind, int nin, int nout, const void *const *in, T *const *out, const SpecParams &sp) {
    Phase ph(ctx, 0);
    spectral_apply<T>(ctx->g, kind, nin, nout, in, out, static_cast<cx<T> *>(ctx->spec), twiddles<T>(ctx), sp,
                      ctx->stream);
}

// ---- individual spectral operators ----
template <typename T, typename S = T>
void op_grad(mireg_ctx *ctx, const T *u, T *out) {
    const long long N = ctx->N();
    const void *in[1] = {u};
    T *o[3] = {out, out + N, out + 2 * N};
    spec<T, S>(ctx, SPEC_GRAD, 1, 3, in, o, spec_params<T>(ctx));
}
template <typename T, typename S = T>
void op_div(mireg_ctx *ctx, const T *v, T *out) {
    const long long N = ctx->N();
    const void *in[3] = {v, v + N, v + 2 * N};
    T *o[1] = {out};
    spec<T, S>(ctx, SPEC_DIV, 3, 1, in, o, spec_params<T>(ctx));
}
template <typename T, typename S = T>
void op_scale(mireg_ctx *ctx, int sym, int nf, double alpha, double sigma, const T *u, T *out) {
    const long long N = ctx->N();
    const void *in[3] = {u, u + N, u + 2 * N};
    T *o[3] = {out, out + N, out + 2 * N};
    SpecParams sp = spec_params<T>(ctx);
    sp.sym = sym;
    sp.nf = nf;
    sp.alpha = alpha;
    sp.sigma = sigma;
    spec<T, S>(ctx, SPEC_SCALE, nf, nf, in, o, sp);
}
template <typename T, typename S = T>
void op_proj(mireg_ctx *ctx, int div, const T *u, T *out) {
    const long long N = ctx->N();
    const void *in[3] = {u, u + N, u + 2 * N};
    T *o[3] = {out, out + N, out + 2 * N};
    SpecParams sp = spec_params<T>(ctx);
    sp.div = div;
    spec<T, S>(ctx, SPEC_PROJ, 3, 3, in, o, sp);
}
// out = alpha A u + K b
template <typename T, typename S = T>
void op_tail(mireg_ctx *ctx, double alpha, const T *u, const T *b, T *out) {
    const long long N = ctx->N();
    const void *in[6] = {u, u + N, u + 2 * N, b, b + N, b + 2 * N};
    T *o[3] = {out, out + N, out + 2 * N};
    SpecParams sp = spec_params<T>(ctx);
    sp.alpha = alpha;
    spec<T, S>(ctx, SPEC_TAIL, 6, 3, in, o, sp);
}

// ---- velocity-dependent caches ----
// Largest stencil box of the displacement (a D_a) b_a over the transport
// tiles, read back to the host (synchronises the stream); it sizes the LDS
// of the transport launches that use D.  0 when staging is switched off.
template <typename T>
int measure_box(mireg_ctx *ctx, const T *D, double a, const double b[3], int *tiles = nullptr) {
    if (ctx->g.lds_cap == 0) return 0;
    unsigned *dev = reinterpret_cast<unsigned *>(ctx->dres);
    // the reduction partials (4 kRedBlocks doubles) serve as the 1024 slots
    sl_box_volume<T>(ctx->g, ctx->p.interp_order, D, a, b, dev, reinterpret_cast<unsigned *>(ctx->partials),
                     tiles, ctx->stream);
    if (readback(ctx, 1) != MIREG_OK) return INT_MAX;  // every tile then takes the largest LDS
    unsigned v = 0;
    memcpy(&v, ctx->hres, sizeof v);
    return v > (unsigned)INT_MAX ? INT_MAX : (int)v;
}
template <typename T>
int box_of_displacement(mireg_ctx *ctx, const T *D) {
    const double one[3] = {1.0, 1.0, 1.0};
    return measure_box<T>(ctx, D, 1.0, one);
}
// Largest box and every tile's box of a displacement field kept for the
// velocity (X or Y), for the current tile shape.  The per-tile boxes are
// handed to the kernels only when the measurement ran to completion.
template <typename T>
SlBox tile_boxes(mireg_ctx *ctx, const T *D, int *tiles) {
    const double one[3] = {1.0, 1.0, 1.0};
    if (!ctx->tile_boxes) tiles = nullptr;
    const int cap = measure_box<T>(ctx, D, 1.0, one, tiles);
    return SlBox(cap, (cap > 0 && cap < INT_MAX) ? tiles : nullptr);
}
// Characteristic feet of one step (sign -1: X, +1: Y) from velocity v.
template <typename T>
void compute_departure(mireg_ctx *ctx, int sign, const T *v, T *out) {
    const double two_pi = 6.283185307179586476925;
    const double ih[3] = {ctx->g.n1 / two_pi, ctx->g.n2 / two_pi, ctx->g.n3 / two_pi};
    const double dt = 1.0 / ctx->p.nt;
    const int box = measure_box<T>(ctx, v, sign * dt, ih);  // predictor displacement
    Phase ph(ctx, 1);
    departure<T>(ctx->g, ctx->p.interp_order, sign, dt, v, out, box, ctx->stream);
}
template <typename T, typename S = T>
void ensure_X(mireg_ctx *ctx) {
    if (ctx->have_X) return;
    compute_departure<T>(ctx, -1, ctx->f<T>(ctx->v), ctx->f<T>(ctx->X));
    ctx->box_X = tile_boxes<T>(ctx, ctx->f<T>(ctx->X), ctx->tbox_X);
    ctx->have_X = true;
}
template <typename T, typename S = T>
void ensure_Y(mireg_ctx *ctx) {
    if (ctx->have_Y) return;
    compute_departure<T>(ctx, +1, ctx->f<T>(ctx->v), ctx->f<T>(ctx->Y));
    ctx->box_Y = tile_boxes<T>(ctx, ctx->f<T>(ctx->Y), ctx->tbox_Y);
    ctx->have_Y = true;
}
// State equation forward in time: m^0 = mT, m^{j+1} = I[m^j](X).  The state
// history is held in T in every storage mode: lam(1) = mR - m(1) is a small
// difference of O(1) values, so FP16 rounding of m would reach lam, and the
// gradient, amplified by |m| / |lam|.
template <typename T, typename S = T>
void ensure_state(mireg_ctx *ctx) {
    if (ctx->have_state) return;
    ensure_X<T, S>(ctx);
    const long long N = ctx->N();
    T *m = ctx->f<T>(ctx->m);
    hipMemcpyAsync(m, ctx->mT, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream);
    Phase ph(ctx, 1);
    for (int j = 0; j < ctx->p.nt; ++j)
        interp_field<T, T, T>(ctx->g, ctx->p.interp_order, m + j * N, ctx->f<T>(ctx->X), m + (j + 1) * N,
                              ctx->box_X, ctx->stream);
    ctx->have_state = true;
}
template <typename T, typename S = T>
void ensure_gradm(mireg_ctx *ctx) {
    if (ctx->have_gradm) return;
    ensure_state<T, S>(ctx);
    const long long N = ctx->N();
    for (int j = ctx->have_gradm0 ? 1 : 0; j <= ctx->p.nt; ++j)
        op_grad<T, S>(ctx, ctx->f<T>(ctx->m) + j * N, ctx->f<T>(ctx->gradm) + 3 * j * N);
    ctx->have_gradm = ctx->have_gradm0 = true;
}
template <typename T, typename S = T>
void ensure_d(mireg_ctx *ctx) {
    if (ctx->have_d) return;
    op_div<T, S>(ctx, ctx->f<T>(ctx->v), ctx->f<T>(ctx->d));
    ctx->have_d = true;
}


// Backward sweep shared by the adjoint and the incremental adjoint: from
// lam^nt in the history buffer, lam^j for j = nt-1..1, then the last step
// fused with the time integral b = sum_j a_j lam^j grad m^j.
template <typename T, typename S = T>
void backward_sweep(mireg_ctx *ctx, S *lam, T *b) {
    const int nt = ctx->p.nt;
    const long long N = ctx->N();
    const double dt = 1.0 / nt;
    Phase ph(ctx, 1);
    for (int j = nt - 1; j >= 1; --j)
        adjoint_step<T, S>(ctx->g, ctx->p.interp_order, dt, lam + (j + 1) * N, ctx->f<T>(ctx->d),
                           ctx->f<T>(ctx->Y), lam + j * N, ctx->box_Y, ctx->stream);
    adjoint_step_accumulate<T, S>(ctx->g, ctx->p.interp_order, dt, nt, lam, ctx->f<T>(ctx->d), ctx->f<T>(ctx->Y),
                               ctx->f<T>(ctx->gradm), b, ctx->box_Y, ctx->stream);
}

template <typename T, typename S = T>
int dot_h(mireg_ctx *ctx, const T *a, const T *b, long long n, double *out) {
    dot<T>(a, b, n, ctx->partials, ctx->dres, ctx->stream);
    int rc = readback(ctx, 1);
    if (rc) return rc;
    *out = ctx->cell() * ctx->hres[0];
    return MIREG_OK;
}

// ---- objective ----
template <typename T, typename S = T>
int impl_objective(mireg_ctx *ctx, double *J, double *mism, double *reg) {
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    ensure_state<T, S>(ctx);
    const long long N = ctx->N();
    const int nt = ctx->p.nt;
    sumsq_diff<T, T>(ctx->f<T>(ctx->m) + nt * N, ctx->f<T>(ctx->mR), N, ctx->partials, ctx->dres, ctx->stream);
    int rc = readback(ctx, 1);
    if (rc) return rc;
    const double mis = 0.5 * ctx->cell() * ctx->hres[0];
    // the regulariser beta_v/2 <A v, v> (+ beta_w/2 (||grad w||^2 + ||w||^2)
    // for the near-incompressible model, w = div v eliminated), by Parseval
    // from one forward transform of v (nothing transformed back)
    {
        const T *v = ctx->f<T>(ctx->v);
        const void *in[3] = {v, v + N, v + 2 * N};
        T *o[1] = {nullptr};
        SpecParams sp = spec_params<T>(ctx);
        sp.red = ctx->xpart;
        sp.red_out = ctx->dres;
        spec<T, S>(ctx, SPEC_REG, 3, 0, in, o, sp);
    }
    if ((rc = readback(ctx, 1))) return rc;
    const double r = ctx->cell() * ctx->hres[0];
    if (J) *J = mis + r;
    if (mism) *mism = mis;
    if (reg) *reg = r;
    return check_launch(ctx);
}

int alloc(mireg_ctx *ctx, void **p, size_t bytes);
template <typename T>
int make_twiddles_into(mireg_ctx *ctx, void *const *dst);

// out = beta_v A u + K b, the tail of the reduced gradient (u = v) and of
// the matvec entry point (u = vt).  An FP32 forward transform of u leaves
// roundoff of about eps ||u|| on every mode, which A multiplies by up to
// 3 (n/2)^2 (H1; its square for H2): at 256^3 that alone is 2.5e-5 of the
// gradient.  In FP32 contexts the spectrum of u is therefore formed with
// FP64 arithmetic (from the FP32 field) and read by the FP32 operator pass
// mode by mode; the spectrum of b, the multipliers and the inverse
// transform stay FP32, whose errors are relative to their own output.  The
// FP64 twiddles and 6 FP64 half spectra are allocated on first use; the
// Krylov slot KV_H is scratch outside PCG.  (PCG keeps its directions as
// spectra and never transforms them forward.)
template <typename T>
int ensure_tail64(mireg_ctx *ctx) {
    if (std::is_same<T, double>::value || ctx->spec64) return MIREG_OK;
    const long long NS = ctx->g.NS;
    const int n[3] = {ctx->g.n1, ctx->g.n2, ctx->g.n3};
    int rc;
    for (int a = 0; a < 3; ++a)
        if ((rc = alloc(ctx, &ctx->tw64[a], (size_t)n[a] * sizeof(cx<double>)))) return rc;
    if ((rc = make_twiddles_into<double>(ctx, ctx->tw64))) return rc;
    if ((rc = alloc(ctx, (void **)&ctx->spec64, (size_t)6 * NS * sizeof(cx<double>)))) return rc;
    return MIREG_OK;
}

template <typename T, typename S = T>
int accurate_tail(mireg_ctx *ctx, const T *u, const T *b, T *out) {
    if constexpr (std::is_same<T, double>::value) {
        op_tail<T, S>(ctx, ctx->p.beta_v, u, b, out);
        return MIREG_OK;
    } else {
        const long long N = ctx->N(), NS = ctx->g.NS;
        int rc;
        if ((rc = ensure_tail64<T>(ctx))) return rc;
        Phase ph(ctx, 0);
        const T *up[3] = {u, u + N, u + 2 * N}, *bp[3] = {b, b + N, b + 2 * N};
        cx<double> *uh[3] = {ctx->spec64 + 3 * NS, ctx->spec64 + 4 * NS, ctx->spec64 + 5 * NS};
        Twiddles<double> tw64;
        for (int a = 0; a < 3; ++a) tw64.t[a] = static_cast<const cx<double> *>(ctx->tw64[a]);
        krylov_forward_wide(ctx->g, up, uh, ctx->spec64, tw64, ctx->stream);
        cx<T> *hh[3] = {ctx->khat<T>(KV_H, 0), ctx->khat<T>(KV_H, 1), ctx->khat<T>(KV_H, 2)};
        const cx<double> *uhc[3] = {uh[0], uh[1], uh[2]};
        krylov_hessian_wide(ctx->g, bp, uhc, hh, static_cast<cx<T> *>(ctx->spec), twiddles<T>(ctx),
                            spec_params<T>(ctx), ctx->stream);
        const cx<T> *hhc[3] = {hh[0], hh[1], hh[2]};
        T *op[3] = {out, out + N, out + 2 * N};
        krylov_inverse<T>(ctx->g, hhc, nullptr, nullptr, op, static_cast<cx<T> *>(ctx->spec), twiddles<T>(ctx),
                          ctx->stream);
        return MIREG_OK;
    }
}

// ---- reduced gradient ----
template <typename T, typename S = T>
int impl_gradient(mireg_ctx *ctx, T *g, double *gnorm) {
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    ensure_state<T, S>(ctx);
    ensure_gradm<T, S>(ctx);
    ensure_d<T, S>(ctx);
    ensure_Y<T, S>(ctx);
    const long long N = ctx->N();
    const int nt = ctx->p.nt;
    S *lam = ctx->f<S>(ctx->lam);
    T *b = ctx->f<T>(ctx->b);
    {
        Phase ph(ctx, 2);
        adjoint_init<T, S>(ctx->g, ctx->f<T>(ctx->mR), ctx->f<T>(ctx->m) + nt * N, lam + nt * N, ctx->stream);
    }
    backward_sweep<T, S>(ctx, lam, b);
    int rc = accurate_tail<T, S>(ctx, ctx->f<T>(ctx->v), b, g);
    if (rc) return rc;
    if (gnorm) {
        double gg = 0;
        if ((rc = dot_h<T>(ctx, g, g, 3 * N, &gg))) return rc;
        *gnorm = std::sqrt(gg);
    }
    return check_launch(ctx);
}

// ---- Gauss-Newton Hessian matvec ----
// Transport part: ctx->b = the time integral of the incremental adjoint for
// the direction vt (the caches it reads are current).
template <typename T, typename S = T>
void matvec_transport(mireg_ctx *ctx, const T *vt) {
    const long long N = ctx->N();
    const int nt = ctx->p.nt;
    const double dt = 1.0 / nt;
    S *q0 = ctx->f<S>(ctx->q), *q1 = q0 + N, *lam = ctx->f<S>(ctx->lam);
    T *b = ctx->f<T>(ctx->b);
    const T *gm = ctx->f<T>(ctx->gradm);
    {
        Phase ph(ctx, 1);
        // incremental state: q^0 = mt^0 + dt/2 f^0 with mt^0 = 0
        incstate_init<T, S>(ctx->g, dt, gm, vt, q0, ctx->stream);
        S *cur = q0, *nxt = q1;
        for (int j = 0; j < nt; ++j) {
            if (j < nt - 1) {
                // q^{j+1} = I[q^j](X) + dt f^{j+1}
                incstate_step<T, S>(ctx->g, ctx->p.interp_order, dt, 1.0, cur, ctx->f<T>(ctx->X), gm + 3 * (j + 1) * N,
                                 vt, nxt, ctx->box_X, ctx->stream);
                S *t = cur;
                cur = nxt;
                nxt = t;
            } else {
                // mt(1) = I[q](X) + dt/2 f^nt; the incremental adjoint starts at lt^nt = -mt(1)
                incstate_step<T, S>(ctx->g, ctx->p.interp_order, 0.5 * dt, -1.0, cur, ctx->f<T>(ctx->X),
                                 gm + 3 * nt * N, vt, lam + nt * N, ctx->box_X, ctx->stream);
            }
        }
    }
    backward_sweep<T, S>(ctx, lam, b);
}

// Hvt = beta_v A vt + K b~: the Gauss-Newton Hessian matvec in grid space
// (eq. "hessian-matvec", Sec. 2.3.2)
template <typename T, typename S = T>
int impl_matvec(mireg_ctx *ctx, const T *vt, T *Hvt) {
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    ensure_state<T, S>(ctx);
    ensure_gradm<T, S>(ctx);
    ensure_d<T, S>(ctx);
    ensure_Y<T, S>(ctx);
    matvec_transport<T, S>(ctx, vt);
    int rc = accurate_tail<T, S>(ctx, vt, ctx->f<T>(ctx->b), Hvt);
    if (rc) return rc;
    return check_launch(ctx);
}

// Matvec of the spectral PCG: the spectrum of H s from the kept spectrum of
// s (KV_S) and the transport output, into KV_H; dres[0] = sum_x s . Hs.
// flags KF_SQRT: the nested CG's scaled operator c H c (s = c times KV_S).
template <typename T, typename S = T>
int impl_matvec_spectral(mireg_ctx *ctx, const T *s, int flags = 0) {
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    ensure_state<T, S>(ctx);
    ensure_gradm<T, S>(ctx);
    ensure_d<T, S>(ctx);
    ensure_Y<T, S>(ctx);
    matvec_transport<T, S>(ctx, s);
    const long long N = ctx->N();
    const T *b = ctx->f<T>(ctx->b);
    const T *bp[3] = {b, b + N, b + 2 * N};
    const cx<T> *sh[3] = {ctx->khat<T>(KV_S, 0), ctx->khat<T>(KV_S, 1), ctx->khat<T>(KV_S, 2)};
    cx<T> *hh[3] = {ctx->khat<T>(KV_H, 0), ctx->khat<T>(KV_H, 1), ctx->khat<T>(KV_H, 2)};
    SpecParams sp = spec_params<T>(ctx);
    sp.red = ctx->xpart;
    sp.red_out = ctx->dres;
    {
        Phase ph(ctx, 0);
        krylov_hessian<T>(ctx->g, bp, sh, hh, static_cast<cx<T> *>(ctx->spec), twiddles<T>(ctx), sp, flags,
                          ctx->stream);
    }
    return check_launch(ctx);
}

// Hessian matvec of PCG (spectral: the spectrum of H vt in KV_H, Hvt unused,
// and dres[0] = sum_x vt . Hvt) or of the entry point (Hvt = H vt), through
// a captured graph of the whole matvec when graphs are on (kernels only: no
// host synchronisation, no memset), re-captured when the velocity, the
// buffers or the kind change; the caches it reads are built eagerly first.
// Graphs are used when neither timers nor kernel statistics are on.
template <typename T, typename S = T>
int matvec_body(mireg_ctx *ctx, const T *vt, T *Hvt, bool spectral, int flags) {
    return spectral ? impl_matvec_spectral<T, S>(ctx, vt, flags) : impl_matvec<T, S>(ctx, vt, Hvt);
}
template <typename T, typename S = T>
int matvec_graph(mireg_ctx *ctx, const T *vt, T *Hvt, bool spectral = false, int flags = 0) {
    if (!ctx->use_graphs || ctx->tm.on || ctx->stats_on) return matvec_body<T, S>(ctx, vt, Hvt, spectral, flags);
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    int rc0 = ensure_tail64<T>(ctx);  // allocates: not inside the capture
    if (rc0) return rc0;
    ensure_state<T, S>(ctx);
    ensure_gradm<T, S>(ctx);
    ensure_d<T, S>(ctx);
    ensure_Y<T, S>(ctx);
    if (!ctx->mv_exec || ctx->mv_version != ctx->vel_version || ctx->mv_in != vt || ctx->mv_out != Hvt ||
        ctx->mv_spectral != spectral || ctx->mv_flags != flags) {
        if (ctx->mv_exec) {
            hipGraphExecDestroy(ctx->mv_exec);
            ctx->mv_exec = nullptr;
        }
        if (!ctx->cap_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        // the capture stream must see the work already queued on the context's stream
        HIP_OK(hipStreamSynchronize(ctx->stream));
        hipStream_t own = ctx->stream;
        ctx->stream = ctx->cap_stream;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        int rc = MIREG_OK;
        if (e == hipSuccess) {
            rc = matvec_body<T, S>(ctx, vt, Hvt, spectral, flags);
            e = hipStreamEndCapture(ctx->cap_stream, &graph);
        }
        ctx->stream = own;
        if (rc) return rc;
        if (e != hipSuccess) return ctx->fail(MIREG_E_HIP, "matvec capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&ctx->mv_exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return ctx->fail(MIREG_E_HIP, "graph instantiation: %s", hipGetErrorString(e));
        ctx->mv_version = ctx->vel_version;
        ctx->mv_in = vt;
        ctx->mv_out = Hvt;
        ctx->mv_spectral = spectral;
        ctx->mv_flags = flags;
    }
    HIP_OK(hipGraphLaunch(ctx->mv_exec, ctx->stream));
    return check_launch(ctx);
}

template <typename T, typename S = T>
int impl_precond(mireg_ctx *ctx, const T *r, T *z) {
    op_scale<T, S>(ctx, SYM_AINV, 3, ctx->p.beta_v, 0.0, r, z);
    return check_launch(ctx);
}

// out = spectral resampling of the vector field in (grid gs of ctx a) to
// grid gd of ctx b, through the two contexts' spectrum buffers.
template <typename T>
void resample3(mireg_ctx *a, mireg_ctx *b, const T *in, T *out, int nf) {
    const long long Na = a->N(), Nb = b->N();
    const T *ip[3] = {in, in + Na, in + 2 * Na};
    T *op[3] = {out, out + Nb, out + 2 * Nb};
    Phase ph(a, 0);
    spectral_resample<T>(a->g, b->g, nf, ip, op, static_cast<cx<T> *>(a->spec), static_cast<cx<T> *>(b->spec),
                         twiddles<T>(a), twiddles<T>(b), a->stream);
}

// Two-level preconditioner (Sec. 2.3.3): z = Hreg^{-1/2} (Q_P u + F_H t),
// t = Hreg^{-1/2} r, u ~ (Hreg_c^{-1/2} H_c Hreg_c^{-1/2})^{-1} Q_R t by CG on
// the coarse context to kappa * eps_h.
// The coarse problem follows the fine images and velocity (spectral resampling).
template <typename T>
void coarse_sync(mireg_ctx *ctx) {
    mireg_ctx *c = ctx->coarse;
    if (!ctx->coarse_images) {
        resample3<T>(ctx, c, ctx->f<T>(ctx->mT), c->f<T>(c->mT), 1);
        resample3<T>(ctx, c, ctx->f<T>(ctx->mR), c->f<T>(c->mR), 1);
        c->have_images = true;
        c->have_state = c->have_gradm = c->have_gradm0 = false;
        ctx->coarse_images = true;
    }
    if (ctx->coarse_vel_version != ctx->vel_version) {
        resample3<T>(ctx, c, ctx->f<T>(ctx->v), c->f<T>(c->v), 3);
        c->invalidate();
        ctx->coarse_vel_version = ctx->vel_version;
    }
}

template <typename T, typename S = T>
int two_level_apply(mireg_ctx *ctx, const T *r, T *z, double eps_h) {
    mireg_ctx *c = ctx->coarse;
    const long long n = 3 * ctx->N(), nc = 3 * c->N();
    int rc;
    coarse_sync<T>(ctx);
    T *t = ctx->vec<T>(7);
    op_scale<T, S>(ctx, SYM_AINV_SQRT, 3, ctx->p.beta_v, 0.0, r, t);
    T *b = c->vec<T>(4), *u = c->vec<T>(5), *w = c->vec<T>(6), *y = c->vec<T>(7);
    T *cr = c->vec<T>(0), *cp = c->vec<T>(1), *cq = c->vec<T>(2);
    resample3<T>(ctx, c, t, b, 3);
    // CG on S u = b, S = Hreg_c^{-1/2} H_c Hreg_c^{-1/2}, u0 = 0
    fill<T>(nc, (T)0, u, c->stream);
    HIP_OK(hipMemcpyAsync(cr, b, nc * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(cp, b, nc * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    double rr = 0;
    if ((rc = dot_h<T>(c, cr, cr, nc, &rr))) return rc;
    const double r0 = std::sqrt(rr), tol = ctx->pc_kappa * eps_h * r0;
    for (int it = 0; it < ctx->pc_max_inner && std::sqrt(rr) > tol; ++it) {
        op_scale<T, S>(c, SYM_AINV_SQRT, 3, c->p.beta_v, 0.0, cp, w);
        if ((rc = impl_matvec<T, S>(c, w, y))) return rc;
        ctx->coarse_matvecs += 1;
        op_scale<T, S>(c, SYM_AINV_SQRT, 3, c->p.beta_v, 0.0, y, cq);
        double pq = 0;
        if ((rc = dot_h<T>(c, cp, cq, nc, &pq))) return rc;
        if (!(pq > 0)) break;
        const double alpha = rr / pq;
        pcg_update<T>(nc, alpha, cp, cq, u, cr, c->partials, c->dres, c->stream);
        if ((rc = readback(c, 1))) return rc;
        const double rr_new = c->cell() * c->hres[0];
        if (std::sqrt(rr_new) <= tol) break;
        xpay<T>(nc, cr, rr_new / rr, cp, cp, c->stream);  // p = r + beta p
        rr = rr_new;
    }
    op_scale<T, S>(ctx, SYM_HIGHPASS, 3, 1.0, 0.0, t, z);
    resample3<T>(c, ctx, u, t, 3);
    axpby<T>(n, (T)1, t, (T)1, z, ctx->stream);  // z = F_H t + Q_P u
    op_scale<T, S>(ctx, SYM_AINV_SQRT, 3, ctx->p.beta_v, 0.0, z, z);
    return check_launch(ctx);
}

// Tile shape of the transport kernels; the stencil boxes (measured per tile)
// and any captured matvec depend on it.
template <typename T, typename S = T>
void set_tile(mireg_ctx *ctx, int shape) {
    ctx->g.sl_tile = shape;
    if (ctx->have_X) ctx->box_X = tile_boxes<T>(ctx, ctx->f<T>(ctx->X), ctx->tbox_X);
    if (ctx->have_Y) ctx->box_Y = tile_boxes<T>(ctx, ctx->f<T>(ctx->Y), ctx->tbox_Y);
    if (ctx->mv_exec) {
        hipGraphExecDestroy(ctx->mv_exec);
        ctx->mv_exec = nullptr;
    }
}

// Krylov x1 workgroup width (16 or 32 columns on FP32 256-point lines); a
// captured matvec holds the launches of the old width.
void set_x1_narrow(mireg_ctx *ctx, int narrow) {
    ctx->g.x1_narrow = narrow;
    if (ctx->mv_exec) {
        hipGraphExecDestroy(ctx->mv_exec);
        ctx->mv_exec = nullptr;
    }
}

// The preconditioner PCG uses, with the PCG's relative tolerance eps_h.
template <typename T, typename S = T>
int apply_precond(mireg_ctx *ctx, const T *r, T *z, double eps_h) {
    if (ctx->pc_kind == MIREG_PC_TWO_LEVEL) return two_level_apply<T, S>(ctx, r, z, eps_h);
    return impl_precond<T, S>(ctx, r, z);
}

// The two-level preconditioner on Krylov spectra: KV_Z = M^{-1} KV_R and
// *rz = <r, z>.  The nested CG runs on the coarse context's spectra: u
// (KV_X), its residual (KV_R), direction p (KV_S) and S p (KV_H), S = c H_c c
// with c = (beta_v a(k))^{-1/2}; each direction's transport takes c p on the
// coarse grid (coarse vector 2).  Same iteration as two_level_apply.
template <typename T, typename S = T>
int two_level_spectral(mireg_ctx *ctx, double eps_h, double *rz) {
    mireg_ctx *c = ctx->coarse;
    int rc;
    coarse_sync<T>(ctx);
    ensure_state<T, S>(c);
    ensure_gradm<T, S>(c);
    ensure_d<T, S>(c);
    ensure_Y<T, S>(c);
    const long long Nc = c->N();
    T *w = c->vec<T>(2);
    T *wp[3] = {w, w + Nc, w + 2 * Nc};
    cx<T> *rf[3], *zf[3], *uc[3], *rcs[3], *pc[3], *qc[3];
    for (int a = 0; a < 3; ++a) {
        rf[a] = ctx->khat<T>(KV_R, a);
        zf[a] = ctx->khat<T>(KV_Z, a);
        uc[a] = c->khat<T>(KV_X, a);
        rcs[a] = c->khat<T>(KV_R, a);
        pc[a] = c->khat<T>(KV_S, a);
        qc[a] = c->khat<T>(KV_H, a);
    }
    cx<T> *cwork = static_cast<cx<T> *>(c->spec);
    const Twiddles<T> tw = twiddles<T>(c);
    const SpecParams sp = spec_params<T>(c);
    const double h3c = c->cell();
    {
        Phase ph(ctx, 0);  // r = p = Q_R c r_fine, u = 0
        twolevel_restrict<T>(ctx->g, c->g, rf, rcs, pc, sp, c->stream);
        fill<T>(6 * c->g.NS, (T)0, reinterpret_cast<T *>(uc[0]), c->stream);
        krylov_update<T>(c->g, false, 2, c->dres, rcs, qc, sp, c->partials, c->stream);
    }
    if ((rc = readback(c, 3))) return rc;
    double rr = h3c * c->hres[2];
    const double tol = ctx->pc_kappa * eps_h * std::sqrt(rr);
    if (rr > 0) {
        Phase ph(ctx, 0);
        krylov_direction<T>(c->g, rcs, pc, 0.0, KF_FIRST | KF_ZRAW | KF_SQRT, uc, nullptr, wp, cwork, tw, sp,
                            c->stream);
    }
    c->use_graphs = ctx->use_graphs;
    // The step length alpha = rr / pq is formed on the device (c->dres[3]) by
    // the update, so an iteration reads back once; u takes alpha p in the
    // next direction pass, or in the combine when the loop stops on the
    // tolerance.
    bool pending = false;
    for (int it = 0; it < ctx->pc_max_inner && std::sqrt(rr) > tol; ++it) {
        if ((rc = matvec_graph<T, S>(c, w, nullptr, true, KF_SQRT))) return rc;  // S p into KV_H, pq
        ctx->coarse_matvecs += 1;
        krylov_update<T>(c->g, true, 2, c->dres, rcs, qc, sp, c->partials, c->stream);
        if ((rc = readback(c, 3))) return rc;
        const double pq = h3c * c->hres[0];
        if (!(pq > 0)) break;  // r was left unchanged
        const double rr_new = h3c * c->hres[2];
        if (std::sqrt(rr_new) <= tol) {
            pending = true;
            break;
        }
        {
            Phase ph(ctx, 0);  // u += alpha p, then p = r + beta p
            krylov_direction<T>(c->g, rcs, pc, rr_new / rr, KF_ZRAW | KF_SQRT, uc, c->dres + 3, wp, cwork, tw, sp,
                                c->stream);
        }
        rr = rr_new;
    }
    {
        Phase ph(ctx, 0);
        twolevel_combine<T>(ctx->g, c->g, rf, uc, pc, pending ? c->dres + 3 : nullptr, zf, spec_params<T>(ctx),
                            ctx->partials, ctx->dres + 1, ctx->stream);
    }
    if ((rc = readback(ctx, 2))) return rc;
    *rz = ctx->cell() * ctx->hres[1];
    return check_launch(ctx);
}

// ---- PCG (Algorithm "inner iteration") ----
// The Krylov vectors x, r and s are kept as half spectra (KV_X, KV_R, KV_S;
// H s as KV_H): the spectral preconditioner is a pointwise multiplier there
// and the two-level one (KV_Z) pointwise apart from its nested CG, H s is
// needed only as a spectrum, and only the direction s is transformed back
// (the transport needs it on the grid).  Inner products come from Parseval.
template <typename T, typename S = T>
int impl_pcg_spectral(mireg_ctx *ctx, const T *rhs, T *x, double rtol, int maxit, int *iters, double *relres,
                      int *status, int *matvecs, bool rhs_is_minus_h = false) {
    const long long N = ctx->N();
    const double h3 = ctx->cell();
    T *s = ctx->vec<T>(2);
    T *sp3[3] = {s, s + N, s + 2 * N}, *xp[3] = {x, x + N, x + 2 * N};
    const T *rp[3] = {rhs, rhs + N, rhs + 2 * N};
    const bool two_level = ctx->pc_kind == MIREG_PC_TWO_LEVEL;
    cx<T> *xh[3], *rh[3], *sh[3], *hh[3], *zh[3];
    for (int a = 0; a < 3; ++a) {
        xh[a] = ctx->khat<T>(KV_X, a);
        rh[a] = ctx->khat<T>(KV_R, a);
        sh[a] = ctx->khat<T>(KV_S, a);
        hh[a] = ctx->khat<T>(KV_H, a);
        zh[a] = ctx->khat<T>(KV_Z, a);
    }
    // z = M^{-1} r: from r in the direction pass (spectral), or KV_Z (two-level)
    cx<T> *const *zsrc = two_level ? zh : rh;
    const int zflag = two_level ? KF_ZRAW : 0;
    cx<T> *work = static_cast<cx<T> *>(ctx->spec);
    const Twiddles<T> tw = twiddles<T>(ctx);
    const SpecParams sp = spec_params<T>(ctx);
    int rc;
    {
        Phase ph(ctx, 0);
        if (rhs_is_minus_h)  // rhs = -g and KV_H still holds the spectrum of g (the gradient's tail)
            affine<T>(6 * ctx->g.NS, reinterpret_cast<const T *>(hh[0]), -1.0, 0.0, reinterpret_cast<T *>(rh[0]),
                      ctx->stream);
        else
            krylov_forward<T>(ctx->g, rp, rh, work, tw, ctx->stream);  // r = rhs, x = 0
        fill<T>(6 * ctx->g.NS, (T)0, reinterpret_cast<T *>(xh[0]), ctx->stream);
        krylov_update<T>(ctx->g, false, 1, ctx->dres, rh, hh, sp, ctx->partials, ctx->stream);
    }
    if ((rc = readback(ctx, 3))) return rc;
    const double r0 = std::sqrt(h3 * ctx->hres[2]);
    double rz = h3 * ctx->hres[1];
    int it = 0, mv = 0, st = r0 > 0 ? MIREG_MAXIT : MIREG_CONVERGED_REL;
    double rnorm = r0;
    bool x_is_s = false;
    // The step length alpha = rz / sHs is formed on the device (dres[3]) by
    // the update, so an iteration reads back once; x takes alpha s in the next
    // direction pass, or in the final transform when the loop stops on the
    // tolerance.
    bool pending = false;
    if (r0 > 0) {
        if (two_level && (rc = two_level_spectral<T, S>(ctx, rtol, &rz))) return rc;
        {
            Phase ph(ctx, 0);  // s = z = M^{-1} r
            krylov_direction<T>(ctx->g, zsrc, sh, 0.0, KF_FIRST | zflag, xh, nullptr, sp3, work, tw, sp,
                                ctx->stream);
        }
        while (it < maxit) {
            if ((rc = matvec_graph<T, S>(ctx, s, nullptr, true))) return rc;  // H s, sHs
            ++mv;
            {
                Phase ph(ctx, 2);
                krylov_update<T>(ctx->g, true, 1, ctx->dres, rh, hh, sp, ctx->partials, ctx->stream);
            }
            if ((rc = readback(ctx, 3))) return rc;
            const double sHs = h3 * ctx->hres[0];
            if (!(sHs > 0)) {  // non-positive curvature (r was left unchanged): keep the current
                               // iterate (z on the first)
                x_is_s = it == 0;
                st = MIREG_NEG_CURV;
                break;
            }
            ++it;
            rnorm = std::sqrt(h3 * ctx->hres[2]);
            if (rnorm <= rtol * r0) {
                pending = true;
                st = MIREG_CONVERGED_REL;
                break;
            }
            double rz_new = h3 * ctx->hres[1];
            if (two_level && (rc = two_level_spectral<T, S>(ctx, rtol, &rz_new))) return rc;
            const double mu = rz_new / rz;
            rz = rz_new;
            {
                Phase ph(ctx, 0);  // x += alpha s, then s = z + mu s
                krylov_direction<T>(ctx->g, zsrc, sh, mu, zflag, xh, ctx->dres + 3, sp3, work, tw, sp, ctx->stream);
            }
        }
    }
    if (x_is_s) {
        HIP_OK(hipMemcpyAsync(x, s, 3 * N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    } else if (it > 0) {
        Phase ph(ctx, 0);
        krylov_inverse<T>(ctx->g, xh, pending ? sh : nullptr, ctx->dres + 3, xp, work, tw, ctx->stream);
    } else {
        fill<T>(3 * N, (T)0, x, ctx->stream);
    }
    if (iters) *iters = it;
    if (relres) *relres = r0 > 0 ? rnorm / r0 : 0.0;
    if (status) *status = st;
    if (matvecs) *matvecs = mv;
    return check_launch(ctx);
}

template <typename T, typename S = T>
int impl_pcg(mireg_ctx *ctx, const T *rhs, T *x, double rtol, int maxit, int *iters, double *relres,
             int *status = nullptr, int *matvecs = nullptr, bool rhs_is_minus_h = false) {
    return impl_pcg_spectral<T, S>(ctx, rhs, x, rtol, maxit, iters, relres, status, matvecs, rhs_is_minus_h);
}

// Autotuner: mean time of a PCG iteration (`reps` iterations from the
// current velocity as right-hand side, the setup and final transform
// included) per transport tile shape and, where both exist, per Krylov x1
// workgroup width; keeps the fastest pair.  ms[shape]: the best time of that
// shape over the widths.  Tile shapes give identical bits; the widths group
// the FP64 partial sums of <s, Hs> differently.
template <typename T, typename S = T>
int impl_autotune(mireg_ctx *ctx, int reps, double *ms, int *shape) {
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    ensure_state<T, S>(ctx);
    ensure_gradm<T, S>(ctx);
    ensure_d<T, S>(ctx);
    ensure_Y<T, S>(ctx);
    const long long n = 3 * ctx->N();
    // right-hand side and iterate outside PCG's own vectors (0..3)
    T *in = ctx->vec<T>(4), *out = ctx->vec<T>(5);
    HIP_OK(hipMemcpyAsync(in, ctx->v, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    double best = 1e300;
    int best_shape = ctx->g.sl_tile, best_narrow = ctx->g.x1_narrow, rc = MIREG_OK;
    const int widths = (sizeof(T) == 4 && ctx->g.n1 == 256) ? 2 : 1;
    for (int sh = 0; sh < 3 && !rc; ++sh) {
        set_tile<T, S>(ctx, sh);
        double best_sh = 1e300;
        for (int w = 0; w < widths && !rc; ++w) {
            set_x1_narrow(ctx, w);
            int its = 0;
            rc = impl_pcg<T, S>(ctx, in, out, 0.0, 1, &its, nullptr);  // warm-up (and graph capture)
            hipEventRecord(e0, ctx->stream);
            if (!rc) rc = impl_pcg<T, S>(ctx, in, out, 0.0, reps, &its, nullptr);
            hipEventRecord(e1, ctx->stream);
            hipEventSynchronize(e1);
            float t = 0;
            hipEventElapsedTime(&t, e0, e1);
            const double m = (double)t / (its > 0 ? its : 1);
            if (m < best_sh) best_sh = m;
            if (m < best) {
                best = m;
                best_shape = sh;
                best_narrow = w;
            }
        }
        if (ms) ms[sh] = best_sh;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    set_tile<T, S>(ctx, best_shape);
    set_x1_narrow(ctx, best_narrow);
    if (shape) *shape = best_shape;
    return check_launch(ctx);
}

template <typename T, typename S = T>
int impl_set_velocity(mireg_ctx *ctx, const T *v);

// ---- GN (Algorithm "outer iteration") ----
template <typename T, typename S = T>
int impl_gn(mireg_ctx *ctx, T *v_io, const mireg_solve_opts *o, mireg_report *rep) {
    auto t0 = std::chrono::steady_clock::now();
    const long long n = 3 * ctx->N();
    const double h3 = ctx->cell();
    mireg_report R{};
    const long long coarse0 = ctx->coarse_matvecs;
    // vectors 0..3 belong to PCG; 4: g, 5: vt, 6: accepted v
    T *g = ctx->vec<T>(4), *vt = ctx->vec<T>(5), *vk = ctx->vec<T>(6);
    int rc;
    if ((rc = impl_set_velocity<T, S>(ctx, v_io))) return rc;
    HIP_OK(hipMemcpyAsync(vk, v_io, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    double J = 0;
    if ((rc = impl_objective<T, S>(ctx, &J, nullptr, nullptr))) return rc;
    double gn = 0;
    if ((rc = impl_gradient<T, S>(ctx, g, &gn))) return rc;
    // counted as the paper's tables count them (Sec. 4.7: 3 iterations, 3
    // matvecs, 15 PDE solves): a state solve for J and one for g, and the
    // adjoint solve, although the gradient reuses the objective's state here
    R.pde_solves += 3;
    const double g0 = gn;
    R.J0 = J;
    R.gnorm0 = g0;
    int k = 0;
    for (;;) {
        if (o->log_level > 0)
            fprintf(stderr, "[mireg] gn %d J %.6e |g| %.6e |g|/|g0| %.3e\n", k, J, gn, g0 > 0 ? gn / g0 : 0.0);
        if (gn <= o->grad_rtol * g0) {
            R.status = MIREG_CONVERGED_REL;
            break;
        }
        if (gn <= o->grad_atol) {
            R.status = MIREG_CONVERGED_ABS;
            break;
        }
        if (k >= o->max_gn) {
            R.status = MIREG_MAXIT;
            break;
        }
        const double eps_h = std::fmin(0.5, std::sqrt(gn / g0));
        // rhs = -g in vector 7
        T *rhs = ctx->vec<T>(7);
        affine<T>(n, g, -1.0, 0.0, rhs, ctx->stream);
        int its = 0, pst = 0, mv = 0;
        // in FP32 contexts the gradient's tail leaves the spectrum of g in KV_H
        // (untouched since): PCG starts from it instead of transforming -g again
        constexpr bool ghat = std::is_same<T, float>::value;
        if ((rc = impl_pcg<T, S>(ctx, rhs, vt, eps_h, o->max_pcg, &its, nullptr, &pst, &mv, ghat))) return rc;
        R.matvecs += mv;
        R.pcg_iters += its;
        R.pde_solves += 2 * mv;
        R.neg_curv += pst == MIREG_NEG_CURV;
        double slope = 0;
        if ((rc = dot_h<T>(ctx, g, vt, n, &slope))) return rc;
        double alpha = 1.0, Jt = 0, alpha_tried = 0;
        bool accepted = false;
        for (int ls = 0; ls < o->max_ls; ++ls) {
            // trial velocity v = vk + alpha vt, written into the context velocity
            alpha_tried = alpha;
            xpay<T>(n, vk, alpha, vt, ctx->f<T>(ctx->v), ctx->stream);
            ctx->invalidate();
            if ((rc = impl_objective<T, S>(ctx, &Jt, nullptr, nullptr))) return rc;
            R.ls_trials += 1;
            R.pde_solves += 1;
            if (Jt <= J + o->armijo_c1 * alpha * slope) {
                accepted = true;
                break;
            }
            alpha *= 0.5;
        }
        if (ctx->jlog)
            fprintf(ctx->jlog,
                    "{\"event\": \"gn\", \"iter\": %d, \"J\": %.17g, \"gnorm\": %.17g, \"gnorm_rel\": %.17g, "
                    "\"eps_h\": %.17g, \"pcg_iters\": %d, \"pcg_status\": %d, \"pcg_matvecs\": %d, "
                    "\"slope\": %.17g, \"alpha\": %.17g, \"accepted\": %s, \"J_trial\": %.17g, "
                    "\"matvecs\": %d, \"pde_solves\": %d, \"ls_trials\": %d, \"seconds\": %.6f}\n",
                    k, J, gn, g0 > 0 ? gn / g0 : 0.0, eps_h, its, pst, mv, slope, alpha_tried, accepted ? "true" : "false",
                    Jt, R.matvecs, R.pde_solves, R.ls_trials,
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        if (!accepted) {
            HIP_OK(hipMemcpyAsync(ctx->v, vk, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
            ctx->invalidate();
            R.status = MIREG_LS_FAIL;
            break;
        }
        HIP_OK(hipMemcpyAsync(vk, ctx->v, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
        J = Jt;
        if ((rc = impl_gradient<T, S>(ctx, g, &gn))) return rc;
        R.pde_solves += 1;
        ++k;
    }
    R.gn_iters = k;
    R.J = J;
    R.gnorm = gn;
    R.gnorm_rel = g0 > 0 ? gn / g0 : 0.0;
    // mismatch_rel = ||m(1) - mR||^2 / ||mT - mR||^2
    ensure_state<T, S>(ctx);
    const long long N = ctx->N();
    sumsq_diff<T, T>(ctx->f<T>(ctx->m) + ctx->p.nt * N, ctx->f<T>(ctx->mR), N, ctx->partials, ctx->dres,
                     ctx->stream);
    if ((rc = readback(ctx, 1))) return rc;
    const double num = ctx->hres[0];
    sumsq_diff<T, T>(ctx->f<T>(ctx->mT), ctx->f<T>(ctx->mR), N, ctx->partials, ctx->dres, ctx->stream);
    if ((rc = readback(ctx, 1))) return rc;
    R.mismatch_rel = ctx->hres[0] > 0 ? num / ctx->hres[0] : 0.0;
    HIP_OK(hipMemcpyAsync(v_io, vk, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    R.coarse_matvecs = (int)(ctx->coarse_matvecs - coarse0);
    (void)h3;
    if (ctx->jlog) {
        fprintf(ctx->jlog,
                "{\"event\": \"done\", \"status\": %d, \"gn_iters\": %d, \"pcg_iters\": %d, \"matvecs\": %d, "
                "\"coarse_matvecs\": %d, \"pde_solves\": %d, \"ls_trials\": %d, \"neg_curv\": %d, \"J0\": %.17g, "
                "\"J\": %.17g, \"gnorm0\": %.17g, \"gnorm\": %.17g, \"gnorm_rel\": %.17g, "
                "\"mismatch_rel\": %.17g, \"seconds\": %.6f}\n",
                R.status, R.gn_iters, R.pcg_iters, R.matvecs, R.coarse_matvecs, R.pde_solves, R.ls_trials, R.neg_curv,
                R.J0, R.J, R.gnorm0, R.gnorm, R.gnorm_rel, R.mismatch_rel, R.seconds);
        fflush(ctx->jlog);
    }
    if (rep) *rep = R;
    return check_launch(ctx);
}

template <typename T, typename S = T>
int check_finite(mireg_ctx *ctx, const T *a, long long n, const char *what) {
    minmax_nonfinite<T>(a, n, ctx->partials, ctx->dres, ctx->stream);
    int rc = readback(ctx, 3);
    if (rc) return rc;
    if (ctx->hres[2] != 0) return ctx->fail(MIREG_E_NONFINITE, "%s contains %.0f non-finite values", what, ctx->hres[2]);
    return MIREG_OK;
}

template <typename T, typename S = T>
int impl_set_images(mireg_ctx *ctx, const T *mT, const T *mR) {
    const long long N = ctx->N();
    int rc;
    if ((rc = check_finite<T, S>(ctx, mT, N, "mT"))) return rc;
    if ((rc = check_finite<T, S>(ctx, mR, N, "mR"))) return rc;
    HIP_OK(hipMemcpyAsync(ctx->mT, mT, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->mR, mR, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    ctx->have_images = true;
    ctx->have_state = ctx->have_gradm = ctx->have_gradm0 = false;
    ctx->coarse_images = false;
    return MIREG_OK;
}

template <typename T, typename S>
int impl_set_velocity(mireg_ctx *ctx, const T *v) {
    const long long n = 3 * ctx->N();
    int rc;
    if ((rc = check_finite<T, S>(ctx, v, n, "v"))) return rc;
    if (v != ctx->v) HIP_OK(hipMemcpyAsync(ctx->v, v, n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    ctx->invalidate();
    return MIREG_OK;
}

template <typename T, typename S = T>
int impl_op(mireg_ctx *ctx, int opcode, const T *in, T *out, double arg) {
    const long long N = ctx->N();
    switch (opcode) {
        case MIREG_OP_GRAD: op_grad<T, S>(ctx, in, out); break;
        case MIREG_OP_DIV: op_div<T, S>(ctx, in, out); break;
        case MIREG_OP_LAPLACE: op_scale<T, S>(ctx, SYM_LAP, 1, 1.0, 0.0, in, out); break;
        case MIREG_OP_APPLY_A: op_scale<T, S>(ctx, SYM_A, 3, 1.0, 0.0, in, out); break;
        case MIREG_OP_APPLY_K: op_proj<T, S>(ctx, ctx->p.div, in, out); break;
        case MIREG_OP_LERAY: op_proj<T, S>(ctx, MIREG_DIV_LERAY, in, out); break;
        case MIREG_OP_PRECOND: impl_precond<T, S>(ctx, in, out); break;
        case MIREG_OP_GAUSS:
            if (!(arg >= 0)) return ctx->fail(MIREG_E_ARG, "Gaussian width must be >= 0");
            op_scale<T, S>(ctx, SYM_GAUSS, 1, 1.0, arg, in, out);
            break;
        case MIREG_OP_DEPARTURE_X:
        case MIREG_OP_DEPARTURE_Y:
            compute_departure<T>(ctx, opcode == MIREG_OP_DEPARTURE_X ? -1 : +1, in, out);
            break;
        case MIREG_OP_TRANSPORT_STATE: {
            ensure_X<T, S>(ctx);
            // intermediate slices in T, as the state history is held
            T *a = ctx->vec<T>(7), *b = a + N;
            const T *X = ctx->f<T>(ctx->X);
            const int nt = ctx->p.nt, ord = ctx->p.interp_order;
            const SlBox box = ctx->box_X;
            Phase ph(ctx, 1);
            if (nt == 1) {
                interp_field<T, T, T>(ctx->g, ord, in, X, out, box, ctx->stream);
            } else {
                // step 0 writes a; step j in 1..nt-2 reads the previous output
                // and writes b for odd j, a for even j; step nt-1 writes out
                interp_field<T, T, T>(ctx->g, ord, in, X, a, box, ctx->stream);
                for (int j = 1; j < nt - 1; ++j) {
                    interp_field<T, T, T>(ctx->g, ord, (j & 1) ? a : b, X, (j & 1) ? b : a, box, ctx->stream);
                }
                interp_field<T, T, T>(ctx->g, ord, ((nt - 2) & 1) ? b : a, X, out, box, ctx->stream);
            }
            break;
        }
        case MIREG_OP_TRANSPORT_ADJOINT: {
            // lam^nt = in, then nt backward steps along Y in the storage type
            // of the adjoint history (its buffer is scratch between sweeps)
            ensure_Y<T, S>(ctx);
            ensure_d<T, S>(ctx);
            const int nt = ctx->p.nt;
            const double dt = 1.0 / nt;
            S *lam = ctx->f<S>(ctx->lam);
            Phase ph(ctx, 1);
            if constexpr (std::is_same<S, T>::value)
                HIP_OK(hipMemcpyAsync(lam + nt * N, in, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
            else
                convert_field<T, T, S>(N, in, lam + nt * N, ctx->stream);
            for (int j = nt - 1; j >= 0; --j)
                adjoint_step<T, S>(ctx->g, ctx->p.interp_order, dt, lam + (j + 1) * N, ctx->f<T>(ctx->d),
                                   ctx->f<T>(ctx->Y), lam + j * N, ctx->box_Y, ctx->stream);
            if constexpr (std::is_same<S, T>::value)
                HIP_OK(hipMemcpyAsync(out, lam, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
            else
                convert_field<T, S, T>(N, lam, out, ctx->stream);
            break;
        }
        case MIREG_OP_INTERP: {
            const int box = box_of_displacement<T>(ctx, in + N);
            Phase ph(ctx, 1);
            interp_field<T, T, T>(ctx->g, ctx->p.interp_order, in, in + N, out, box, ctx->stream);
            break;
        }
        case MIREG_OP_RESCALE01: {
            minmax_nonfinite<T>(in, N, ctx->partials, ctx->dres, ctx->stream);
            int rc = readback(ctx, 3);
            if (rc) return rc;
            const double lo = ctx->hres[0], hi = ctx->hres[1];
            if (!(hi > lo)) return ctx->fail(MIREG_E_ARG, "constant field cannot be rescaled");
            affine<T>(N, in, 1.0 / (hi - lo), -lo / (hi - lo), out, ctx->stream);
            break;
        }
        case MIREG_OP_SCALE_MAXNORM: {
            max_norm2<T>(in, N, ctx->partials, ctx->dres, ctx->stream);
            int rc = readback(ctx, 1);
            if (rc) return rc;
            const double peak = std::sqrt(ctx->hres[0]);
            if (!(peak > 0)) return ctx->fail(MIREG_E_ARG, "zero field cannot be scaled");
            affine<T>(3 * N, in, arg / peak, 0.0, out, ctx->stream);
            break;
        }
        default: return ctx->fail(MIREG_E_ARG, "unknown opcode %d", opcode);
    }
    return check_launch(ctx);
}

template <typename T>
int make_twiddles_into(mireg_ctx *ctx, void *const *dst) {
    const int n[3] = {ctx->g.n1, ctx->g.n2, ctx->g.n3};
    for (int a = 0; a < 3; ++a) {
        std::vector<cx<T>> h(n[a]);
        for (int j = 0; j < n[a]; ++j) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * j / n[a];
            h[j].re = (T)cosl(ang);
            h[j].im = (T)sinl(ang);
        }
        // on the context's stream: a copy on the legacy stream would invalidate
        // a graph capture running in another thread
        HIP_OK(hipMemcpyAsync(dst[a], h.data(), n[a] * sizeof(cx<T>), hipMemcpyHostToDevice, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return MIREG_OK;
}

template <typename T, typename S = T>
int make_twiddles(mireg_ctx *ctx) {
    return make_twiddles_into<T>(ctx, ctx->tw);
}

int alloc(mireg_ctx *ctx, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return ctx->fail(MIREG_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    ctx->allocs.push_back(*p);
    ctx->bytes += bytes;
    return MIREG_OK;
}

// Installs the context's kernel observer for the duration of an entry point.
struct HookGuard {
    explicit HookGuard(mireg_ctx *ctx) { mireg::g_hook = (ctx && ctx->stats_on) ? &ctx->stats : nullptr; }
    ~HookGuard() { mireg::g_hook = nullptr; }
};

// Typed dispatch: F32 -> <float, float>, F64 -> <double, double>,
// F32 with FP16 storage of the transported fields -> <float, __half>.
// CALL is an expression in the type aliases T (arithmetic and boundary type)
// and S (storage of the transported fields).
#define DISPATCH(ctx, CALL)                                                                            \
    (HookGuard{ctx},                                                                                   \
     ((ctx)->p.dtype == MIREG_F64                                                                      \
          ? [&] { using T = double; using S = double; return CALL; }()                                 \
          : (ctx)->p.dtype == MIREG_F32_H16 ? [&] { using T = float; using S = __half; return CALL; }() \
                                            : [&] { using T = float; using S = float; return CALL; }()))

}  // namespace

// ===========================================================================
// Batched solves: several problems of any supported sizes in lockstep (not in
// the paper; many registration pairs on one GPU).  Every problem keeps its
// own context and follows exactly its single-problem arithmetic; what the
// batch shares is the launch: each transport step of the Hessian matvec runs
// once across all running problems (k_sl_multi over their tiles numbered one
// after the other), and the per-iteration host read-back of the PCG scalars
// is one synchronisation for all of them.
// ===========================================================================
struct mireg_batch {
    std::vector<mireg_ctx *> ctx;
    hipStream_t stream = nullptr;
    void *htab = nullptr;  // pinned host copy of the step tables
    void *dtab = nullptr;  // device step tables
    hipEvent_t tab_done = nullptr;  // the last table upload has completed after this event
    bool tab_pending = false;
    mireg::TabArena arena;  // pointer tables of the multi-problem Krylov passes
    std::string err;
    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

namespace {

// nres results of every listed problem to its host mirror: the copies are
// enqueued first, then one synchronisation of the common stream.
int batch_readback(mireg_batch *B, const std::vector<int> &idx, int nres) {
    for (int i : idx) {
        mireg_ctx *c = B->ctx[i];
        hipError_t e = hipMemcpyAsync(c->hres, c->dres, nres * sizeof(double), hipMemcpyDeviceToHost, B->stream);
        if (e != hipSuccess) return B->fail(MIREG_E_HIP, "read-back: %s", hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return B->fail(MIREG_E_HIP, "read-back: %s", hipGetErrorString(e));
    return MIREG_OK;
}

// Step tables of the batched matvec transport for the listed problems (their
// PCG direction, vector 2, as the transported increment).
template <typename T, typename S>
int batch_tables(mireg_batch *B, const std::vector<int> &idx, std::vector<SlProblem> &pr) {
    pr.clear();
    for (int i : idx) {
        mireg_ctx *c = B->ctx[i];
        SlProblem q;
        q.g = c->g;
        q.gradm = c->gradm;
        q.vt = c->vec<T>(2);
        q.X = c->X;
        q.Y = c->Y;
        q.d = c->d;
        q.q = c->q;
        q.lam = c->lam;
        q.b = c->b;
        q.boxX = c->box_X;
        q.boxY = c->box_Y;
        pr.push_back(q);
    }
    if (pr.empty()) return MIREG_OK;
    if (B->tab_pending) {  // the host tables are rewritten only after their last upload
        hipError_t e = hipEventSynchronize(B->tab_done);
        if (e != hipSuccess) return B->fail(MIREG_E_HIP, "table upload: %s", hipGetErrorString(e));
    }
    matvec_transport_tables<T, S>(pr.data(), (int)pr.size(), B->ctx[0]->p.nt, B->htab, B->dtab, B->stream);
    hipError_t e = hipEventRecord(B->tab_done, B->stream);
    if (e != hipSuccess) return B->fail(MIREG_E_HIP, "table upload: %s", hipGetErrorString(e));
    B->tab_pending = true;
    return MIREG_OK;
}

int batch_ctx_error(mireg_batch *B, mireg_ctx *c, int rc) {
    return B->fail(rc, "%s", c->err.c_str());
}

// Problems of one grid size and one regularisation share the Krylov
// passes' launches: key of a problem's class.
std::tuple<int, int, int, int, int, double, double> krylov_class(const mireg_ctx *c) {
    return std::make_tuple(c->g.n1, c->g.n2, c->g.n3, c->p.reg, c->p.div, c->p.beta_v, c->p.beta_w);
}

// Lockstep PCG (the spectral preconditioner; the iteration of
// impl_pcg_spectral, problem by problem) for the problems idx: H_i x_i =
// rhs_i to rtol[k] (k the position in idx), at most maxit iterations.  Per
// iteration: one launch per transport step across the running problems, one
// launch per Krylov pass per class of problems of one grid size, one
// read-back.
template <typename T, typename S>
int batch_pcg(mireg_batch *B, const std::vector<int> &idx, const T *const *rhs, T *const *x, const double *rtol,
              int maxit, int *iters, double *relres, int *status, int *matvecs) {
    struct Run {
        double r0 = 0, rz = 0, rnorm = 0, mu = 0;
        int it = 0, mv = 0, st = MIREG_CONVERGED_REL;
        bool x_is_s = false, pending = false;
    };
    const int n = (int)idx.size();
    std::vector<Run> run(n);
    TabArena &ar = B->arena;
    int rc;
    // positions k of idx grouped by Krylov class, in order of first appearance
    std::vector<std::vector<int>> classes;
    {
        std::vector<std::tuple<int, int, int, int, int, double, double>> keys;
        for (int k = 0; k < n; ++k) {
            const auto key = krylov_class(B->ctx[idx[k]]);
            size_t c = 0;
            while (c < keys.size() && keys[c] != key) ++c;
            if (c == keys.size()) {
                keys.push_back(key);
                classes.emplace_back();
            }
            classes[c].push_back(k);
        }
    }
    // the members of the class listed in `ks` that `sel` keeps
    auto members = [&](const std::vector<int> &ks, const std::vector<char> &sel) {
        std::vector<int> out;
        for (int k : ks)
            if (sel[k]) out.push_back(k);
        return out;
    };
    // one class's multi-problem passes; operand arrays built per call
    auto hessian_update = [&](const std::vector<int> &ks, bool update, bool hess) -> int {
        if (ks.empty()) return MIREG_OK;
        const int np = (int)ks.size();
        mireg_ctx *c0 = B->ctx[idx[ks[0]]];
        std::vector<const T *> b(3 * np);
        std::vector<const cx<T> *> sh(3 * np), hhc(3 * np);
        std::vector<cx<T> *> hh(3 * np), rh(3 * np), work(np);
        std::vector<double *> red(np), rout(np), res(np), part(np);
        for (int j = 0; j < np; ++j) {
            mireg_ctx *c = B->ctx[idx[ks[j]]];
            const long long N = c->N();
            const T *bb = c->f<T>(c->b);
            for (int a = 0; a < 3; ++a) {
                b[3 * j + a] = bb + a * N;
                sh[3 * j + a] = c->khat<T>(KV_S, a);
                hh[3 * j + a] = c->khat<T>(KV_H, a);
                hhc[3 * j + a] = hh[3 * j + a];
                rh[3 * j + a] = c->khat<T>(KV_R, a);
            }
            work[j] = static_cast<cx<T> *>(c->spec);
            red[j] = c->xpart;
            rout[j] = c->dres;
            res[j] = c->dres;
            part[j] = c->partials;
        }
        const SpecParams sp = spec_params<T>(c0);
        bool ok = true;
        if (hess) {
            Phase ph(c0, 0);
            ok = krylov_hessian_multi<T>(c0->g, np, b.data(), sh.data(), hh.data(), work.data(), red.data(),
                                         rout.data(), twiddles<T>(c0), sp, ar, B->stream);
        }
        if (ok) {
            Phase ph(c0, 2);
            ok = krylov_update_multi<T>(c0->g, np, update, 1, res.data(), rh.data(), hhc.data(), part.data(), sp, ar,
                                        B->stream);
        }
        return ok ? MIREG_OK : B->fail(MIREG_E_NOMEM, "table arena exhausted");
    };
    auto direction = [&](const std::vector<int> &ks, bool first) -> int {
        if (ks.empty()) return MIREG_OK;
        const int np = (int)ks.size();
        mireg_ctx *c0 = B->ctx[idx[ks[0]]];
        std::vector<const cx<T> *> rh(3 * np);
        std::vector<cx<T> *> sh(3 * np), xh(3 * np), work(np);
        std::vector<T *> so(3 * np);
        std::vector<const double *> alpha(np);
        std::vector<double> mu(np);
        for (int j = 0; j < np; ++j) {
            mireg_ctx *c = B->ctx[idx[ks[j]]];
            const long long N = c->N();
            T *sg = c->vec<T>(2);
            for (int a = 0; a < 3; ++a) {
                rh[3 * j + a] = c->khat<T>(KV_R, a);
                sh[3 * j + a] = c->khat<T>(KV_S, a);
                xh[3 * j + a] = c->khat<T>(KV_X, a);
                so[3 * j + a] = sg + a * N;
            }
            work[j] = static_cast<cx<T> *>(c->spec);
            alpha[j] = c->dres + 3;
            mu[j] = run[ks[j]].mu;
        }
        Phase ph(c0, 0);
        const bool ok = krylov_direction_multi<T>(c0->g, np, rh.data(), sh.data(), first ? nullptr : mu.data(),
                                                  first ? KF_FIRST : 0, xh.data(), first ? nullptr : alpha.data(),
                                                  so.data(), work.data(), twiddles<T>(c0), spec_params<T>(c0), ar,
                                                  B->stream);
        return ok ? MIREG_OK : B->fail(MIREG_E_NOMEM, "table arena exhausted");
    };
    auto readback_all = [&](const std::vector<int> &ks_all) -> int {
        std::vector<int> ids;
        for (int k : ks_all) ids.push_back(idx[k]);
        const int r = batch_readback(B, ids, 3);
        ar.reset();  // every table upload issued so far has completed
        return r;
    };
    for (int k = 0; k < n; ++k) {
        mireg_ctx *c = B->ctx[idx[k]];
        ensure_state<T, S>(c);
        ensure_gradm<T, S>(c);
        ensure_d<T, S>(c);
        ensure_Y<T, S>(c);
        const long long N = c->N();
        const T *rp[3] = {rhs[k], rhs[k] + N, rhs[k] + 2 * N};
        cx<T> *rh[3] = {c->khat<T>(KV_R, 0), c->khat<T>(KV_R, 1), c->khat<T>(KV_R, 2)};
        Phase ph(c, 0);
        krylov_forward<T>(c->g, rp, rh, static_cast<cx<T> *>(c->spec), twiddles<T>(c), B->stream);
        fill<T>(6 * c->g.NS, (T)0, reinterpret_cast<T *>(c->khat<T>(KV_X, 0)), B->stream);
    }
    std::vector<int> all(n);
    for (int k = 0; k < n; ++k) all[k] = k;
    for (const auto &cl : classes)
        if ((rc = hessian_update(cl, false, false))) return rc;
    if ((rc = readback_all(all))) return rc;
    std::vector<char> live(n, 0);
    for (int k = 0; k < n; ++k) {
        mireg_ctx *c = B->ctx[idx[k]];
        const double h3 = c->cell();
        Run &R = run[k];
        R.r0 = std::sqrt(h3 * c->hres[2]);
        R.rz = h3 * c->hres[1];
        R.rnorm = R.r0;
        if (R.r0 > 0) R.st = MIREG_MAXIT;
    }
    std::vector<char> pos(n, 0);
    for (int k = 0; k < n; ++k) pos[k] = run[k].r0 > 0;
    for (const auto &cl : classes)
        if ((rc = direction(members(cl, pos), true))) return rc;  // s = z = M^{-1} r
    std::vector<int> livek;
    for (int k = 0; k < n; ++k)
        if (run[k].r0 > 0 && maxit > 0) {
            live[k] = 1;
            livek.push_back(k);
        }
    std::vector<SlProblem> pr;
    auto tables = [&]() {
        std::vector<int> ids;
        for (int k : livek) ids.push_back(idx[k]);
        return batch_tables<T, S>(B, ids, pr);
    };
    if (!livek.empty() && (rc = tables())) return rc;
    const int order = B->ctx[0]->p.interp_order, nt = B->ctx[0]->p.nt;
    while (!livek.empty()) {
        {
            Phase ph(B->ctx[idx[livek[0]]], 1);
            matvec_transport_batch<T, S>(pr.data(), (int)pr.size(), order, nt, B->htab, B->dtab, B->stream);
        }
        for (const auto &cl : classes)
            if ((rc = hessian_update(members(cl, live), true, true))) return rc;
        if ((rc = readback_all(livek))) return rc;
        std::vector<int> next;
        std::vector<char> dir(n, 0);
        for (int k : livek) {
            mireg_ctx *c = B->ctx[idx[k]];
            const double h3 = c->cell();
            Run &R = run[k];
            ++R.mv;
            live[k] = 0;
            const double sHs = h3 * c->hres[0];
            if (!(sHs > 0)) {
                R.x_is_s = R.it == 0;
                R.st = MIREG_NEG_CURV;
                continue;
            }
            ++R.it;
            R.rnorm = std::sqrt(h3 * c->hres[2]);
            if (R.rnorm <= rtol[k] * R.r0) {
                R.pending = true;
                R.st = MIREG_CONVERGED_REL;
                continue;
            }
            const double rz_new = h3 * c->hres[1];
            R.mu = rz_new / R.rz;
            R.rz = rz_new;
            dir[k] = 1;  // x += alpha s, then s = z + mu s
            if (R.it < maxit) {
                next.push_back(k);
                live[k] = 1;
            }
        }
        for (const auto &cl : classes)
            if ((rc = direction(members(cl, dir), false))) return rc;
        const bool same = next == livek;
        livek.swap(next);
        if (!same && !livek.empty() && (rc = tables())) return rc;
    }
    for (int k = 0; k < n; ++k) {
        mireg_ctx *c = B->ctx[idx[k]];
        const Run &R = run[k];
        const long long N = c->N();
        if (R.x_is_s) {
            hipError_t e = hipMemcpyAsync(x[k], c->vec<T>(2), 3 * N * sizeof(T), hipMemcpyDeviceToDevice, B->stream);
            if (e != hipSuccess) return B->fail(MIREG_E_HIP, "copy: %s", hipGetErrorString(e));
        } else if (R.it > 0) {
            cx<T> *xh[3], *sh[3];
            for (int a = 0; a < 3; ++a) {
                xh[a] = c->khat<T>(KV_X, a);
                sh[a] = c->khat<T>(KV_S, a);
            }
            T *xp[3] = {x[k], x[k] + N, x[k] + 2 * N};
            Phase ph(c, 0);
            krylov_inverse<T>(c->g, xh, R.pending ? sh : nullptr, c->dres + 3, xp, static_cast<cx<T> *>(c->spec),
                              twiddles<T>(c), B->stream);
        } else {
            fill<T>(3 * N, (T)0, x[k], B->stream);
        }
        if (iters) iters[k] = R.it;
        if (relres) relres[k] = R.r0 > 0 ? R.rnorm / R.r0 : 0.0;
        if (status) status[k] = R.st;
        if (matvecs) matvecs[k] = R.mv;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return B->fail(MIREG_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return MIREG_OK;
}

// Lockstep GN (Algorithm "outer iteration" for every problem, impl_gn's
// arithmetic): the Newton steps of all problems that have not stopped are
// one batched PCG; the objective, gradient and line search run problem by
// problem on the common stream.
template <typename T, typename S>
int batch_gn(mireg_batch *B, T *const *v_io, const mireg_solve_opts *o, mireg_report *reps) {
    auto t0 = std::chrono::steady_clock::now();
    const int P = (int)B->ctx.size();
    struct St {
        mireg_report R{};
        double J = 0, gn = 0, g0 = 0;
        int k = 0;
        bool done = false;
        long long coarse0 = 0;
    };
    std::vector<St> st(P);
    int rc;
    double pcg_s = 0;
    int pcg_calls = 0;
    for (int p = 0; p < P; ++p) {
        mireg_ctx *c = B->ctx[p];
        const long long n = 3 * c->N();
        T *g = c->vec<T>(4), *vk = c->vec<T>(6);
        if ((rc = impl_set_velocity<T, S>(c, v_io[p]))) return batch_ctx_error(B, c, rc);
        hipError_t e = hipMemcpyAsync(vk, v_io[p], n * sizeof(T), hipMemcpyDeviceToDevice, B->stream);
        if (e != hipSuccess) return B->fail(MIREG_E_HIP, "copy: %s", hipGetErrorString(e));
        if ((rc = impl_objective<T, S>(c, &st[p].J, nullptr, nullptr))) return batch_ctx_error(B, c, rc);
        if ((rc = impl_gradient<T, S>(c, g, &st[p].gn))) return batch_ctx_error(B, c, rc);
        st[p].R.pde_solves += 3;  // the paper's count for J and g at the initial velocity
        st[p].g0 = st[p].gn;
        st[p].R.J0 = st[p].J;
        st[p].R.gnorm0 = st[p].g0;
        st[p].coarse0 = c->coarse_matvecs;
    }
    for (;;) {
        std::vector<int> A;
        std::vector<const T *> rhs;
        std::vector<T *> vts;
        std::vector<double> eps;
        for (int p = 0; p < P; ++p) {
            St &s = st[p];
            if (s.done) continue;
            if (o->log_level > 0)
                fprintf(stderr, "[mireg batch %d] gn %d J %.6e |g| %.6e |g|/|g0| %.3e\n", p, s.k, s.J, s.gn,
                        s.g0 > 0 ? s.gn / s.g0 : 0.0);
            if (s.gn <= o->grad_rtol * s.g0) {
                s.R.status = MIREG_CONVERGED_REL;
                s.done = true;
            } else if (s.gn <= o->grad_atol) {
                s.R.status = MIREG_CONVERGED_ABS;
                s.done = true;
            } else if (s.k >= o->max_gn) {
                s.R.status = MIREG_MAXIT;
                s.done = true;
            }
            if (s.done) continue;
            mireg_ctx *c = B->ctx[p];
            const long long n = 3 * c->N();
            T *rv = c->vec<T>(7);
            affine<T>(n, c->vec<T>(4), -1.0, 0.0, rv, B->stream);
            A.push_back(p);
            rhs.push_back(rv);
            vts.push_back(c->vec<T>(5));
            eps.push_back(std::fmin(0.5, std::sqrt(s.gn / s.g0)));
        }
        if (A.empty()) break;
        std::vector<int> its(A.size()), pst(A.size()), mv(A.size());
        const auto tp = std::chrono::steady_clock::now();
        if ((rc = batch_pcg<T, S>(B, A, rhs.data(), vts.data(), eps.data(), o->max_pcg, its.data(), nullptr,
                                  pst.data(), mv.data())))
            return rc;
        if (o->log_level > 1) {
            hipStreamSynchronize(B->stream);
            pcg_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
            ++pcg_calls;
        }
        for (size_t a = 0; a < A.size(); ++a) {
            const int p = A[a];
            St &s = st[p];
            mireg_ctx *c = B->ctx[p];
            const long long n = 3 * c->N();
            T *g = c->vec<T>(4), *vt = c->vec<T>(5), *vk = c->vec<T>(6);
            s.R.matvecs += mv[a];
            s.R.pcg_iters += its[a];
            s.R.pde_solves += 2 * mv[a];
            s.R.neg_curv += pst[a] == MIREG_NEG_CURV;
            double slope = 0;
            if ((rc = dot_h<T>(c, g, vt, n, &slope))) return batch_ctx_error(B, c, rc);
            double alpha = 1.0, Jt = 0;
            bool accepted = false;
            for (int ls = 0; ls < o->max_ls; ++ls) {
                xpay<T>(n, vk, alpha, vt, c->f<T>(c->v), B->stream);
                c->invalidate();
                if ((rc = impl_objective<T, S>(c, &Jt, nullptr, nullptr))) return batch_ctx_error(B, c, rc);
                s.R.ls_trials += 1;
                s.R.pde_solves += 1;
                if (Jt <= s.J + o->armijo_c1 * alpha * slope) {
                    accepted = true;
                    break;
                }
                alpha *= 0.5;
            }
            if (!accepted) {
                hipError_t e = hipMemcpyAsync(c->v, vk, n * sizeof(T), hipMemcpyDeviceToDevice, B->stream);
                if (e != hipSuccess) return B->fail(MIREG_E_HIP, "copy: %s", hipGetErrorString(e));
                c->invalidate();
                s.R.status = MIREG_LS_FAIL;
                s.done = true;
                continue;
            }
            hipError_t e = hipMemcpyAsync(vk, c->v, n * sizeof(T), hipMemcpyDeviceToDevice, B->stream);
            if (e != hipSuccess) return B->fail(MIREG_E_HIP, "copy: %s", hipGetErrorString(e));
            s.J = Jt;
            if ((rc = impl_gradient<T, S>(c, g, &s.gn))) return batch_ctx_error(B, c, rc);
            s.R.pde_solves += 1;
            ++s.k;
        }
    }
    for (int p = 0; p < P; ++p) {
        St &s = st[p];
        mireg_ctx *c = B->ctx[p];
        const long long N = c->N(), n = 3 * N;
        s.R.gn_iters = s.k;
        s.R.J = s.J;
        s.R.gnorm = s.gn;
        s.R.gnorm_rel = s.g0 > 0 ? s.gn / s.g0 : 0.0;
        ensure_state<T, S>(c);
        sumsq_diff<T, T>(c->f<T>(c->m) + c->p.nt * N, c->f<T>(c->mR), N, c->partials, c->dres, B->stream);
        if ((rc = readback(c, 1))) return batch_ctx_error(B, c, rc);
        const double num = c->hres[0];
        sumsq_diff<T, T>(c->f<T>(c->mT), c->f<T>(c->mR), N, c->partials, c->dres, B->stream);
        if ((rc = readback(c, 1))) return batch_ctx_error(B, c, rc);
        s.R.mismatch_rel = c->hres[0] > 0 ? num / c->hres[0] : 0.0;
        hipError_t e = hipMemcpyAsync(v_io[p], c->vec<T>(6), n * sizeof(T), hipMemcpyDeviceToDevice, B->stream);
        if (e != hipSuccess) return B->fail(MIREG_E_HIP, "copy: %s", hipGetErrorString(e));
        s.R.coarse_matvecs = (int)(c->coarse_matvecs - s.coarse0);
    }
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return B->fail(MIREG_E_HIP, "synchronise: %s", hipGetErrorString(e));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (o->log_level > 1)
        fprintf(stderr, "[mireg batch] %.4f s, of which %.4f s in %d lockstep PCG solves\n", secs, pcg_s, pcg_calls);
    for (int p = 0; p < P; ++p) {
        st[p].R.seconds = secs;
        if (reps) reps[p] = st[p].R;
    }
    return MIREG_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

void mireg_default_params(mireg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->n[0] = p->n[1] = p->n[2] = 32;
    p->nt = 4;
    p->interp_order = 3;
    p->reg = MIREG_H1;
    p->div = MIREG_DIV_NONE;
    p->beta_v = 1e-2;
    p->beta_w = 0.0;
    p->dtype = MIREG_F32;
}

void mireg_default_solve_opts(mireg_solve_opts *o) {
    if (!o) return;
    o->grad_rtol = 5e-2;
    o->grad_atol = 1e-6;
    o->max_gn = 50;
    o->max_pcg = 100;
    o->armijo_c1 = 1e-4;
    o->max_ls = 10;
    o->log_level = 0;
}

int mireg_create(const mireg_params *p, void *stream, mireg_ctx **out) {
    if (!p || !out) return MIREG_E_ARG;
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (!supported_axis(p->n[a])) return MIREG_E_SHAPE;
    if (p->nt < 1 || p->nt > 64 || (p->interp_order != 1 && p->interp_order != 3) ||
        (p->reg != MIREG_H1 && p->reg != MIREG_H2) || p->div < 0 || p->div > 2 || !(p->beta_v > 0) ||
        !(p->beta_w >= 0) || (p->div == MIREG_DIV_NEAR && !(p->beta_w > 0)) ||
        (p->dtype != MIREG_F32 && p->dtype != MIREG_F64 && p->dtype != MIREG_F32_H16))
        return MIREG_E_ARG;
    mireg_ctx *ctx = new (std::nothrow) mireg_ctx;
    if (!ctx) return MIREG_E_NOMEM;
    ctx->p = *p;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->g.n1 = p->n[0];
    ctx->g.n2 = p->n[1];
    ctx->g.n3 = p->n[2];
    ctx->g.k3 = p->n[2] / 2 + 1;
    ctx->g.N = (long long)p->n[0] * p->n[1] * p->n[2];
    ctx->g.NS = (long long)p->n[0] * p->n[1] * ctx->g.k3;
    // MIREG_LDS_STENCIL=0 makes every semi-Lagrangian step gather from global
    // memory (the path taken by tiles whose stencil box exceeds LDS).
    {
        const char *e = getenv("MIREG_LDS_STENCIL");
        ctx->g.lds_cap = (e && atoi(e) == 0) ? 0 : INT_MAX;
        // MIREG_SL_TILE selects the tile shape of the transport kernels:
        // 0: 4x8x32, 1: 8x8x16, 2: 8x16x16 (x1 x x2 x x3).
        const char *t = getenv("MIREG_SL_TILE");
        ctx->g.sl_tile = t ? atoi(t) : 1;
        if (ctx->g.sl_tile < 0 || ctx->g.sl_tile > 2) ctx->g.sl_tile = 1;
        // MIREG_TILE_BOXES=0: each transport launch reduces its tiles' stencil
        // boxes itself instead of reading the ones measured with X and Y.
        const char *b = getenv("MIREG_TILE_BOXES");
        ctx->tile_boxes = !(b && atoi(b) == 0);
    }
    ctx->elem = p->dtype == MIREG_F64 ? 8 : 4;
    const size_t F = (size_t)ctx->g.N * ctx->elem;
    // adjoint history and incremental fields: FP16 in the F32_H16 mode
    const size_t FS = (size_t)ctx->g.N * (p->dtype == MIREG_F32_H16 ? 2 : ctx->elem);
    const int nt = p->nt;
    int rc = MIREG_OK;
    if (!rc) rc = alloc(ctx, &ctx->mT, F);
    if (!rc) rc = alloc(ctx, &ctx->mR, F);
    if (!rc) rc = alloc(ctx, &ctx->v, 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->X, 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->Y, 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->m, (size_t)(nt + 1) * F);
    if (!rc) rc = alloc(ctx, &ctx->gradm, (size_t)(nt + 1) * 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->d, F);
    if (!rc) rc = alloc(ctx, &ctx->lam, (size_t)(nt + 1) * FS);
    if (!rc) rc = alloc(ctx, &ctx->q, 2 * FS);
    if (!rc) rc = alloc(ctx, &ctx->b, 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->vecs, (size_t)mireg_ctx::kVecs * 3 * F);
    if (!rc) rc = alloc(ctx, &ctx->spec, (size_t)6 * ctx->g.NS * 2 * ctx->elem);
    if (!rc) rc = alloc(ctx, &ctx->kspec, (size_t)15 * ctx->g.NS * 2 * ctx->elem);
    for (int a = 0; a < 3 && !rc; ++a) rc = alloc(ctx, &ctx->tw[a], (size_t)p->n[a] * 2 * ctx->elem);
    if (!rc) rc = alloc(ctx, (void **)&ctx->partials, 4 * kRedBlocks * sizeof(double));
    if (!rc) rc = alloc(ctx, (void **)&ctx->xpart, ((size_t)ctx->g.n2 * ctx->g.k3 / 8 + 16) * sizeof(double));
    if (!rc) rc = alloc(ctx, (void **)&ctx->dres, 8 * sizeof(double));
    if (!rc) rc = alloc(ctx, (void **)&ctx->tbox_X, (size_t)sl_box_words(ctx->g) * sizeof(int));
    if (!rc) rc = alloc(ctx, (void **)&ctx->tbox_Y, (size_t)sl_box_words(ctx->g) * sizeof(int));
    if (!rc && hipHostMalloc((void **)&ctx->hres, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        rc = ctx->fail(MIREG_E_NOMEM, "hipHostMalloc failed");
    if (!rc) rc = DISPATCH(ctx, (make_twiddles<T, S>(ctx)));
    if (!rc && (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess))
        rc = ctx->fail(MIREG_E_HIP, "hipEventCreate failed");
    if (!rc) {
        // zero initial velocity
        if (hipMemsetAsync(ctx->v, 0, 3 * F, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            rc = ctx->fail(MIREG_E_HIP, "initialising the velocity failed");
    }
    if (rc) {
        fprintf(stderr, "[mireg] create failed: %s\n", ctx->err.c_str());
        mireg_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return MIREG_OK;
}

int mireg_destroy(mireg_ctx *ctx) {
    if (!ctx) return MIREG_E_ARG;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    else hipDeviceSynchronize();
    if (ctx->coarse) mireg_destroy(ctx->coarse);
    if (ctx->mv_exec) hipGraphExecDestroy(ctx->mv_exec);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    for (void *p : ctx->allocs) hipFree(p);
    if (ctx->hres) hipHostFree(ctx->hres);
    if (ctx->ev0) hipEventDestroy(ctx->ev0);
    if (ctx->ev1) hipEventDestroy(ctx->ev1);
    if (ctx->jlog) fclose(ctx->jlog);
    delete ctx;
    return MIREG_OK;
}

const char *mireg_last_error(const mireg_ctx *ctx) { return ctx ? ctx->err.c_str() : mireg::noalloc_error(); }

size_t mireg_workspace_bytes(const mireg_ctx *ctx) { return ctx ? ctx->bytes : 0; }

int mireg_set_images(mireg_ctx *ctx, const void *mT, const void *mR) {
    if (!ctx || !mT || !mR) return ctx ? ctx->fail(MIREG_E_ARG, "null image pointer") : MIREG_E_ARG;
    return DISPATCH(ctx, (impl_set_images<T, S>(ctx, (const T *)mT, (const T *)mR)));
}

int mireg_set_velocity(mireg_ctx *ctx, const void *v) {
    if (!ctx || !v) return ctx ? ctx->fail(MIREG_E_ARG, "null velocity pointer") : MIREG_E_ARG;
    return DISPATCH(ctx, (impl_set_velocity<T, S>(ctx, (const T *)v)));
}

int mireg_get_velocity(mireg_ctx *ctx, void *v) {
    if (!ctx || !v) return ctx ? ctx->fail(MIREG_E_ARG, "null velocity pointer") : MIREG_E_ARG;
    HIP_OK(hipMemcpyAsync(v, ctx->v, 3 * ctx->N() * ctx->elem, hipMemcpyDeviceToDevice, ctx->stream));
    return MIREG_OK;
}

int mireg_objective(mireg_ctx *ctx, double *J, double *mismatch, double *reg) {
    if (!ctx) return MIREG_E_ARG;
    return DISPATCH(ctx, (impl_objective<T, S>(ctx, J, mismatch, reg)));
}

int mireg_gradient(mireg_ctx *ctx, void *g, double *gnorm) {
    if (!ctx || !g) return ctx ? ctx->fail(MIREG_E_ARG, "null gradient pointer") : MIREG_E_ARG;
    return DISPATCH(ctx, (impl_gradient<T, S>(ctx, (T *)g, gnorm)));
}

int mireg_hessian_matvec(mireg_ctx *ctx, const void *vt, void *Hvt) {
    if (!ctx || !vt || !Hvt) return ctx ? ctx->fail(MIREG_E_ARG, "null matvec pointer") : MIREG_E_ARG;
    if (vt == Hvt) return ctx->fail(MIREG_E_ARG, "vt and Hvt must not alias");
    return DISPATCH(ctx, (matvec_graph<T, S>(ctx, (const T *)vt, (T *)Hvt)));
}

int mireg_precond_apply(mireg_ctx *ctx, const void *r, void *z) {
    if (!ctx || !r || !z) return ctx ? ctx->fail(MIREG_E_ARG, "null pointer") : MIREG_E_ARG;
    if (ctx->pc_kind == MIREG_PC_TWO_LEVEL && !ctx->have_images)
        return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    return DISPATCH(ctx, (apply_precond<T, S>(ctx, (const T *)r, (T *)z, 1.0)));
}

int mireg_set_tuning(mireg_ctx *ctx, int tile_shape, int x1_narrow) {
    if (!ctx) return MIREG_E_ARG;
    if (tile_shape < 0 || tile_shape > 2 || (x1_narrow != 0 && x1_narrow != 1))
        return ctx->fail(MIREG_E_ARG, "tile shape must be 0, 1 or 2 and the x1 width 0 or 1");
    // only FP32 grids with 256-point x1 lines have a second Krylov width
    if (ctx->p.dtype == MIREG_F64 || ctx->g.n1 != 256) x1_narrow = 0;
    set_x1_narrow(ctx, x1_narrow);
    return DISPATCH(ctx, (set_tile<T, S>(ctx, tile_shape), MIREG_OK));
}

int mireg_get_tuning(const mireg_ctx *ctx, int *tile_shape, int *x1_narrow) {
    if (!ctx) return MIREG_E_ARG;
    if (tile_shape) *tile_shape = ctx->g.sl_tile;
    if (x1_narrow) *x1_narrow = ctx->g.x1_narrow;
    return MIREG_OK;
}

int mireg_set_log_jsonl(mireg_ctx *ctx, const char *path) {
    if (!ctx) return MIREG_E_ARG;
    if (ctx->jlog) {
        fclose(ctx->jlog);
        ctx->jlog = nullptr;
    }
    if (path && path[0]) {
        ctx->jlog = fopen(path, "a");
        if (!ctx->jlog) return ctx->fail(MIREG_E_ARG, "cannot open %s for appending", path);
    }
    return MIREG_OK;
}

int mireg_set_graphs(mireg_ctx *ctx, int on) {
    if (!ctx) return MIREG_E_ARG;
    ctx->use_graphs = on != 0;
    if (!ctx->use_graphs && ctx->mv_exec) {
        hipGraphExecDestroy(ctx->mv_exec);
        ctx->mv_exec = nullptr;
    }
    return MIREG_OK;
}

int mireg_autotune(mireg_ctx *ctx, int reps, double *ms, int *shape) {
    if (!ctx) return MIREG_E_ARG;
    if (reps < 1) return ctx->fail(MIREG_E_ARG, "reps must be >= 1");
    if (ctx->g.lds_cap == 0) {  // staging switched off: every shape gathers globally
        if (shape) *shape = ctx->g.sl_tile;
        return MIREG_OK;
    }
    return DISPATCH(ctx, (impl_autotune<T, S>(ctx, reps, ms, shape)));
}

int mireg_set_precond(mireg_ctx *ctx, int kind, double kappa, int max_inner) {
    if (!ctx) return MIREG_E_ARG;
    if (kind != MIREG_PC_SPECTRAL && kind != MIREG_PC_TWO_LEVEL) return ctx->fail(MIREG_E_ARG, "unknown preconditioner");
    if (!(kappa > 0 && kappa < 1) || max_inner < 1) return ctx->fail(MIREG_E_ARG, "kappa must be in (0, 1), max_inner >= 1");
    if (kind == MIREG_PC_TWO_LEVEL && !ctx->coarse) {
        if (ctx->g.n1 < 16 || ctx->g.n2 < 16 || ctx->g.n3 < 16 || !supported_axis(ctx->g.n1 / 2) ||
            !supported_axis(ctx->g.n2 / 2) || !supported_axis(ctx->g.n3 / 2))
            return ctx->fail(MIREG_E_SHAPE,
                             "the two-level preconditioner needs at least 16 points per axis and a supported n/2");
        mireg_params p = ctx->p;
        p.n[0] = ctx->g.n1 / 2;
        p.n[1] = ctx->g.n2 / 2;
        p.n[2] = ctx->g.n3 / 2;
        int rc = mireg_create(&p, ctx->stream, &ctx->coarse);
        if (rc) return ctx->fail(rc, "creating the coarse context failed");
        ctx->coarse_images = false;
        ctx->coarse_vel_version = -1;
    }
    ctx->pc_kind = kind;
    ctx->pc_kappa = kappa;
    ctx->pc_max_inner = max_inner;
    return MIREG_OK;
}

int mireg_pcg_solve(mireg_ctx *ctx, const void *rhs, void *x, double rtol, int maxit, int *iters,
                    double *relres, int *status) {
    if (!ctx || !rhs || !x) return ctx ? ctx->fail(MIREG_E_ARG, "null pointer") : MIREG_E_ARG;
    if (maxit < 0 || !(rtol >= 0)) return ctx->fail(MIREG_E_ARG, "invalid rtol/maxit");
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    return DISPATCH(ctx, (impl_pcg<T, S>(ctx, (const T *)rhs, (T *)x, rtol, maxit, iters, relres, status)));
}

int mireg_gn_solve(mireg_ctx *ctx, void *v_inout, const mireg_solve_opts *opts, mireg_report *rep) {
    if (!ctx || !v_inout) return ctx ? ctx->fail(MIREG_E_ARG, "null velocity pointer") : MIREG_E_ARG;
    if (!ctx->have_images) return ctx->fail(MIREG_E_STATE, "set_images has not been called");
    mireg_solve_opts o;
    mireg_default_solve_opts(&o);
    if (opts) o = *opts;
    if (o.max_gn < 0 || o.max_pcg < 0 || o.max_ls < 0) return ctx->fail(MIREG_E_ARG, "negative iteration cap");
    return DISPATCH(ctx, (impl_gn<T, S>(ctx, (T *)v_inout, &o, rep)));
}

int mireg_batch_create(mireg_ctx *const *ctxs, int n, mireg_batch **out) {
    if (!ctxs || !out || n < 1) return MIREG_E_ARG;
    *out = nullptr;
    for (int i = 0; i < n; ++i)
        if (!ctxs[i]) return MIREG_E_ARG;
    const mireg_ctx *c0 = ctxs[0];
    for (int i = 1; i < n; ++i) {
        const mireg_ctx *c = ctxs[i];
        if (c->p.dtype != c0->p.dtype || c->p.nt != c0->p.nt || c->p.interp_order != c0->p.interp_order ||
            c->stream != c0->stream || c->g.sl_tile != c0->g.sl_tile || c->g.lds_cap != c0->g.lds_cap)
            return MIREG_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return MIREG_E_ARG;
    }
    mireg_batch *B = new (std::nothrow) mireg_batch;
    if (!B) return MIREG_E_NOMEM;
    B->ctx.assign(ctxs, ctxs + n);
    B->stream = c0->stream;
    mireg_ctx *cm = ctxs[0];
    const size_t bytes = DISPATCH(cm, (batch_table_bytes<T, S>(n, cm->p.nt)));
    // pointer tables of one PCG iteration: under 1 KB per problem
    B->arena.cap = (size_t)4096 * n + (size_t)64 * 1024;
    if (hipMalloc(&B->dtab, bytes) != hipSuccess || hipHostMalloc(&B->htab, bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&B->arena.d, B->arena.cap) != hipSuccess ||
        hipHostMalloc((void **)&B->arena.h, B->arena.cap, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&B->tab_done, hipEventDisableTiming) != hipSuccess) {
        mireg_batch_destroy(B);
        return MIREG_E_NOMEM;
    }
    *out = B;
    return MIREG_OK;
}

int mireg_batch_destroy(mireg_batch *b) {
    if (!b) return MIREG_E_ARG;
    if (b->stream) hipStreamSynchronize(b->stream);
    else hipDeviceSynchronize();
    if (b->dtab) hipFree(b->dtab);
    if (b->htab) hipHostFree(b->htab);
    if (b->arena.d) hipFree(b->arena.d);
    if (b->arena.h) hipHostFree(b->arena.h);
    if (b->tab_done) hipEventDestroy(b->tab_done);
    delete b;
    return MIREG_OK;
}

const char *mireg_batch_last_error(const mireg_batch *b) { return b ? b->err.c_str() : "null batch"; }

int mireg_batch_pcg_solve(mireg_batch *b, const void *const *rhs, void *const *x, const double *rtol, int maxit,
                          int *iters, double *relres, int *status) {
    if (!b || !rhs || !x || !rtol) return b ? b->fail(MIREG_E_ARG, "null pointer") : MIREG_E_ARG;
    const int P = (int)b->ctx.size();
    if (maxit < 0) return b->fail(MIREG_E_ARG, "negative iteration cap");
    std::vector<int> idx(P);
    for (int p = 0; p < P; ++p) {
        idx[p] = p;
        if (!rhs[p] || !x[p] || !(rtol[p] >= 0)) return b->fail(MIREG_E_ARG, "problem %d: invalid argument", p);
        if (!b->ctx[p]->have_images) return b->fail(MIREG_E_STATE, "problem %d: set_images has not been called", p);
        if (b->ctx[p]->pc_kind != MIREG_PC_SPECTRAL)
            return b->fail(MIREG_E_ARG, "problem %d: batched PCG takes the spectral preconditioner", p);
    }
    mireg_ctx *c0 = b->ctx[0];
    return DISPATCH(c0, (batch_pcg<T, S>(b, idx, reinterpret_cast<const T *const *>(rhs),
                                          reinterpret_cast<T *const *>(x), rtol, maxit, iters, relres, status,
                                          nullptr)));
}

int mireg_batch_gn_solve(mireg_batch *b, void *const *v_inout, const mireg_solve_opts *opts, mireg_report *reps) {
    if (!b || !v_inout) return b ? b->fail(MIREG_E_ARG, "null pointer") : MIREG_E_ARG;
    const int P = (int)b->ctx.size();
    for (int p = 0; p < P; ++p) {
        if (!v_inout[p]) return b->fail(MIREG_E_ARG, "problem %d: null velocity", p);
        if (!b->ctx[p]->have_images) return b->fail(MIREG_E_STATE, "problem %d: set_images has not been called", p);
        if (b->ctx[p]->pc_kind != MIREG_PC_SPECTRAL)
            return b->fail(MIREG_E_ARG, "problem %d: batched solves take the spectral preconditioner", p);
    }
    mireg_solve_opts o;
    mireg_default_solve_opts(&o);
    if (opts) o = *opts;
    if (o.max_gn < 0 || o.max_pcg < 0 || o.max_ls < 0) return b->fail(MIREG_E_ARG, "negative iteration cap");
    mireg_ctx *c0 = b->ctx[0];
    return DISPATCH(c0, (batch_gn<T, S>(b, reinterpret_cast<T *const *>(v_inout), &o, reps)));
}

int mireg_op(mireg_ctx *ctx, int opcode, const void *in, void *out, double arg) {
    if (!ctx || !in || !out) return ctx ? ctx->fail(MIREG_E_ARG, "null pointer") : MIREG_E_ARG;
    return DISPATCH(ctx, (impl_op<T, S>(ctx, opcode, (const T *)in, (T *)out, arg)));
}

int mireg_kernel_stats_enable(mireg_ctx *ctx, int on) {
    if (!ctx) return MIREG_E_ARG;
    ctx->stats.stream = ctx->stream;
    ctx->stats_on = on != 0;
    return MIREG_OK;
}

int mireg_kernel_stats_read(mireg_ctx *ctx, mireg_kernel_stat *out, int max, int *count, int reset) {
    if (!ctx || (max > 0 && !out)) return MIREG_E_ARG;
    ctx->stats.harvest();
    int k = 0;
    for (int id = 0; id < K_COUNT && k < max; ++id) {
        const auto &a = ctx->stats.acc[id];
        if (a.n == 0) continue;
        std::memset(&out[k], 0, sizeof out[k]);
        std::snprintf(out[k].name, sizeof out[k].name, "%s", kKernelNames[id]);
        out[k].launches = a.n;
        out[k].total_ms = a.ms;
        out[k].bytes_per_launch = a.bytes / a.n;
        ++k;
    }
    if (count) *count = k;
    if (reset) ctx->stats.reset();
    return MIREG_OK;
}

int mireg_timers_enable(mireg_ctx *ctx, int on) {
    if (!ctx) return MIREG_E_ARG;
    ctx->tm.on = on != 0;
    return MIREG_OK;
}

int mireg_timers_read(mireg_ctx *ctx, mireg_timers *t, int reset) {
    if (!ctx || !t) return MIREG_E_ARG;
    t->fft_ms = ctx->tm.fft_ms;
    t->interp_ms = ctx->tm.interp_ms;
    t->other_ms = ctx->tm.other_ms;
    t->launches = ctx->tm.launches;
    if (reset) {
        bool on = ctx->tm.on;
        ctx->tm = Timers{};
        ctx->tm.on = on;
    }
    return MIREG_OK;
}

}  // extern "C"
