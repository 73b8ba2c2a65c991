/*
 * mireg: reduced-space Gauss-Newton-Krylov registration hot path on one
 * MI355X (gfx950), after Mang, Gholami, Davatzikos and Biros, "CLAIRE: A
 * distributed-memory solver for constrained large deformation diffeomorphic
 * image registration" (arXiv 1808.04487).
 *
 * Problem (Sec. 2.1, eq. "varopt"): find a stationary velocity v on the
 * periodic box (0, 2 pi)^3 minimising
 *     J(v) = 1/2 ||m(1) - mR||^2 + beta_v/2 <A v, v> [+ beta_w/2 (||grad w||^2 + ||w||^2)]
 * where m solves dm/dt + grad m . v = 0, m(0) = mT, and w = div v.
 *
 * Conventions shared by every entry point:
 *  - Grid: n = (n1, n2, n3), each a power of two in [8, 512] or one of
 *    48, 80, 96, 160 (radix-3 and radix-5 transforms); point
 *    (i1, i2, i3) sits at x_a = 2 pi i_a / n_a.  Scalar fields are dense
 *    C-ordered [n1][n2][n3] arrays (x3 fastest); vector fields are
 *    [3][n1][n2][n3].  Element type is the context's boundary type: float
 *    for MIREG_F32 and MIREG_F32_H16, double for MIREG_F64.
 *  - Memory: every field pointer is a DEVICE pointer owned by the caller,
 *    borrowed for the duration of the call only.  Scalars (J, norms, counts)
 *    are HOST pointers.  mireg_set_images / mireg_set_velocity copy their
 *    input into library-owned device memory.
 *  - Streams: all work is enqueued on the stream given to mireg_create
 *    (a hipStream_t, NULL for the default stream).  Calls returning host
 *    scalars synchronise that stream before returning.  A context is not
 *    thread safe; use one context per host thread.
 *  - Errors: functions return MIREG_OK (0) or a negative MIREG_E_* code;
 *    mireg_last_error gives a message.  Non-convergence of a solve is not an
 *    error: it is reported in mireg_report.status.
 *  - Inner products and norms are the trapezoidal L2 ones of the grid,
 *    h1 h2 h3 sum(a b), accumulated in FP64 for both dtypes.
 */
#ifndef MIREG_H
#define MIREG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MIREG_OK = 0,
    MIREG_E_ARG = -1,       /* invalid argument or NULL pointer */
    MIREG_E_SHAPE = -2,     /* unsupported grid size */
    MIREG_E_STATE = -3,     /* call order violated (e.g. no images set) */
    MIREG_E_HIP = -4,       /* a HIP runtime call failed */
    MIREG_E_NOMEM = -5,     /* device allocation failed */
    MIREG_E_NONFINITE = -6  /* NaN or Inf in an input */
};

/* Arithmetic and storage: F32 and F64 compute and store every field in that
 * type; F32_H16 computes in FP32 and exchanges FP32 fields at the boundary,
 * but holds the adjoint history lambda^j and the incremental fields mt, lt
 * (the fields the Hessian matvec streams) in FP16.  The state history m^j
 * stays FP32: lambda(1) = mR - m(1) is a small difference of O(1) values,
 * so FP16 rounding of m would reach the gradient amplified by |m|/|lambda|.
 * Reductions are FP64 always. */
typedef enum { MIREG_F32 = 0, MIREG_F64 = 1, MIREG_F32_H16 = 2 } mireg_dtype;

/* Regularisation operator A = B*B (Sec. 2.1): H1 seminorm B = grad gives
 * A = -Lap; H2 seminorm B = -Lap gives A = Lap^2. */
typedef enum { MIREG_H1 = 1, MIREG_H2 = 2 } mireg_reg;

/* Projection K of the reduced gradient (Sec. 2.2): identity without a
 * divergence constraint, the near-incompressible operator
 * K = I - grad (beta_v (beta_w(-Lap + I))^{-1} + I)^{-1} Lap^{-1} div, or the
 * Leray projection I - grad Lap^{-1} div of the incompressible model. */
typedef enum { MIREG_DIV_NONE = 0, MIREG_DIV_NEAR = 1, MIREG_DIV_LERAY = 2 } mireg_div;

typedef struct {
    int n[3];           /* grid size: powers of two in [8, 512], or 48, 80, 96, 160 */
    int nt;             /* number of time steps (the paper uses 4), 1..64 */
    int interp_order;   /* 3: tricubic Lagrange (paper), 1: trilinear */
    int reg;            /* mireg_reg */
    int div;            /* mireg_div */
    double beta_v;      /* > 0, weight of the velocity regulariser */
    double beta_w;      /* >= 0, weight of the divergence penalty (DIV_NEAR) */
    int dtype;          /* mireg_dtype of every field passed in or out */
} mireg_params;

typedef struct {
    double grad_rtol;   /* stop when ||g_k|| <= grad_rtol ||g_0|| (paper: 5e-2) */
    double grad_atol;   /* or when ||g_k|| <= grad_atol (paper: 1e-6) */
    int max_gn;         /* GN iteration cap (50) */
    int max_pcg;        /* PCG iteration cap per Newton step (100) */
    double armijo_c1;   /* sufficient-decrease constant (1e-4) */
    int max_ls;         /* line-search trials, step halved each time (10) */
    int log_level;      /* 0 silent, 1 one line per GN iteration on stderr */
} mireg_solve_opts;

enum {
    MIREG_CONVERGED_REL = 1,
    MIREG_CONVERGED_ABS = 2,
    MIREG_MAXIT = 3,
    MIREG_LS_FAIL = 4,
    MIREG_NEG_CURV = 5  /* PCG met <s, H s> <= 0 (Algorithm "inner iteration" has no
                           safeguard; the solve stops there and keeps its iterate) */
};

typedef struct {
    int status;         /* MIREG_CONVERGED_REL / _ABS / MIREG_MAXIT / MIREG_LS_FAIL: why the
                           outer loop ended (a PCG stop on curvature is counted in neg_curv;
                           GN goes on with the direction that PCG returned) */
    int gn_iters;       /* accepted GN steps */
    int matvecs;        /* Hessian matvecs: the PCG iterations, plus one for each PCG
                           solve that stopped on non-positive curvature */
    int pde_solves;     /* PDE solves as the paper's tables count them (Sec. 4.7, Table
                           S3: #PDE = 2 #matvecs + 2 #iter + 3 with one trial per step):
                           3 for J and g at the initial velocity, 2 per matvec, 1 per
                           line-search trial, 1 per accepted step (the new adjoint) */
    int pcg_iters;
    int ls_trials;      /* objective evaluations in the line search */
    double J0, J;       /* objective at the initial and final velocity */
    double mismatch_rel;/* ||m(1) - mR||^2 / ||mT - mR||^2 at the final velocity */
    double gnorm0, gnorm, gnorm_rel;
    double seconds;     /* wall time of the solve */
    int coarse_matvecs; /* coarse-grid Hessian matvecs of the two-level preconditioner */
    int neg_curv;       /* Newton steps whose PCG stopped on <s, H s> <= 0 */
} mireg_report;

typedef struct mireg_ctx mireg_ctx;

/* Fill *p / *o with the defaults named above (n and beta_v still to set). */
void mireg_default_params(mireg_params *p);
void mireg_default_solve_opts(mireg_solve_opts *o);

/* Create a context for one problem size on the current HIP device and
 * allocate all of its device workspace (about 75 fields).  `stream` is a
 * hipStream_t or NULL.  Returns MIREG_E_SHAPE for unsupported sizes,
 * MIREG_E_ARG for invalid parameters, MIREG_E_NOMEM if allocation fails. */
int mireg_create(const mireg_params *p, void *stream, mireg_ctx **out);
int mireg_destroy(mireg_ctx *ctx);
const char *mireg_last_error(const mireg_ctx *ctx);
/* Bytes of device memory the context holds. */
size_t mireg_workspace_bytes(const mireg_ctx *ctx);

/* Template mT (transported from t = 0) and reference mR (Sec. 2.1), scalar
 * fields.  Copied; checked for NaN/Inf (MIREG_E_NONFINITE). */
int mireg_set_images(mireg_ctx *ctx, const void *mT, const void *mR);

/* Current velocity v, vector field.  Copied; checked for NaN/Inf; every
 * cached quantity that depends on v is invalidated.  The initial velocity
 * of a new context is zero. */
int mireg_set_velocity(mireg_ctx *ctx, const void *v);
int mireg_get_velocity(mireg_ctx *ctx, void *v);

/* Objective (eq. "varopt:objective") at the current v: *J = *mismatch +
 * *reg (host doubles; any may be NULL).  One state solve (Sec. 2.3.1). */
int mireg_objective(mireg_ctx *ctx, double *J, double *mismatch, double *reg);

/* Reduced gradient g = beta_v A v + K[int_0^1 lambda grad m dt] (eq.
 * "reduced-gradient") at the current v, written to the device vector field
 * g; *gnorm (may be NULL) gets its L2 norm.  State and adjoint solves. */
int mireg_gradient(mireg_ctx *ctx, void *g, double *gnorm);

/* Gauss-Newton Hessian matvec (eqs. "inc-state", "inc-adj",
 * "hessian-matvec", GN form of Sec. 2.3.2): Hvt = beta_v A vt +
 * K[int_0^1 lt grad m dt] at the current v.  vt and Hvt are device vector
 * fields and must not alias.  Incremental state and adjoint solves; no host
 * synchronisation. */
int mireg_hessian_matvec(mireg_ctx *ctx, const void *vt, void *Hvt);

/* Preconditioner z = M^{-1} r (see mireg_set_precond; by default the
 * spectral (beta_v A)^{-1} with the zero singular value of the regulariser
 * set to one, Sec. 2.3.3).  r and z may alias. */
int mireg_precond_apply(mireg_ctx *ctx, const void *r, void *z);

/* Preconditioner of PCG and of mireg_precond_apply (Sec. 2.3.3):
 *  MIREG_PC_SPECTRAL: M^{-1} = (beta_v A)^{-1} (the default);
 *  MIREG_PC_TWO_LEVEL: M^{-1} = Hreg^{-1/2} P^{-1} Hreg^{-1/2}, Hreg = beta_v A
 *    (symbol 1 at k = 0), where P approximates Hreg^{-1/2} H Hreg^{-1/2}: the
 *    modes with |k_a| < n_a/4 (F_L) are restricted spectrally to the n/2 grid
 *    (Q_R), solved there with CG to the relative tolerance kappa * eps_H on
 *    the coarse operator built from the restricted images and velocity
 *    (direct, non-Galerkin), and prolongated back (Q_P); the other modes
 *    (F_H) pass unchanged.  eps_H is the tolerance of the enclosing PCG (1
 *    for mireg_precond_apply); max_inner caps the coarse iterations.  The
 *    coarse context (n/2 per axis, every axis >= 16) is created on first use.
 * kappa in (0, 1) (the paper: 0.1).  MIREG_E_SHAPE if the grid is too small
 * or n/2 is not a supported size (48 and 80 have none). */
typedef enum { MIREG_PC_SPECTRAL = 0, MIREG_PC_TWO_LEVEL = 1 } mireg_precond_kind;
int mireg_set_precond(mireg_ctx *ctx, int kind, double kappa, int max_inner);

/* Launch-overhead and tuning controls (not in the paper; for many small
 * problems and for each grid size):
 * mireg_set_graphs: on != 0 makes PCG and mireg_hessian_matvec replay the
 *   Hessian matvec from a captured HIP graph (captured on a private stream,
 *   launched on the context's stream; re-captured when the velocity, the
 *   vt / Hvt pointers or the caller (PCG or the entry point) change); off
 *   while timers or kernel statistics are enabled.  Results are identical.  HIP
 *   invalidates a running capture when any thread uses the legacy (null)
 *   stream: with graphs on in one thread, other threads must keep their
 *   work off the null stream (mireg_create with a null stream uses it), or
 *   the capturing call fails with MIREG_E_HIP.
 * mireg_autotune: times `reps` PCG iterations (right-hand side: the current
 *   velocity; setup and final transform included) with each tile shape of
 *   the transport kernels (0: 4x8x32, 1: 8x8x16, 2: 8x16x16 points in x1 x
 *   x2 x x3) and, for FP32 grids with 256 points along x1, each workgroup
 *   width of the Krylov x1 passes (32 or 16 columns), and keeps the fastest
 *   pair; ms (host, 3 values, may be NULL) receives the mean time per
 *   iteration of each shape (its best width), *shape (may be NULL) the
 *   chosen shape.  The shapes compute identical bits; the widths group the
 *   FP64 partial sums of <s, H s> differently.  Needs set_images;
 *   synchronises.
 * mireg_get_tuning / mireg_set_tuning: the context's tile shape (0..2) and
 *   Krylov x1 width (1: 16 columns; forced to 0 where there is only one),
 *   e.g. to give the contexts of a lockstep batch one tuned shape; get takes
 *   host ints (either may be NULL); set re-measures the stencil boxes of the
 *   cached departure points; MIREG_E_ARG for values out of range. */
int mireg_set_graphs(mireg_ctx *ctx, int on);
int mireg_autotune(mireg_ctx *ctx, int reps, double *ms, int *shape);
int mireg_get_tuning(const mireg_ctx *ctx, int *tile_shape, int *x1_narrow);
int mireg_set_tuning(mireg_ctx *ctx, int tile_shape, int x1_narrow);

/* Per-iteration log of mireg_gn_solve (the paper's solver reports, Sec. 4,
 * list #iter, #matvecs, #PDE, mismatch and gradient norms per solve; this
 * adds one record per GN iteration).  path (host string) is opened for
 * appending; NULL or "" closes the log.  Each GN iteration appends one JSON
 * object on its own line, after its line search: {"event": "gn", "iter",
 * "J", "gnorm", "gnorm_rel" (at the iterate the step starts from), "eps_h",
 * "pcg_iters", "pcg_status", "pcg_matvecs", "slope" (<g, step>), "alpha"
 * (last step length tried), "accepted", "J_trial", and the running totals
 * "matvecs", "pde_solves", "ls_trials", "seconds"}; the solve ends with
 * {"event": "done", ...} carrying the fields of mireg_report.  The lockstep
 * batch solve writes no log.  MIREG_E_ARG if the file cannot be opened. */
int mireg_set_log_jsonl(mireg_ctx *ctx, const char *path);

/* PCG (Algorithm "inner iteration") for H x = rhs at the current v, x0 = 0;
 * stops when ||r|| <= rtol ||rhs|| (*status = MIREG_CONVERGED_REL, also for
 * rhs = 0), after maxit iterations (MIREG_MAXIT), or on non-positive
 * curvature <s, H s> <= 0 (MIREG_NEG_CURV: x is the iterate so far, or
 * M^{-1} rhs if the first direction had it).  *iters counts the completed
 * iterations (the matvec that found the curvature is not one); iters,
 * relres and status are host pointers and may be NULL. */
int mireg_pcg_solve(mireg_ctx *ctx, const void *rhs, void *x, double rtol, int maxit,
                    int *iters, double *relres, int *status);

/* Inexact GN-Krylov solve (Algorithm "outer iteration", Sec. 2.3.2) with
 * forcing eps_H = min(0.5, sqrt(||g_k||/||g_0||)) and Armijo line search,
 * starting from v_inout (device vector field; a warm start or zeros) and
 * writing the final velocity back to it.  opts may be NULL (defaults).
 * On return the context's current velocity is the final one. */
int mireg_gn_solve(mireg_ctx *ctx, void *v_inout, const mireg_solve_opts *opts,
                   mireg_report *rep);

/* Batched solves (not in the paper: many registration problems on one GPU).
 * A batch groups n >= 1 distinct contexts of any supported grid sizes that
 * share the dtype, nt, the interpolation order, the stream, the transport
 * tile shape (mireg_autotune changes it) and the LDS switch; it does not own
 * them (destroy the batch first).  Each problem keeps its context and
 * follows its single-problem algorithm step for step -- results equal those
 * of mireg_pcg_solve / mireg_gn_solve on each context alone up to rounding
 * (the multi-problem kernels are separate compilations whose operation
 * contraction may differ; FP64 iterates measured identical) -- but every
 * transport step of the Hessian matvec (incremental state and adjoint
 * sweeps) runs as one launch across all problems still iterating, each
 * Krylov pass as one launch per grid size, and the PCG iteration reads its
 * scalars back once for all of them.  Only the spectral preconditioner.  Returns MIREG_E_ARG for mismatched contexts,
 * MIREG_E_NOMEM if its step tables cannot be allocated. */
typedef struct mireg_batch mireg_batch;
int mireg_batch_create(mireg_ctx *const *ctxs, int n, mireg_batch **out);
int mireg_batch_destroy(mireg_batch *b);
const char *mireg_batch_last_error(const mireg_batch *b);
/* Lockstep PCG: for every problem i, H_i x_i = rhs_i at its current v, as
 * mireg_pcg_solve does it (rtol[i], the common maxit); rhs, x: n device
 * pointers; rtol: n host doubles; iters, relres, status: n host values each
 * (may be NULL).  Synchronises the stream. */
int mireg_batch_pcg_solve(mireg_batch *b, const void *const *rhs, void *const *x, const double *rtol, int maxit,
                          int *iters, double *relres, int *status);
/* Lockstep GN-Krylov: mireg_gn_solve for every problem (v_inout: n device
 * pointers, warm starts or zeros, overwritten by the final velocities; reps:
 * n reports, may be NULL; seconds is the batch's wall time).  The Newton
 * steps of the problems that have not stopped form one batched PCG; the
 * objectives, gradients and line searches run problem by problem. */
int mireg_batch_gn_solve(mireg_batch *b, void *const *v_inout, const mireg_solve_opts *opts, mireg_report *reps);

/* Individual operators for tests and input preparation.  `in` and `out`
 * are device fields of the context dtype; `arg` is an op parameter. */
enum {
    MIREG_OP_GRAD = 1,           /* scalar -> vector, spectral gradient */
    MIREG_OP_DIV = 2,            /* vector -> scalar, spectral divergence */
    MIREG_OP_LAPLACE = 3,        /* scalar -> scalar, Lap */
    MIREG_OP_APPLY_A = 4,        /* vector -> vector, A (H1 or H2 of the context) */
    MIREG_OP_APPLY_K = 5,        /* vector -> vector, K of the context */
    MIREG_OP_LERAY = 6,          /* vector -> vector, Leray projection */
    MIREG_OP_PRECOND = 7,        /* vector -> vector, (beta_v A)^{-1}, zero mode -> 1 */
    MIREG_OP_GAUSS = 8,          /* scalar -> scalar, Gaussian, arg = sigma in cells */
    MIREG_OP_DEPARTURE_X = 9,    /* vector v -> vector displacement (cells) of X */
    MIREG_OP_DEPARTURE_Y = 10,   /* vector v -> vector displacement (cells) of Y */
    MIREG_OP_TRANSPORT_STATE = 11,/* scalar mT -> scalar m(1) at the current v */
    MIREG_OP_INTERP = 12,        /* scalar f -> scalar I[f](x + d): `in` holds f
                                    followed by the displacement field d */
    MIREG_OP_RESCALE01 = 13,     /* scalar -> scalar, (u - min u)/(max u - min u) */
    MIREG_OP_SCALE_MAXNORM = 14, /* vector -> vector scaled so max_x |v(x)|_2 = arg */
    MIREG_OP_TRANSPORT_ADJOINT = 15 /* scalar lam(1) -> scalar lam(0) at the current v: the
                                    adjoint equation (eq. "adj", Sec. 2.2) solved backward over
                                    nt semi-Lagrangian steps along Y with its source lam div v
                                    (explicit Heun); F32_H16 holds the steps in FP16 as the
                                    gradient does.  `in` and `out` may alias. */
};
int mireg_op(mireg_ctx *ctx, int opcode, const void *in, void *out, double arg);

/* Allocation-free interpolation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): out = I[f](x + disp), the result of mireg_op(ctx,
 * MIREG_OP_INTERP, ...) bit for bit, without a context.  n: grid as in
 * mireg_params (at most 512 per axis); order 3 (tricubic) or 1 (trilinear);
 * dtype MIREG_F32 or MIREG_F64 (element type of f, disp and out); f a scalar
 * field, disp a displacement field [3][n1][n2][n3] in cell units, out a
 * scalar field, all device pointers owned by the caller; stream a
 * hipStream_t or NULL.  The call enqueues its kernels on `stream` and
 * returns without synchronising; it calls no allocator.  Its scratch (every
 * tile's stencil box and the box-measurement slots, 4 MiB) is one static
 * device array per GPU, held until the process ends and shared by every
 * call on that GPU, each call overwriting what the last one left: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Errors: MIREG_E_ARG (null pointer, order,
 * dtype), MIREG_E_SHAPE (unsupported axis, or a grid beyond the scratch),
 * MIREG_E_HIP; mireg_last_error(NULL) gives the message of the last failed
 * call in the calling thread. */
int mireg_interp_noalloc(const int n[3], int order, int dtype, const void *f, const void *disp, void *out,
                         void *stream);

/* Per-phase GPU time accumulated since the last reset (milliseconds), for
 * the FFT / interpolation split the paper reports. */
typedef struct {
    double fft_ms, interp_ms, other_ms;
    long launches;
} mireg_timers;
int mireg_timers_enable(mireg_ctx *ctx, int on);
int mireg_timers_read(mireg_ctx *ctx, mireg_timers *t, int reset);

/* Per-kernel statistics: when enabled, every kernel launch of the context is
 * bracketed by HIP events on the context stream; reading synchronises the
 * stream and returns, per kernel kind, the number of launches, the summed
 * event time and the algorithmic bytes of one launch (compulsory reads and
 * writes of its distinct operands, stencil re-reads not counted).  The
 * events add a little launch overhead; timing runs use them on their own. */
typedef struct {
    char name[32];
    long launches;
    double total_ms;
    double bytes_per_launch;  /* average over the launches */
} mireg_kernel_stat;
int mireg_kernel_stats_enable(mireg_ctx *ctx, int on);
/* Writes up to `max` entries (kernel kinds with at least one launch) and
 * sets *count; reset != 0 clears the accumulators. */
int mireg_kernel_stats_read(mireg_ctx *ctx, mireg_kernel_stat *out, int max, int *count, int reset);

#ifdef __cplusplus
}
#endif

#endif /* MIREG_H */
