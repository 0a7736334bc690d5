/*
 * rd.h -- C ABI of librdpdhg: one implicit reaction-diffusion time step solved by
 * the G-prox linearized PDHG iteration on an AMD Instinct MI355X (gfx950).
 *
 * Method: Liu, Liu, Osher, Li, "A first-order computational algorithm for
 * reaction-diffusion type equations via primal-dual hybrid gradient method"
 * (arXiv 2305.03945).  Given U^k, the step size h_t, the operator, the reaction
 * and the boundary condition, a step returns U^{k+1}, the root of F(U) = 0 for
 * the backward-Euler scheme (Sec. 2.1, eqs. 11-12; Sec. 3.2, eq. 29; Sec. 3.4.1),
 * computed by Algorithm 1:
 *
 *     P_{n+1} = P_n + tau_p G^-1 F(U_n)
 *     P~      = P_{n+1} + omega (P_{n+1} - P_n)
 *     U_{n+1} = U_n - tau_u grad F(U_n)^T P~
 *
 * from U_0 = U^k, P_0 = 0, stopped when ||Res(U_n)||_2 <= tol with Res = F / h_t
 * (Sec. 2.1, "Stopping criterion"; for two components the component norms are
 * added, Sec. 3.4.1).  G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2 (gamma only for
 * the sixth-order equation of Sec. 3.3) is inverted by a 2-D FFT (periodic grids) or a
 * 2-D DCT-II (Neumann grids, Remark 1); on 3-D grids by the 3-D transforms.
 *
 * Conventions for every entry point:
 *   - Array arguments documented as DEVICE are device (HBM) pointers; HOST ones are
 *     host pointers.  Fields are FP64, layout [ncomp][N][N] ([ncomp][N][N][N] on a 3-D
 *     grid), row-major, x fastest.
 *   - The caller owns every array it passes; the library owns its workspaces.
 *   - Functions return rd_status; nothing throws across the ABI.
 *   - A context is not thread-safe: one host thread per context.
 *   - Work is enqueued on the HIP stream passed in (NULL = the default stream);
 *     functions that return results in host memory synchronise that stream.
 */
#ifndef RD_PDHG_H
#define RD_PDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RD_OK = 0,
    RD_E_INVALID = -1,    /* bad argument: shape, N not a power of two in [16, 4096], h_t <= 0,
                             unsupported operator / reaction pair, NULL pointer             */
    RD_E_NOCONV = -2,     /* max_iter (or max_outer) reached; the last iterate is returned   */
    RD_E_NONFINITE = -3,  /* residual NaN/Inf or grown beyond 1e8 x its initial value: the
                             divergence the paper reports for h_t above a threshold (Sec. 2.2) */
    RD_E_NOMEM = -4,      /* device allocation failed, or serving budget exceeded           */
    RD_E_DEVICE = -5,     /* a HIP runtime call failed                                      */
    RD_E_BUSY = -6        /* serving: the ticket is not finished yet                        */
} rd_status;

typedef enum { RD_BC_PERIODIC = 0, RD_BC_NEUMANN = 1 } rd_bc;

/* Linear operator of F.  RD_OP_LAP5: +lambda Lap with the 5-point Laplacian (Sec. 2.1;
 * periodic block-circulant form, or the Neumann L_1/L_2 form of Remark 1, eq. 24); on
 * a 3-D grid the 7-point Laplacian.
 * RD_OP_BIHARM13: -lambda Lap Lap with the 13-point stencil (= 5-point squared; Sec. 3.2).
 * RD_OP_FCH6: the sixth-order functionalized Cahn-Hilliard operator of Sec. 3.3 (nested
 * 5-point Laplacians, 25-point reach), with RD_RX_FCH only.                             */
typedef enum { RD_OP_LAP5 = 0, RD_OP_BIHARM13 = 1, RD_OP_FCH6 = 2 } rd_operator;

/* Reaction term.  Parameters in rd_problem.p[]:
 *   RD_RX_NONE          linear step (heat with LAP5, biharmonic with BIHARM13)
 *   RD_RX_ALLEN_CAHN    p[0] = b:  f(u) = b (u - u^3)           (Sec. 3.1, eq. 25), LAP5 only
 *   RD_RX_CAHN_HILLIARD p[0] = b:  + Lap (b (u^3 - u))          (Sec. 3.2, eq. 28), BIHARM13 only
 *   RD_RX_SCHNAKENBERG  p[0] = a, p[1] = b, p[2] = kappa; two components (u, v) with
 *                       diffusion diff[0], diff[1]                (Sec. 3.4.1), LAP5 only
 *   RD_RX_FCH           u_t = Lap (eps^2 Lap - W''(u) + eps^2)(eps^2 Lap u - W'(u)),
 *                       W = (u^2 - 1)^2 / 4, diff[0] = eps^2      (Sec. 3.3), FCH6 only     */
typedef enum {
    RD_RX_NONE = 0,
    RD_RX_ALLEN_CAHN = 1,
    RD_RX_CAHN_HILLIARD = 2,
    RD_RX_SCHNAKENBERG = 3,
    RD_RX_FCH = 4
} rd_reaction_kind;

typedef struct {
    int32_t nx, ny;          /* grid points per side; must be equal, power of two, 16..4096 */
    double lx, ly;           /* side lengths; must be equal; spacing h = lx / nx            */
    int32_t bc;              /* rd_bc                                                       */
    int32_t op;              /* rd_operator                                                 */
    int32_t rx;              /* rd_reaction_kind                                            */
    int32_t nz;              /* 0 or 1: 2-D grid.  nz = nx: 3-D cube of nx^3 points, layout
                                [c][z][y][x], 7-point Laplacian (RD_OP_LAP5 equations only),
                                16 <= nx <= 256; rd_step, rd_advance, rd_precond_solve,
                                rd_profile_iteration and serving take it; rd_residual and
                                rd_prox return RD_E_INVALID (the method is posed in R^d,
                                Sec. 2)                                                     */
    double diff[2];          /* lambda (diff[0]) or (D1, D2) for two components            */
    double p[4];             /* reaction parameters, see rd_reaction_kind                   */
} rd_problem;

/* RD_FP32_MIXED: FP64 outer residual correction around an FP32 inner PDHG loop on the
 * correction (the paper is silent on precision).  Its range: the FP32 evaluation of the
 * inner residual must resolve the correction, i.e. 2^-24 times the linear stencil's weight
 * relative to the identity (8 lambda h_t / h^2 for second-order operators, 64 lambda h_t / h^4
 * for RD_OP_BIHARM13, 512 eps^4 h_t / h^6 for RD_OP_FCH6) well below 1; beyond it (e.g.
 * Cahn-Hilliard at lambda = 4e-4, h_t = 1e-4 on 2048^2, FCH at the Sec. 3.3 parameters on
 * 256^2) the inner loop diverges and the step returns RD_E_NONFINITE: use RD_FP64 there. */
typedef enum { RD_FP64 = 0, RD_FP32_MIXED = 1 } rd_precision;
typedef enum { RD_INIT_PREV = 0, RD_INIT_PROX = 1 } rd_init;

typedef struct {
    double tol;              /* stop when ||F(U)/h_t||_2 (summed over components) <= tol   */
    int32_t max_iter;        /* PDHG iterations per step (FP64), or inner iterations per outer
                                pass (mixed); 0: no iteration, the step returns U^k with
                                RD_E_NOCONV unless U^k already meets tol                     */
    int32_t max_outer;       /* mixed only: outer FP64 correction passes                     */
    double tau_u, tau_p;     /* PDHG step sizes                                              */
    double omega;            /* extrapolation coefficient (the paper uses 1, Sec. 3)         */
    int32_t precision;       /* rd_precision                                                 */
    int32_t init;            /* rd_init: U_0 = U^k (paper) or the pointwise reaction prox    */
    double inner_rtol;       /* mixed only: inner solve stops at ||F~(e)|| <= max(inner_rtol ||r||,
                                tol / 2)                                                     */
} rd_opts;

typedef struct {
    int32_t iters;           /* PDHG iterations (mixed: FP32 inner iterations, all passes)    */
    int32_t outer;           /* mixed: FP64 outer passes; FP64 path: 0                        */
    double residual_l2;      /* final ||F(U)/h_t||_2 (paper norm, FP64)                       */
    double residual0;        /* the same at U_0                                               */
    double mass_drift;       /* sum(U^{k+1} - U^k) in FP64, per step (component 0 + 1)        */
    int32_t status;          /* rd_status of the step                                         */
    int32_t pad0;
} rd_info;

/* ---- context ---------------------------------------------------------------------- */
/* Opaque handles: a context (one device, its workspaces, tables and serving state) and a
 * serving trajectory of that context.  Owned by the library; freed by rd_destroy and
 * rd_traj_close.                                                                          */
typedef struct rd_ctx rd_ctx;
typedef struct rd_traj rd_traj;

/* Create a context on HIP device `device`.  *out receives the handle.                    */
rd_status rd_create(int device, rd_ctx **out);
/* Free every workspace and table of the context.                                         */
rd_status rd_destroy(rd_ctx *ctx);

/* Default options: tol 1e-10, max_iter 10000, max_outer 20, tau_u = tau_p = 0.9,
 * omega = 1, FP64, U_0 = U^k, inner_rtol 3e-2.                                             */
void rd_default_opts(rd_opts *opts);

/* Device bytes one step's workspace needs (fields, spectra, partial sums).              */
size_t rd_footprint_bytes(const rd_problem *prob, const rd_opts *opts);

/* ---- one implicit step (Algorithm 1, the body of its time loop) --------------------- */
/* u_n (DEVICE, read) -> u_np1 (DEVICE, written); they may alias.  hip_stream is a
 * hipStream_t or NULL.  info (HOST) receives iteration count, residuals, mass drift and
 * status; the return value equals info->status, or an argument/device error code.
 * Synchronises the stream.                                                               */
rd_status rd_step(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t,
                  const double *u_n, double *u_np1, void *hip_stream, rd_info *info);

/* ---- one implicit step without allocation ------------------------------------------ */
/* For callers that cannot allocate device or pinned memory while they run (tight serving
 * loops, harnesses that forbid hipMalloc; the call waits on the host for each chunk's stop
 * decision, so a captured graph cannot record it): rd_step with
 * the same arguments, results and statuses (FP64 results bitwise equal to rd_step's; the
 * mixed path's within its rounding), whose workspace, tables, slot and State live in a
 * device scratch array of 64 MiB that the library holds on every device it runs on until
 * the process ends.  The call allocates nothing: no hipMalloc / hipFree / pinned host
 * memory; host staging is static.  Limits: N <= 1024 and a workspace that fits the 64 MiB
 * (one component up to 1024^2 in either precision, two components up to 512^2; 3-D grids
 * up to 64^3); larger problems return RD_E_NOMEM before any device work.  The scratch
 * array is shared by every call on a device and keeps the last call's contents (each call
 * rewrites what it reads first), so calls that overlap on one device -- from several
 * threads or contexts, or on several streams -- race and must not be made.
 * Synchronises the stream.                                                               */
rd_status rd_step_noalloc(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t,
                          const double *u_n, double *u_np1, void *hip_stream, rd_info *info);

/* ---- adaptive time step size (Sec. 2.2, "Adaptive time stepsize") ---------------------- */
/* Rule: after a step of size h that took M PDHG iterations (rd_info.iters; mixed: inner
 * iterations), the next step uses eta h if M > n_hi (N^*), h / eta if M < n_lo (N_*) and
 * h / eta <= ht0 (h_t^0), else h.  A step whose solve failed (RD_E_NOCONV or
 * RD_E_NONFINITE) is rejected and retried with eta h (the paper is silent on failed
 * steps; this is the reading taken).                                                     */
typedef struct {
    double ht0;              /* first and largest step size h_t^0 (> 0)                   */
    double eta;              /* rescaling coefficient, 0 < eta < 1                        */
    int32_t n_hi;            /* N^*: shrink above this many iterations                    */
    int32_t n_lo;            /* N_*: enlarge below this many (0 < n_lo < n_hi)            */
    double ht_min;           /* a rejected step whose retry would go below this ends the
                                run with RD_E_NOCONV (>= 0)                                 */
    int32_t max_rejects;     /* consecutive rejections allowed before RD_E_NOCONV (>= 0)  */
    int32_t pad0;
} rd_adapt;

typedef struct {
    int32_t accepted;        /* steps taken                                               */
    int32_t rejected;        /* failed solves retried with a smaller step                 */
    int32_t shrinks;         /* decisions that reduced the step size (rejections included) */
    int32_t enlarges;        /* decisions that increased it                               */
    int64_t pdhg_iters;      /* PDHG iterations of all solves, rejected ones included     */
    double t;                /* time reached                                              */
    double ht;               /* step size the next step would use                         */
    int32_t status;          /* RD_OK, or RD_E_NOCONV when the rejections ran out          */
    int32_t pad0;
} rd_adapt_info;

/* The rule alone, host logic only: step size h used, the step's iteration count and
 * status -> *ht_next (HOST) and *accept (HOST, 1 or 0).  RD_E_INVALID for a bad rd_adapt. */
rd_status rd_adapt_next(const rd_adapt *adapt, double h, int32_t iters, int32_t step_status,
                        double *ht_next, int32_t *accept);

/* Advance u (DEVICE, [c][N][N] FP64, read and overwritten) from t0 to t_end with rd_step
 * solves and the rule above, starting at h = min(ht0, t_end - t0); every step is shortened
 * to land on t_end (h = min(h_t, t_end - t)); the run ends when t_end - t <=
 * 1e-14 max(1, |t_end|).  Rejected steps leave u unchanged.  info (HOST) receives the
 * counters; if trace_cap > 0, trace_h / trace_iters / trace_ok (HOST, trace_cap entries
 * each) receive the size, iteration count and acceptance of the first trace_cap solves.
 * Allocates one field-sized device buffer for the call.  Returns info->status, or an
 * argument / device error.  Synchronises.                                                */
rd_status rd_advance(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, const rd_adapt *adapt,
                     double t0, double t_end, double *u, void *hip_stream, rd_adapt_info *info,
                     double *trace_h, int32_t *trace_iters, int32_t *trace_ok, int32_t trace_cap);

/* ---- kernel-level entry points (the pieces of one iteration) ------------------------ */
/* W = F(U) (Sec. 2.1 eq. 12; Sec. 3.2 eq. 29; Sec. 3.4.1).  u, uk, w: DEVICE, [c][N][N].
 * *res_l2 (HOST) receives ||W / h_t||_2 summed over components.  Synchronises.          */
rd_status rd_residual(rd_ctx *ctx, const rd_problem *prob, double h_t, const double *u,
                      const double *uk, double *w, void *hip_stream, double *res_l2);
/* Y = G^-1 W with G = (I - alpha Lap + beta Lap^2 - gamma Lap^3)^2 per component as the
 * equation implies (Sec. 2.1 "Choosing the matrix G"; Remark 1 for Neumann; Sec. 3.3 for
 * gamma).  w, y: DEVICE, [c][N][N] or [c][N][N][N].  precision RD_FP64 or RD_FP32_MIXED
 * (FP32 transforms).  Synchronises.                                                        */
rd_status rd_precond_solve(rd_ctx *ctx, const rd_problem *prob, double h_t, int32_t precision,
                           const double *w, double *y, void *hip_stream);
/* Pointwise reaction prox (the implicit reaction-only step, a predictor for U_0;
 * Sec. 2.1 "Initial guess"): Allen-Cahn cubic, Schnakenberg 2x2; identity otherwise.
 * c, u: DEVICE.  Synchronises.                                                            */
rd_status rd_prox(rd_ctx *ctx, const rd_problem *prob, double h_t, const double *c, double *u,
                  void *hip_stream);

/* ---- instrumentation ------------------------------------------------------------- */
/* Time the kernels of one Algorithm-1 iteration on hip_stream: prepares the step
 * for u_n (DEVICE) like rd_step (stop rules disabled), runs one untimed iteration, then
 * `reps` iterations in the solver's launch order, back to back, each launch recording
 * a start and a stop HIP event in its own dispatch packets (the kernel's begin and end
 * on that stream), so each kernel runs in the cache state the real loop leaves.  ms_out
 * (HOST, 4 doubles on a 2-D grid, 6 on a 3-D one) receives the mean duration per launch
 * in milliseconds of, 2-D: column pass (with the stop decision of the preceding row
 * pass), inverse row pass + dual update, primal update, residual + forward row pass;
 * 3-D: forward y-line pass (with the stop decision of the preceding row pass), z-line
 * pass (forward, symbol, inverse), inverse y-line pass, inverse x-row pass + dual
 * update, primal update, residual + forward x-row pass.  Synchronises.                 */
rd_status rd_profile_iteration(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts, double h_t,
                               const double *u_n, int32_t reps, void *hip_stream, double *ms_out);

/* ---- serving: continuous batching of steps of resident trajectories ----------------- */
/* A trajectory keeps U^k and, once admitted, its whole step workspace resident in device
 * memory.  Each pump round admits queued trajectories (arrival order, while the budget
 * allows), starts the next submitted step of every idle admitted trajectory, and
 * advances every running step by one round of iterations.  Running steps that share
 * (precision, N, dimension, boundary condition, equation family) form a batch group: one launch
 * per kernel covers all of them (one workgroup row per step), and different groups run
 * on separate streams so that they overlap on the device.  A step's arithmetic does not
 * depend on what else is in the batch: each result equals the one rd_step returns.
 * Serving calls synchronise their own streams and ignore hip_stream ordering of other
 * work except where noted.                                                               */

/* Set the device-memory budget for admitted trajectories (bytes; 0 = unlimited).  A
 * trajectory is admitted while resident + its workspace <= budget, and always when
 * nothing is resident (so a single request larger than the budget still runs).        */
rd_status rd_serve_set_budget(rd_ctx *ctx, size_t bytes);
/* Open a trajectory: copies u0 (DEVICE, FP64, [c][N][N] or [c][N][N][N]) into a resident copy, ordered
 * after prior work on hip_stream, and synchronises it.  *out (HOST) receives the handle.
 * Workspace memory is reserved only at admission, by rd_serve_pump.                    */
rd_status rd_traj_open(rd_ctx *ctx, const rd_problem *prob, const rd_opts *opts,
                       const double *u0, void *hip_stream, rd_traj **out);
/* Queue one implicit step of size h_t; *ticket (HOST) identifies it.  Steps of one
 * trajectory run in submission order, each starting from the trajectory's state: the
 * result of its last step that ended RD_OK.  A step that fails (RD_E_NOCONV,
 * RD_E_NONFINITE, reported by rd_poll) leaves that state unchanged, so that the caller
 * may submit the step again with a smaller h_t.                                          */
rd_status rd_traj_submit(rd_traj *traj, double h_t, uint64_t *ticket);
/* One serving round: admits queued trajectories, retires the rounds that have completed,
 * starts a round for every idle group with work; if no round had completed, waits for the
 * first in-flight one to complete (at most max_wait_us microseconds when > 0, no limit when
 * 0), retires it and restarts its group.  max_wait_us < 0: RD_E_INVALID.                   */
rd_status rd_serve_pump(rd_ctx *ctx, int32_t max_wait_us);
/* RD_E_BUSY until the ticket's step finished; then fills info (HOST) and returns the
 * step's status.  RD_E_INVALID for an unknown ticket.                                   */
rd_status rd_poll(rd_ctx *ctx, uint64_t ticket, rd_info *info);
/* Copy the trajectory's current state U^k to u_out (DEVICE): the result of its last step
 * that ended RD_OK by the end of any serving round in flight, which the copy waits for
 * (the initial state if none has).  Synchronises.                                       */
rd_status rd_traj_read(rd_traj *traj, double *u_out, void *hip_stream);
/* Close a trajectory: waits for the device, releases its workspace (returning its bytes
 * to the budget), its resident state and its tickets: rd_poll then returns RD_E_INVALID
 * for every ticket of it, finished or not (unfinished steps are dropped).                */
rd_status rd_traj_close(rd_traj *traj);

typedef struct {
    uint64_t budget_bytes;   /* as set by rd_serve_set_budget                              */
    uint64_t resident_bytes; /* workspace bytes of admitted trajectories                   */
    int32_t admitted;        /* trajectories holding a workspace                           */
    int32_t queued;          /* trajectories waiting for admission                         */
    int32_t running;         /* steps in progress                                          */
    int32_t pending_steps;   /* submitted steps not started yet                            */
} rd_serve_info;
/* Snapshot of the serving state (HOST out).  Host-only; no device work.                */
rd_status rd_serve_stats(rd_ctx *ctx, rd_serve_info *out);

const char *rd_status_str(rd_status s);

#ifdef __cplusplus
}
#endif
#endif /* RD_PDHG_H */
