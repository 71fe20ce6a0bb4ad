/*
 * meb.h -- C ABI of libmeb.so: the minimum enclosing ball (MEB) of m balls in
 * R^d on one AMD Instinct MI355X (gfx950), solved by the relative-type inexact
 * proximal augmented Lagrangian method (ripALM) with a semismooth-Newton inner
 * solver and mixed-precision screening (Liang & Yang, "Mixed-Precision GPU
 * Acceleration for Large-Scale Minimum Enclosing Ball Problems").
 *
 * Problem (Section 1, (MEB)): minimize r over (r, c) subject to
 *   ||c - c_i|| + r_i <= r for every ball i,
 * equivalently (Section 2) (r - r_i, c - c_i) in the second-order cone
 *   Q_{d+1} = {(t, s) : ||s|| <= t}.
 * The conic multipliers (u_i, v_i) in Q_{d+1} are the dual variables of
 * Section 2 (dual feasibility: sum u_i = 1, sum v_i = 0).
 *
 * General conventions for every entry point
 *   - Array arguments named C, R, U, V, keep_idx, viol_idx, slack, U_out,
 *     V_out, ws are DEVICE pointers (memory of the current HIP device);
 *     every other pointer is HOST memory.  All device arrays are row-major
 *     and owned by the caller; the library allocates no device memory.
 *   - C is m x d (row i = center c_i), R has m entries (radius r_i >= 0);
 *     R == NULL means a point set (every r_i = 0).  U has m entries, V is
 *     m x d.  x = (r, c) vectors have d + 1 entries with r first.
 *   - dtype is MEB_F64 (double) or MEB_F32 (float) and applies to C, R, U, V.
 *     C and V must be 16-byte aligned (rows are read with 16-byte loads and
 *     16-byte LDS copies; every torch or hipMalloc allocation is); the other
 *     device pointers must be aligned to their element size.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is ordered on it; calls that return host results synchronize it.
 *   - Scratch memory: each call takes a device workspace `ws` of `ws_bytes`
 *     bytes (256-byte aligned); query the size with meb_workspace_size()
 *     or meb_eval_workspace_size().  A workspace may not be shared by calls
 *     that run concurrently.
 *   - Return value: MEB_OK (0), a positive warning, or a negative error;
 *     meb_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses the ABI.  On an error, outputs are undefined.
 *   - Every call is deterministic: the same inputs give bitwise the same
 *     outputs (reductions run in a fixed order; no floating-point atomics).
 */
#ifndef MEB_H
#define MEB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MEB_OK 0
#define MEB_WARN_MAXITER 1    /* tolerance not reached; the ball returned is still feasible */
#define MEB_ERR_ARG (-1)      /* bad argument: sizes, dtype, NULL, alignment, bad option   */
#define MEB_ERR_HIP (-2)      /* HIP runtime or launch failure                            */
#define MEB_ERR_WORKSPACE (-3) /* ws NULL or smaller than the size the query returned    */
#define MEB_ERR_NUMERIC (-4)  /* non-finite value or Newton system not positive definite  */
#define MEB_ERR_UNSUPPORTED (-5) /* a shape this build does not handle (d too large)      */

/* element types */
#define MEB_F64 0
#define MEB_F32 1

/* solve modes */
#define MEB_MODE_FP64 0  /* plain ripALM in FP64 on all m balls                       */
#define MEB_MODE_MIXED 1 /* FP32 screening run, FP64 refinement, full FP64 check      */

/* meb_al_eval output selection */
#define MEB_WANT_PSI 1u
#define MEB_WANT_GRAD 2u
#define MEB_WANT_HESS 4u
#define MEB_WANT_MULT 8u
#define MEB_WANT_DMULT 16u
#define MEB_WANT_KKT 32u

/* Hessian contraction (the rank-one part of the generalized Hessian,
 * sum over the balls in the third projection case of coef_i s_i s_i^T) */
#define MEB_HESS_AUTO 0       /* FP64 run: MFMA_F64 for d >= 128, else F64; FP32 run: MFMA_BF16 for
                                 d >= 256, else F64                                              */
#define MEB_HESS_F64 1        /* FP64 vector FMA accumulation of run-precision rows              */
#define MEB_HESS_MFMA_F64 2   /* FP64 matrix cores (FP64 run only; the FP32 run uses F64)        */
#define MEB_HESS_MFMA_F32 3   /* FP32 inputs, FP32 accumulation on matrix cores (FP32 run only;
                                 the FP64 run uses AUTO's choice)                                */
#define MEB_HESS_MFMA_BF16 4  /* BF16 inputs, FP32 accumulation on matrix cores (FP32 run only)  */

/* Newton-direction solvers (meb_options.newton) */
#define MEB_NEWTON_DENSE 0
#define MEB_NEWTON_CG 1

/* largest supported dimension */
#define MEB_MAX_D 2048 /* odd d: at most 1024 */

/* Solver options.  Penalty and proximal parameters are in units normalized
 * by the instance scale L = max_i (||c_i - c_1|| + r_i) (the radius of a
 * feasible ball centred at c_1, so r* <= L <= 2 r*): the raw values used
 * are sigma/L and tau/L^2, and KKT_max is measured with lengths divided by
 * L.  Fill with meb_default_options() and then change fields. */
typedef struct meb_options {
    double rho;            /* weight of the relative stopping test, in [0, 1) (Algorithm 1); default 0.9 */
    double sigma0;         /* first penalty sigma_0; default 1                                      */
    double sigma_growth;   /* sigma_{k+1} = min(growth * sigma_k, sigma_max); default 5              */
    double sigma_max;      /* default 1e5                                                            */
    double tau;            /* proximal weight tau_k (constant); default 1                            */
    double tol_kkt;        /* final KKT_max tolerance (Section 5 uses 1e-8); default 1e-9, so that the
                              relative radius error stays below 1e-8 on every tested instance  */
    double tol_kkt_low;    /* KKT_max tolerance of the FP32 screening run (Section 5); default 1e-2  */
    double tol_red;        /* screening margin, in units of L (Section 4.2); default 0.03.  A
                              negative value keeps only balls the FP32 ball violates, which
                              forces reinsertion rounds (used to test that path)               */
    double eps_feas_rel;   /* violation threshold eps_feas = eps_feas_rel * (1 + r); default 1e-10   */
    int32_t max_outer;     /* outer iterations per ripALM run; default 200                           */
    int32_t max_inner;     /* semismooth-Newton iterations per outer iteration; default 50           */
    int32_t max_ls;        /* Armijo halvings per Newton step; default 40                            */
    int32_t max_reinsert;  /* reinsertion rounds of the mixed path; default 20                       */
    int32_t mode;          /* MEB_MODE_FP64 or MEB_MODE_MIXED; default MEB_MODE_MIXED                */
    int32_t stall_outer;   /* stop a run after this many outer steps without halving KKT_max; 3     */
    int32_t verbose;       /* 0 = silent; 1 = one line per outer iteration on stderr; 2 = also one
                              line per evaluation pass and Newton step (device printf)          */
    int32_t profile;       /* 1 = time every evaluation pass with HIP events (fills the pass_*
                              fields of meb_stats); default 0                                   */
    int32_t hess;          /* MEB_HESS_*: arithmetic of the Hessian contraction; default AUTO    */
    int32_t first_order_outer; /* the inner solves of the first this-many outer iterations (of the
                              FP64 run, or of the mixed mode's screening run) use the
                              accelerated gradient method (Section 4.1:
                              first-order inner solvers for the early outer iterations, with
                              backtracking and adaptive restart) instead of semismooth
                              Newton; default 0 (Newton throughout)                            */
    int32_t newton;        /* MEB_NEWTON_DENSE: H assembled and factorized (default);
                              MEB_NEWTON_CG: matrix-free, preconditioned conjugate gradients with
                              Hessian-vector products (Section 4.1, for large d); meb_solve only */
    int32_t cg_max_iter;   /* CG iterations per Newton direction (MEB_NEWTON_CG); default 20      */
    double cg_tol;         /* relative residual at which CG stops; default 1e-2                  */
} meb_options;

/* Statistics of one meb_solve.  Index 0 = FP32 screening run (mixed mode),
 * index 1 = FP64 run (the only one in FP64 mode; summed over reinsertion
 * rounds). */
typedef struct meb_stats {
    int32_t outer[2];      /* outer iterations                                  */
    int32_t inner[2];      /* Newton steps                                      */
    int32_t passes[2];     /* data passes of the evaluation kernel              */
    double kkt[2];         /* final normalized KKT_max of each run              */
    double L;              /* instance scale                                    */
    double rbar;           /* radius of the last FP64 iterate                   */
    double delta_max;      /* max_i (r_i + ||c - c_i||) - rbar over all m       */
    int64_t n_red;         /* size of the retained set of the last FP64 run     */
    int32_t reinsert_rounds;
    int32_t status;        /* same as the return value                          */
    double ms_total;       /* wall time of the call, ms                         */
    double ms_phase[4];    /* ms: prepare+FP32 run, screen+gather, FP64 run(s), checks */
    /* with opts->profile: summed device time and algorithmic bytes (input rows,
     * radii, multipliers read; multipliers written) of the evaluation-pass
     * launches of each run, and the number of launches */
    double pass_ms[2];
    double pass_bytes[2];
    int32_t pass_launches[2];
    int32_t reserved;
    /* rows of the rank-one Hessian contraction (balls in the third
     * projection case), summed over the passes of each run, and the largest
     * count of one pass */
    double mid_rows[2];
    double mid_rows_max[2];
    /* breakdown guard of the Newton solve (H is positive definite in exact
     * arithmetic, Section 4): systems solved with a raised diagonal, and
     * inner solves ended at their iterate because no raise succeeded */
    int32_t newton_shifted[2];
    int32_t inner_breaks[2];
    /* iterations of the first-order inner solver (first_order_outer) */
    int32_t first_order_steps[2];
    /* conjugate-gradient iterations (MEB_NEWTON_CG) */
    int32_t cg_iterations[2];
} meb_stats;

/* Fills *opts with the defaults listed above.  Returns MEB_OK. */
int meb_default_options(meb_options* opts);

/* Thread-local description of the last error ("" if none).  Valid until the
 * next call on the same thread. */
const char* meb_last_error(void);

/* SHA-256 (hex) over the library's sources, fixed when it was built; lets a
 * caller recognise a library built from other sources.  Static storage. */
const char* meb_source_hash(void);

/* Device workspace (bytes) that meb_solve needs for an instance of this
 * shape and options.  Returns MEB_ERR_ARG for m < 1, d < 1, d > MEB_MAX_D. */
int meb_workspace_size(int64_t m, int32_t d, int32_t dtype, const meb_options* opts, size_t* bytes);

/* Device workspace (bytes) that meb_al_eval, meb_screen, meb_check_feasible
 * and meb_prepare_f32 need for an instance of this shape. */
int meb_eval_workspace_size(int64_t m, int32_t d, int32_t dtype, size_t* bytes);

/* Minimum enclosing ball of the m balls (C, R).
 *
 * Runs ripALM (Algorithm 1) with the semismooth Newton method (Algorithm 2)
 * as inner solver.  In MEB_MODE_MIXED it follows the mixed-precision
 * reduction of Section 4.2: an FP32 run to tol_kkt_low on all balls,
 * screening {i : rhat - r_i - ||chat - c_i|| <= tol_red * L}, an FP64 run on
 * the retained balls warm-started from the FP32 point and multipliers, a
 * full FP64 check of every ball, and reinsertion of violated discarded balls
 * followed by a new FP64 run, until no discarded ball is violated.
 * C and R may be MEB_F64 or MEB_F32.  FP32 input is first widened exactly
 * into an FP64 copy inside the workspace (meb_workspace_size with dtype
 * MEB_F32 includes it), so the solve is the one of the widened data; the FP32
 * copy of the mixed mode is made internally either way.
 * Input errors: a negative radius, or a NaN or infinite coordinate or
 * radius, returns MEB_ERR_ARG (detected by the first pass over the data).
 *
 * Outputs: *r_out and c_out[d] (host) hold the ball.  r_out is made feasible
 * for every input ball: r_out = max(rbar, max_i (r_i + ||c - c_i||)) with
 * the maximum evaluated in FP64.  U_out (m) and V_out (m x d), device,
 * nullable, receive the final multipliers in FP64 (zero for discarded balls).
 * stats (host, nullable) receives meb_stats.
 * Returns MEB_OK, MEB_WARN_MAXITER (tolerance not reached within max_outer,
 * or a run stalled; the ball is still feasible), or an error. */
int meb_solve(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, const meb_options* opts,
              void* ws, size_t ws_bytes, double* r_out, double* c_out, double* U_out, double* V_out,
              meb_stats* stats, void* stream);

/* One evaluation of the proximal augmented Lagrangian subproblem (Section 3
 * subproblem Psi, Section 4 gradient and generalized Hessian, multiplier
 * update of Algorithm 1) for fixed multipliers (U, V), penalty sigma > 0,
 * proximal weight tau > 0 and proximal center xbar (host, d + 1).
 *
 * Let y = x + dir (dir host, d + 1, nullable = zero) and
 *   z_i = (r_i - y_r, c_i - y_c) + (u_i, v_i) / sigma.
 * Outputs (host unless noted; each only if its `want` bit is set):
 *   psi        Psi(y) = y_r + sigma/2 sum ||Pi(z_i)||^2 - 1/(2 sigma) sum ||(u_i, v_i)||^2
 *                       + tau/(2 sigma) ||y - xbar||^2                       (PSI)
 *   psi_trial  Psi(x + eta_l dir) for l < n_eta (etas host), the single-pass
 *              Armijo trials; requires PSI; nullable when n_eta = 0        (PSI)
 *   g          grad Psi(y) = (1, 0) - sigma sum Pi(z_i) + tau/sigma (y - xbar)  (GRAD)
 *   H          (d+1)^2 row-major, full symmetric: tau/sigma I + sigma sum P_i,
 *              P_i the element of the Clarke Jacobian of Pi at z_i taken as
 *              identity if ||s|| <= t, zero if ||s|| <= -t                  (HESS)
 *   U_new, V_new  device, dtype: sigma Pi(z_i) (multiplier update)          (MULT)
 *   dmult      sum_i ||sigma Pi(z_i) - (u_i, v_i)||^2                       (DMULT)
 *   kkt[5]     the five KKT_max terms (Section 5) at (y, sigma Pi(z_i)),
 *              unnormalized: |1 - sum u|, ||sum v||, max primal cone distance,
 *              max dual cone distance, max |complementarity|            (KKT)
 * U and V may be NULL (zero multipliers).  V rows are read only where
 * u_i != 0 (a multiplier in Q with u_i = 0 has v_i = 0).
 * Bits 8..10 of `want` select the arithmetic of the rank-one part of H
 * (MEB_HESS_* << 8, as for a run of precision dtype; 0 = AUTO).
 * Arithmetic runs in dtype; sums are accumulated in FP64 in a fixed order. */
int meb_al_eval(const void* C, const void* R, const void* U, const void* V, int64_t m, int32_t d, int32_t dtype,
                const double* x, const double* xbar, double sigma, double tau, const double* dir,
                int32_t n_eta, const double* etas, uint32_t want, double* psi, double* psi_trial, double* g,
                double* H, void* U_new, void* V_new, double* dmult, double* kkt, void* ws, size_t ws_bytes,
                void* stream);

/* Matrix-free product of the generalized Hessian of the subproblem with a
 * vector (Section 4.1: H q = tau/sigma q + sigma sum_i P_i q, the products
 * P_i q taken ball by ball and summed), at x with multipliers (U, V),
 * penalty sigma > 0 and proximal weight tau > 0; H is never formed.  This is
 * the product the MEB_NEWTON_CG solver iterates with.  x, q (host, d + 1),
 * Hq (host, d + 1) receives the product.  U, V as for meb_al_eval.  Sums are
 * taken in a fixed order (reproducible); the per-ball rows are formed in
 * dtype.  ws from meb_eval_workspace_size. */
int meb_hess_vec(const void* C, const void* R, const void* U, const void* V, int64_t m, int32_t d, int32_t dtype,
                 const double* x, double sigma, double tau, const double* q, double* Hq, void* ws, size_t ws_bytes,
                 void* stream);

/* Screening of Section 4.2: slack_i = r_hat - r_i - ||c_hat - c_i||,
 * evaluated in FP64 (FP32 inputs are widened exactly), and
 * keep_idx[0 .. *n_keep) = {i : slack_i <= tol_red} in ascending order.
 * keep_idx (device, capacity m), slack (device FP64 m, nullable).
 * tol_red is absolute (same units as r). */
int meb_screen(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r_hat,
               const double* c_hat, double tol_red, int64_t* keep_idx, int64_t* n_keep, double* slack, void* ws,
               size_t ws_bytes, void* stream);

/* A-posteriori feasibility check of Section 4.2 in FP64:
 *   *delta_max = max_i (r_i + ||c - c_i|| - r),  *argmax = smallest index
 *   attaining it, and the violated set {i : r_i + ||c - c_i|| - r > eps}
 *   in ascending order: its size in *n_viol, its first min(n_viol, viol_cap)
 *   indices in viol_idx (device, nullable when viol_cap = 0). */
int meb_check_feasible(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r,
                       const double* c, double eps, double* delta_max, int64_t* argmax, int64_t* viol_idx,
                       int64_t viol_cap, int64_t* n_viol, void* ws, size_t ws_bytes, void* stream);

/* meb_check_feasible without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that forbid
 * allocation).  Same arguments, results and error behaviour as
 * meb_check_feasible, minus ws / ws_bytes.  Its scratch (about 540 KB: the
 * center c, per-wave maxima and counts, their prefix) is a fixed array inside
 * the library, one copy per device, held until the process ends; the call
 * allocates nothing.  It returns MEB_ERR_UNSUPPORTED on a device whose scan
 * needs more than 16384 wave slots (more than 512 compute units).  When some
 * ball is violated and viol_cap > 0 the data are read twice (a counting pass,
 * then a pass that writes each index to its final place).  All calls on one
 * device share the scratch: calls that overlap in time on one device (from
 * several host threads or streams) race and give undefined results.
 * Returns after synchronizing the stream. */
int meb_check_feasible_noalloc(const void* C, const void* R, int64_t m, int32_t d, int32_t dtype, double r,
                               const double* c, double eps, double* delta_max, int64_t* argmax, int64_t* viol_idx,
                               int64_t viol_cap, int64_t* n_viol, void* stream);

/* Precision preparation for the screening run: C32[i] = float(C[i] - origin)
 * (row-wise, origin host d, nullable = 0), R32[i] = float(R[i]) (R32 unused
 * if R is NULL), rounded to nearest.  *L_out (host, nullable) receives
 * max_i (||c_i - origin|| + r_i) computed in FP64 from the FP64 input, or
 * +inf if some r_i is negative or some value is not finite. */
int meb_prepare_f32(const double* C, const double* R, int64_t m, int32_t d, const double* origin, float* C32,
                    float* R32, double* L_out, void* ws, size_t ws_bytes, void* stream);

/* Newton system of Algorithm 2 in FP64: solves H y = b for a symmetric
 * positive definite H (n x n row-major, device) by Cholesky factorization on
 * the device.  b, y device, n entries.  ws from meb_chol_workspace_size.
 * Returns MEB_ERR_NUMERIC if a pivot is not positive. */
int meb_chol_workspace_size(int32_t n, size_t* bytes);
int meb_chol_solve(int32_t n, const double* H, const double* b, double* y, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Multi-instance server (continuous batching).  Not part of the paper; it
 * serves a stream of independent MEB requests on one GPU.
 *
 * Requests are admitted first-in first-out whenever a slot is free and the
 * request's workspace (meb_workspace_size with the server's options) fits in
 * the caller's device pool; the head of the queue waits for room, so no
 * request starves.  An engine thread (one HIP stream, created on the device
 * current at meb_server_create) runs each admitted request as the same
 * phase sequence as meb_solve and steps all requests that are inside a
 * ripALM run together: one launch per kernel covers every such request, each
 * with the blocks, arithmetic and reduction order it has alone, so a result
 * is bitwise the same as meb_solve's on the same input and options, whatever
 * else is in flight.
 * ------------------------------------------------------------------------ */
typedef struct meb_server meb_server;

typedef struct meb_server_result {
    int64_t ticket;       /* from meb_server_submit                            */
    int64_t tag;          /* the caller's tag                                  */
    int64_t m;
    int32_t d;
    int32_t status;       /* meb_solve's return value for this request         */
    double r;             /* radius (feasible by construction)                 */
    double t_submit_ms;   /* server clock (ms, steady clock) at submission     */
    double t_admit_ms;    /* ... at admission                                  */
    double t_done_ms;     /* ... at completion                                 */
    meb_stats stats;      /* as meb_solve's; ms_total = t_done - t_admit       */
    char message[128];    /* error text when status < 0                        */
} meb_server_result;

typedef struct meb_server_stats {
    int64_t submitted, completed, failed;
    int32_t queued, active;
    uint64_t pool_used, pool_peak, pool_capacity; /* bytes of the job region  */
    int64_t ticks;                                 /* batched solver steps     */
    double mean_tick_items;                        /* requests per tick        */
    char message[128];                             /* fatal engine error       */
} meb_server_stats;

/* Creates a server over `pool` (device, 256-byte aligned, caller-owned, kept
 * until meb_server_destroy returns).  A table of max_active entries sits at
 * the start of the pool; the rest holds the requests' workspaces.  max_active
 * in [1, 1024] bounds the requests in flight; max_d bounds d of a request.
 * opts (nullable = defaults) apply to every request; profile must be 0. */
int meb_server_create(void* pool, size_t pool_bytes, const meb_options* opts, int32_t max_active, int32_t max_d,
                      meb_server** out);

/* Queues one request; returns at once.  C (m x d) and R (m, nullable =
 * points) are FP64 device arrays whose contents must be complete when the
 * call is made (synchronize the stream that wrote them) and must stay
 * unchanged until the request's result has been polled.  c_out (host, d
 * doubles, nullable) receives the center at completion.  Returns
 * MEB_ERR_WORKSPACE if the request can never fit in the pool. */
int meb_server_submit(meb_server* srv, const void* C, const void* R, int64_t m, int32_t d, int32_t dtype,
                      int64_t tag, double* c_out, int64_t* ticket);

/* Moves up to `cap` completed results into out[0 .. *n_out), in completion
 * order, waiting up to wait_ms for the first one when none is ready. */
int meb_server_poll(meb_server* srv, meb_server_result* out, int32_t cap, int32_t wait_ms, int32_t* n_out);

int meb_server_info(meb_server* srv, meb_server_stats* info);

/* Finishes every submitted request, then stops the engine and frees the
 * server (not the pool).  Results not yet polled are dropped. */
int meb_server_destroy(meb_server* srv);

/* The server's admission policy on a simulated clock: request i arrives at
 * arrival[i] (non-decreasing), needs bytes[i] of a pool of pool_bytes and
 * holds it for service[i] after admission.  Outputs t_admit, t_done and the
 * pool offset of each request.  For testing the policy without a GPU. */
int meb_sched_simulate(int32_t n, const double* arrival, const double* service, const uint64_t* bytes,
                       uint64_t pool_bytes, int32_t max_active, double* t_admit, double* t_done, uint64_t* offset);

#ifdef __cplusplus
}
#endif

#endif /* MEB_H */
