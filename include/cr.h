/*
 * cr.h - C ABI of the MI355X (gfx950) convex-regression pair engine.
 *
 * The library solves the Tikhonov-regularized least-squares convex-regression
 * QP (Aybat & Wang, "A Parallel Method for Large Scale Convex Regression
 * Problems", Sec. II-C, eq. "regularize"):
 *
 *     min_{y in R^N, xi in R^{N x n}}  1/2 ||y - ybar||^2 + gamma/2 ||xi||^2
 *     s.t.  y_i >= y_j + xi_j^T (x_i - x_j)   for every ordered pair i != j
 *
 * with the ALCC augmented-Lagrangian method (Sec. II-E, Fig. 3) and MAPG, its
 * block-wise accelerated projected-gradient inner solver (Sec. II-E, Fig. 4).
 * The cost of every MAPG iteration is one pass over all N(N-1) constraint
 * pairs (the products with A1, A2, A1^T, A2^T that the paper names as the
 * bottleneck of each MAPG iteration), done on the GPU without ever forming
 * A1 or A2.
 *
 * Conventions for every entry point:
 *  - All pointers named *_dev are device pointers on the device that is
 *    current for the calling thread; arrays are dense and row-major:
 *    X is N x n (row l = x_l), ybar and y are N, xi is N x n (row l = xi_l),
 *    theta (inspection calls only) is N x N with theta[i*N + j] the
 *    multiplier of the pair (i, j).  X, ybar, y and xi are IEEE double in
 *    every precision mode; the precision mode only selects the arithmetic of
 *    the O(N^2) pair pass.
 *  - "stream" is a hipStream_t passed as void* (0 = the null stream).  Work is
 *    enqueued on that stream; the calls marked "host-synchronous" also wait
 *    for it.
 *  - Every call returns a cr_status.  Arguments are validated on the host
 *    before any HIP call, so argument errors are reported without touching a
 *    GPU.  No exception or abort crosses the ABI.
 *  - The library never allocates device memory for problem data: the caller
 *    provides one workspace of cr_workspace_bytes() bytes (256-byte aligned)
 *    and keeps it, X and ybar alive until cr_destroy().
 */
#ifndef CR_H
#define CR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cr_status;
enum {
    CR_OK = 0,
    CR_ERR_ARG = 1,          /* invalid argument (message in cr_last_error) */
    CR_ERR_NOMEM = 2,        /* workspace smaller than cr_workspace_bytes() */
    CR_ERR_HIP = 3,          /* a HIP runtime call failed */
    CR_ERR_NONFINITE = 4,    /* NaN/Inf in X or ybar, or in an iterate */
    CR_NOT_CONVERGED = 5,    /* max_outer reached before kkt_tol; outputs valid */
    CR_ERR_STATE = 6,        /* call not valid in the context's current state */
    CR_ERR_UNSUPPORTED = 7   /* e.g. n above CR_MAX_DIM */
};

/* Arithmetic of the pair pass. */
enum {
    CR_F64 = 0,        /* FP64 MFMA, theta stored in FP64 */
    CR_F32 = 1,        /* FP32 MFMA, theta stored in FP32 */
    CR_MIXED_BF16 = 2  /* BF16 MFMA on hi/lo splits, FP32 accumulation, theta FP32 */
};

/* Modes of cr_pairwise_step. */
enum {
    CR_GRAD = 0,          /* gradient of P_k at (y, xi) */
    CR_THETA_UPDATE = 1   /* ALCC multiplier step at (y, xi) plus KKT residuals */
};

#define CR_MAX_DIM 31     /* largest supported point dimension n */

/*
 * Parameters of ALCC (Fig. 3) and MAPG (Fig. 4).  The paper gives no values;
 * cr_params_default() fills this implementation's defaults.
 *   gamma       Tikhonov weight (> 0)                               [1e-3]
 *   mu1         first penalty parameter mu_1; <= 0 selects 1/(2N)   [0]
 *   c           mu_{k+1} = c mu_k, c > 1                            [4]
 *   kappa       decay exponent of tau_k and alpha_k, > 0            [0.1]
 *   tau1        first subproblem tolerance tau_1 (> 0)              [1]
 *   alpha_y1    MAPG stopping radius for y; <= 0 selects 1e-2 Bbar  [0]
 *   alpha_xi1   MAPG stopping radius for xi; <= 0 selects 1e-2 Bbar [0]
 *   step_scale  MAPG block step is step_scale / L (0 < s <= 1)      [0.5]
 *   kkt_tol     outer stop when the KKT measure is <= kkt_tol       [1e-4]
 *   max_outer   ALCC iteration cap                                  [30]
 *   inner_iters > 0: fixed schedule, exactly this many MAPG
 *               iterations per ALCC iteration and no early stops    [0]
 *   max_inner   cap on l_max_k in the adaptive schedule             [20000]
 *   precision   CR_F64, CR_F32 or CR_MIXED_BF16                     [CR_F64]
 *   tile_rows   rows of theta per pass workgroup (rounded up to 64);
 *               0 selects a heuristic; an autotuner picks it per
 *               (n, precision, N bucket) in the Python layer         [0]
 *   deterministic 1: single-problem runs use the batched form's kernels
 *               (pair pass, reduction, update) instead of completing each
 *               MAPG step inside the next pass, so that a problem solved
 *               alone gives the same bits as inside a cr_solve_batched
 *               batch with the same tile_rows.  Every run is bitwise
 *               reproducible either way (fixed-order sums, no atomics
 *               in any sum)                                          [0]
 *   *_override  > 0 replaces the computed L^y, L^xi, Bbar_y, Bbar_xi [0]
 */
typedef struct {
    double gamma, mu1, c, kappa, tau1, alpha_y1, alpha_xi1, step_scale, kkt_tol;
    int32_t max_outer, inner_iters, max_inner, precision;
    int32_t tile_rows, deterministic;
    double Ly_override, Lxi_override, By_override, Bxi_override;
} cr_params;

/*
 * Result summary.  kkt is max(stat_y, stat_xi, infeas, compl) / (1 + |ybar|_inf)
 * at the last ALCC iterate (y_k, xi_k) with multiplier lam = mu_k (theta_k - r)_+:
 *   stat_y  = |y - ybar - A1^T lam|_inf     stat_xi = |gamma xi - A2^T lam|_inf
 *   infeas  = max_ij (r_ij)_-               compl   = max_ij lam_ij |r_ij|
 * infeas_norm and gap_norm are the paper's normalized infeasibility
 * ||(r)_-||_2 / sqrt(N^2-N) and gap lam^T r / (N^2-N) (Sec. III).
 * pair_updates = N(N-1) * inner_iters; seconds is the wall time of the
 * iteration loop (after initialisation).
 */
typedef struct {
    int32_t outer_iters, status;
    int64_t inner_iters;
    double objective, kkt, stat_y, stat_xi, infeas, compl_, infeas_norm, gap_norm;
    double seconds, pair_updates;
    double sigma2_A1, sigma2_A2, Bbar_y, Bbar_xi;
} cr_info;

typedef struct cr_ctx cr_ctx;

/* Fill *p with the defaults listed above.  CR_ERR_ARG if p is NULL. */
cr_status cr_params_default(cr_params* p);

/* Static text for a status code (never NULL). */
const char* cr_status_string(cr_status s);

/* Last error message of a context, or of the last failed call that had no
 * context (ctx == NULL).  Never NULL; valid until the next call. */
const char* cr_last_error(const cr_ctx* ctx);

/*
 * Bytes of device workspace needed for N points of dimension n under params
 * (dominated by the N x N multiplier array theta of Fig. 3, stored once, in
 * FP64 for CR_F64 and FP32 otherwise).  Pure host arithmetic.
 * Errors: CR_ERR_ARG for N < 2, n < 1, bad params or bytes == NULL;
 * CR_ERR_UNSUPPORTED for n > CR_MAX_DIM or N > 2^20.
 */
cr_status cr_workspace_bytes(int64_t N, int32_t n, const cr_params* params, size_t* bytes);

/*
 * Create a solver context bound to (X, ybar) and to stream.  Borrows X_dev,
 * ybar_dev and the workspace (the caller keeps them alive and unmodified
 * until cr_destroy).  Computes on the device: the pass-precision copies of X,
 * sigma_max(A1)^2 = 2N, sigma_max(A2)^2 = max_j lambda_max(S_j) with
 * S_j = sum_i (x_i - x_j)(x_i - x_j)^T, the least-squares affine fit that
 * supplies the feasible point and the radii Bbar_y = Bbar,
 * Bbar_xi = Bbar / sqrt(gamma) of Sec. II-E, and the ALCC starting point
 * (y_0, xi_0) = that fit, theta_1 = 0.  Host-synchronous.
 * Errors: CR_ERR_ARG (null pointers, N < 2, n < 1, gamma <= 0, c <= 1,
 * kappa <= 0, tau1 <= 0, step_scale not in (0, 1], max_outer < 1,
 * unknown precision), CR_ERR_UNSUPPORTED (n > CR_MAX_DIM or N > 2^20), CR_ERR_NOMEM
 * (ws_bytes too small), CR_ERR_NONFINITE (NaN/Inf in X or ybar),
 * CR_ERR_HIP.  On error *out is NULL.
 */
cr_status cr_init(cr_ctx** out, int64_t N, int32_t n, const cr_params* params,
                  const void* X_dev, const void* ybar_dev, void* workspace_dev,
                  size_t ws_bytes, void* stream);

/* Release the host-side context (the workspace stays the caller's). */
cr_status cr_destroy(cr_ctx* ctx);

/*
 * One pass over all N(N-1) pairs at the point (y_dev, xi_dev) with the
 * context's current theta (Sec. II-E):
 *  CR_GRAD:   r = A1 y + A2 xi, w = (r - theta)_-, and
 *             gy_dev  = (y - ybar)/mu - A1^T w        (= grad_y P_k)
 *             gxi_dev = (gamma/mu) xi - A2^T w        (= grad_xi P_k)
 *             mu_next is ignored; theta is unchanged.
 *  CR_THETA_UPDATE: Fig. 3 step 4, theta <- (mu/mu_next) (r - theta)_-,
 *             with lam = mu (theta_old - r)_+ written as the stationarity
 *             residuals gy_dev = y - ybar - A1^T lam and
 *             gxi_dev = gamma xi - A2^T lam; the KKT scalars of the pass are
 *             returned by the next cr_get_info().
 * Asynchronous on the context stream.  gy_dev (N) and gxi_dev (N x n) are
 * FP64 outputs owned by the caller.
 * Errors: CR_ERR_ARG (null pointers, unknown mode, mu <= 0, or
 * mu_next <= 0 in CR_THETA_UPDATE), CR_ERR_HIP.
 */
cr_status cr_pairwise_step(cr_ctx* ctx, int32_t mode, const void* y_dev, const void* xi_dev,
                           void* gy_dev, void* gxi_dev, double mu, double mu_next);

/*
 * Run ALCC/MAPG from the context's starting point to kkt_tol (adaptive
 * schedule) or for max_outer x inner_iters MAPG iterations (fixed schedule).
 * Writes the final ALCC iterate (y_k, xi_k) to y_dev (N) and xi_dev (N x n),
 * both FP64 buffers owned by the caller, and fills *info if not NULL.
 * Host-synchronous.  The context's theta and starting point are reset
 * first, so repeated calls repeat the same computation.
 * Returns CR_OK, CR_NOT_CONVERGED (adaptive schedule, kkt_tol not reached
 * within max_outer; outputs and info still valid), CR_ERR_NONFINITE,
 * CR_ERR_ARG or CR_ERR_HIP.
 */
cr_status cr_run(cr_ctx* ctx, void* y_dev, void* xi_dev, cr_info* info);

/*
 * cr_init + cr_run + cr_destroy in one call (the workspace is borrowed only
 * for the duration of the call).  Host-synchronous.  Same errors as those.
 */
cr_status cr_solve(const void* X_dev, const void* ybar_dev, int64_t N, int32_t n,
                   const cr_params* params, void* y_dev, void* xi_dev,
                   void* workspace_dev, size_t ws_bytes, cr_info* info, void* stream);

/* Batched form --------------------------------------------------------- */

/*
 * One of P independent problems of the batched form: N points of dimension n,
 * device pointers to its FP64 inputs X (N x n), ybar (N) and outputs y (N),
 * xi (N x n), all owned by the caller.
 */
typedef struct {
    int64_t N;
    int32_t n, tile_rows;    /* tile_rows as in cr_params; 0 = the batch's params value */
    const void* X_dev;
    const void* ybar_dev;
    void* y_dev;
    void* xi_dev;
} cr_problem;

typedef struct cr_batch cr_batch;

/* Bytes of device workspace for the batch (the sum of the single-problem
 * workspaces plus argument tables).  Errors as cr_workspace_bytes, and
 * CR_ERR_UNSUPPORTED for CR_MIXED_BF16 (the batched form runs CR_F64 and
 * CR_F32). */
cr_status cr_batch_workspace_bytes(const cr_problem* probs, int32_t P, const cr_params* params, size_t* bytes);

/*
 * Solve P independent instances of eq. "regularize" (Sec. II-C) with ALCC/MAPG
 * (Fig. 3, Fig. 4), all problems advanced together: each MAPG iteration of
 * every problem still running is one replay step of a captured graph made of
 * one persistent pair pass per operand class (problems with equal
 * ceil((n + 1) / 4)), one batched reduction and one batched update.  Every
 * problem keeps its own schedule, multipliers and stopping tests (the same
 * as cr_run), and a problem that reaches kkt_tol is frozen while the others
 * continue.  The ALCC iterations of all problems advance in lockstep.
 * cr_batch_init borrows the problems' buffers and the workspace until
 * cr_batch_destroy; it runs every problem's set-up (host-synchronous).
 * cr_batch_run is host-synchronous, writes every problem's y and xi, fills
 * infos[0..P-1] when not NULL and the wall seconds when not NULL; returns
 * CR_OK, CR_NOT_CONVERGED (some problem not converged), CR_ERR_NONFINITE or
 * CR_ERR_HIP.  cr_solve_batched = init + run + destroy.
 */
cr_status cr_batch_init(cr_batch** out, const cr_problem* probs, int32_t P, const cr_params* params,
                        void* workspace_dev, size_t ws_bytes, void* stream);
cr_status cr_batch_run(cr_batch* batch, cr_info* infos, double* seconds);
/* cr_batch_run in bounded pieces, for callers that interleave other work or
 * report progress: cr_batch_start restarts every problem (asynchronous);
 * cr_batch_advance launches at most max_replays graph replays (each one
 * MAPG iteration block of every running problem plus the multiplier steps
 * that became due; see cr_params inner_iters) and sets *running to 0 once
 * every problem's schedule has finished (host-synchronous except for a fixed
 * schedule, whose replay count is known and which only enqueues); and
 * cr_batch_finish waits, writes the outputs and infos as cr_batch_run does
 * and returns its status (seconds: since cr_batch_start).  CR_ERR_STATE when
 * advance or finish is called without a start. */
cr_status cr_batch_start(cr_batch* batch);
cr_status cr_batch_advance(cr_batch* batch, int32_t max_replays, int32_t* running);
cr_status cr_batch_finish(cr_batch* batch, cr_info* infos, double* seconds);
cr_status cr_batch_destroy(cr_batch* batch);
/* Host-synchronous timing hook: average device milliseconds of one batched
 * pair pass over every problem (one persistent pass kernel per operand class,
 * back to back), run reps times on the batch's internal stream after one
 * untimed pass, bracketed by HIP events.  Every problem is made active at its
 * current operands first; theta is only read, and a later cr_batch_run starts
 * afresh.  Errors: CR_ERR_ARG (NULL, reps < 1), CR_ERR_HIP. */
cr_status cr_batch_time_pass(cr_batch* batch, int32_t reps, double* avg_ms);
cr_status cr_solve_batched(const cr_problem* probs, int32_t P, const cr_params* params, void* workspace_dev,
                           size_t ws_bytes, cr_info* infos, void* stream);

/* Differentiable form --------------------------------------------------- */

typedef struct cr_diff cr_diff;

/*
 * The fixed-schedule map of ALCC (Fig. 3) with MAPG (Fig. 4): from a given
 * start (y0, xi0) and theta_1 = 0, exactly params->max_outer ALCC iterations
 * of params->inner_iters MAPG steps each, with the constants of cr_run's fixed
 * schedule (mu_k, L^y_k, L^xi_k, the ball radii, the momentum weights); the
 * output is the last ALCC iterate (y_K, xi_K).  The reverse pass gives the
 * vector-Jacobian product of this map with respect to X, ybar, y0 and xi0,
 * holding the step constants and radii fixed (they depend on the data only
 * through sigma_max(A2)^2 and Bbar; the *_override fields fix them).  The
 * derivative of (v)_- is taken as -[v < 0], of the ball projections as that
 * of the branch the forward took.
 *
 * Memory: theta_k of every ALCC iteration k >= 2 is kept (max_outer - 1 pair
 * arrays of the pass precision), the iterate state every checkpoint_every
 * MAPG steps (and at each ALCC iteration's start); the reverse pass recomputes
 * each segment of checkpoint_every steps from its checkpoint.
 *
 * cr_diff_workspace_bytes: bytes of device workspace.  CR_ERR_ARG when
 * inner_iters < 1 (the map needs a fixed schedule) or checkpoint_every < 1,
 * CR_ERR_UNSUPPORTED for CR_MIXED_BF16 (the adjoint runs CR_F64 and CR_F32),
 * and the errors of cr_workspace_bytes.
 */
cr_status cr_diff_workspace_bytes(int64_t N, int32_t n, const cr_params* params, int32_t checkpoint_every,
                                  size_t* bytes);

/*
 * Borrows X (N x n) and ybar (N), FP64 device arrays, and the workspace until
 * cr_diff_destroy; runs the set-up of cr_init (host-synchronous).  stream
 * orders the work as in cr_init.  Errors as cr_diff_workspace_bytes and
 * cr_init.
 */
cr_status cr_diff_init(cr_diff** out, int64_t N, int32_t n, const cr_params* params, int32_t checkpoint_every,
                       const void* X_dev, const void* ybar_dev, void* workspace_dev, size_t ws_bytes,
                       void* stream);

/*
 * Forward map from the start y0_dev (N), xi0_dev (N x n), FP64 device arrays
 * (y0 NULL: y0 = ybar; xi0 NULL: xi0 = 0), writing (y_K, xi_K) to y_dev (N)
 * and xi_dev (N x n) and the checkpoints to the workspace.  info (may be
 * NULL): the KKT scalars of the last multiplier step, inner/outer counts,
 * seconds and pair updates.  Host-synchronous.  CR_OK, CR_ERR_ARG,
 * CR_ERR_NONFINITE, CR_ERR_HIP.
 */
cr_status cr_diff_forward(cr_diff* d, const void* y0_dev, const void* xi0_dev, void* y_dev, void* xi_dev,
                          cr_info* info);

/*
 * Reverse pass of the last forward: for the cotangents gy_dev (N) and gxi_dev
 * (N x n, NULL = 0) of (y_K, xi_K), writes the gradients of
 * <gy, y_K> + <gxi, xi_K> to dX_dev (N x n), dybar_dev (N), dy0_dev (N) and
 * dxi0_dev (N x n), FP64 device arrays owned by the caller.  May be called
 * again for other cotangents.  Host-synchronous.  CR_ERR_STATE before a
 * forward; CR_ERR_ARG, CR_ERR_HIP.
 */
cr_status cr_diff_backward(cr_diff* d, const void* gy_dev, const void* gxi_dev, void* dX_dev, void* dybar_dev,
                           void* dy0_dev, void* dxi0_dev);

cr_status cr_diff_destroy(cr_diff* d);

/* Host-synchronous: average device time in milliseconds of one adjoint pair
 * pass of a MAPG step (with the theta-bar accumulation when max_outer >= 2),
 * at the operands left by the last cr_diff_backward, launched reps times back
 * to back with the reverse pass's launch configuration and bracketed by HIP
 * events.  It only adds to the theta-bar scratch array, which the next
 * backward clears.  CR_ERR_STATE before a backward; CR_ERR_ARG, CR_ERR_HIP. */
cr_status cr_diff_time_adjoint_pass(cr_diff* d, int32_t reps, double* avg_ms);

/* P-APG on the partial dual ------------------------------------------------ */

/*
 * P-APG (Sec. II-B to II-D, Fig. 2).  The N points split into K index sets
 * C_i of Nbar = N / K consecutive points (Sec. II-B); the constraints of
 * pairs in different sets, and y >= 0, are dualised (C = [A3 A4; I 0],
 * eq. "C"), and the dual eq. "lambda_dual" is maximised over
 * Q2 = {theta >= 0, ||theta||_2 <= B_theta} with accelerated projected
 * gradient steps.  Iteration l (theta^(1)_0 = theta^(2)_1 = 0, t_1 = 1):
 *   1. eta_l = (y, xi) minimising the Lagrangian of eq. "g_gamma" at
 *      theta^(2)_l over the within-block constraints: K independent problems,
 *      block i being eq. "regularize" on its points with data
 *      ybar_i + y_shift + (A3^T theta + theta_y)_i and the slope term
 *      gamma/2 ||xi_i - (A4^T theta)_i / gamma||^2, solved together by the
 *      batched ALCC (cr_solve_batched's machinery) with `alcc`'s schedule
 *      (alcc->tile_rows = 0: row chunks sized for about 512 work items over
 *      all blocks, the batched pass's persistent grid),
 *      each from its affine fit with zero within-block multipliers;
 *   2. theta^(1)_l = Pi_Q2(theta^(2)_l - C eta_l / L);
 *   3-4. t_{l+1} = (1 + sqrt(1 + 4 t_l^2))/2 and
 *      theta^(2)_{l+1} = theta^(1)_l + (t_l - 1)/t_{l+1} (theta^(1)_l - theta^(1)_{l-1}).
 * Outputs: eta of the last step 1 (y shifted back by y_shift) and, when the
 * pointers are not NULL, theta^(1) of the last iteration: theta_dev N x N
 * row-major FP64 (entry (i, j) for the pair (i, j); zero inside the diagonal
 * blocks), theta_y_dev N.
 */
typedef struct {
    int32_t K;          /* number of index sets; N % K == 0 and N / K >= 2 */
    int32_t iters;      /* P-APG iterations, >= 1 */
    double L;           /* step constant (L_g of eq. "lischitz" or above); <= 0:
                           (2N + sigma_max(A2)^2 + 1) / gamma, a bound of L_g */
    double B_theta;     /* radius of Q2; <= 0 or +Inf: the nonnegative orthant */
    double y_shift;     /* added to ybar so that y >= 0 holds at the solution
                           (Sec. II-D) and subtracted from y on output;
                           < 0: max(0, max(ybar) - 2 min(ybar)) */
    int32_t method;     /* CR_PAPG_ACCELERATED: Fig. 2; CR_PAPG_GRADIENT: steps
                           3-4 dropped (theta^(2)_{l+1} = theta^(1)_l), the
                           projected gradient ascent P-APG is compared with in Sec. III */
    int32_t power_iters; /* with L <= 0: 0 takes the bound above; > 0 runs that many
                           power iterations on C^T C (from a fixed start) and takes
                           L = min(bound, 1.05 ||C v||^2 / gamma), v the last unit
                           iterate (a lower estimate of sigma_max(C)^2, 5% added) */
} cr_papg_params;

enum { CR_PAPG_ACCELERATED = 0, CR_PAPG_GRADIENT = 1 };

typedef struct {
    double L, y_shift;          /* the constants used */
    double theta_norm;          /* ||theta^(1)|| of the last iteration */
    double infeas_cross;        /* ||(A3 y + A4 xi)_-||_2 of the last eta */
    int64_t inner_iters;        /* MAPG iterations, summed over blocks and P-APG iterations */
    double seconds;
} cr_papg_info;

/* Bytes of device workspace for cr_papg: two N x N FP64 multiplier arrays, the
 * block data and outputs, and the batched ALCC's workspace for K problems of
 * Nbar points.  Errors: CR_ERR_ARG (NULL, bad params, N % K != 0,
 * N / K < 2, iters < 1, unknown method), CR_ERR_UNSUPPORTED (as
 * cr_batch_workspace_bytes). */
cr_status cr_papg_workspace_bytes(int64_t N, int32_t n, const cr_params* alcc, const cr_papg_params* pp,
                                  size_t* bytes);

/* Host-synchronous P-APG run (above).  X (N x n), ybar (N) FP64 device inputs;
 * y (N), xi (N x n) FP64 device outputs; theta_dev, theta_y_dev optional.
 * trace_host (optional, host memory of iters x 3 doubles) receives per
 * iteration l: ||theta^(1)_l||, ||(A3 y + A4 xi)_-||_2 at eta_l and
 * theta^(2)_l^T C eta_l (the objective of eq. "omega_primal" at eta_l minus
 * the Lagrangian of eq. "g_gamma" there).
 * All buffers are the caller's.  `alcc` is the block solves' schedule (its
 * precision CR_F64 or CR_F32).  Errors: as cr_papg_workspace_bytes,
 * CR_ERR_NOMEM (ws_bytes too small), CR_ERR_NONFINITE (NaN/Inf in the inputs
 * or an iterate), CR_ERR_HIP.  A block solve that ends CR_NOT_CONVERGED
 * (adaptive schedule) is not an error; info->inner_iters counts its steps. */
cr_status cr_papg(const void* X_dev, const void* ybar_dev, int64_t N, int32_t n, const cr_params* alcc,
                  const cr_papg_params* pp, void* y_dev, void* xi_dev, void* theta_dev, void* theta_y_dev,
                  double* trace_host, void* workspace_dev, size_t ws_bytes, cr_papg_info* info, void* stream);

/* Estimator evaluation ---------------------------------------------------- */

/* Sec. I: the least-squares estimator is the piecewise-linear convex function
 * that takes the value y_l at x_l with subgradient xi_l there; it is evaluated
 * at a point q as its largest supporting hyperplane,
 *   fhat(q) = max_l ( y_l + xi_l^T (q - x_l) ),
 * and the maximising l (the smallest one on exact ties) names a subgradient
 * xi_l of the estimator at q.  (y, xi) is typically the output of cr_solve;
 * any values are accepted.
 *
 * X (N x n), y (N), xi (N x n) and Q (M x n, the query points): FP64,
 * row-major, on the device of `stream`; borrowed for the call.  Outputs:
 * fhat (M doubles) and, unless arg is NULL, arg (M int64, plane indices).
 * workspace: at least cr_eval_workspace_bytes(N, n) bytes of device memory
 * (packed plane operands), caller-owned, rewritten by each call.
 * Asynchronous on `stream` (a hipStream_t; NULL is the default stream).
 * M = 0 is a no-op.  A query whose plane values are all NaN gets
 * fhat = -Inf and arg = INT64_MAX.
 * Errors (checked on the host, before any HIP call): CR_ERR_ARG (NULL
 * pointers, N < 1, n < 1, M < 0), CR_ERR_UNSUPPORTED (n > CR_MAX_DIM or
 * N >= 2^31 - 64),
 * CR_ERR_NOMEM (workspace too small); CR_ERR_HIP on a failed launch.
 * Messages in cr_last_error(NULL). */
cr_status cr_eval_workspace_bytes(int64_t N, int32_t n, size_t* bytes);
cr_status cr_eval(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n,
                  const void* Q_dev, int64_t M, void* fhat_dev, int64_t* arg_dev, void* workspace_dev,
                  size_t ws_bytes, void* stream);

/* cr_eval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and results as cr_eval, with the packed plane operands in
 * a static device array of 32 MiB that the library holds on each GPU it runs
 * on until the process ends, instead of a caller workspace.  Calls no
 * allocating routine.  Every call on a GPU shares that GPU's array, so calls
 * that overlap on one GPU (on different streams, or from several threads)
 * race and must be ordered by the caller.  Inputs, outputs, ownership,
 * asynchrony and errors as cr_eval, plus CR_ERR_NOMEM when the packed planes,
 * 32 * ceil(N / 32) * 4 * ceil((n + 1) / 4) doubles, exceed 32 MiB (N up to
 * 174752 at n = 20), and CR_ERR_HIP if the array's device address cannot be
 * obtained (looked up once per device, on the first call there). */
cr_status cr_eval_noalloc(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n,
                          const void* Q_dev, int64_t M, void* fhat_dev, int64_t* arg_dev, void* stream);

/* Inspection and test hooks --------------------------------------------- */

/* Copy the context's theta to / from an N x N FP64 device array (diagonal
 * entries are ignored on input and written as 0 on output).  Asynchronous. */
cr_status cr_get_theta(cr_ctx* ctx, void* theta_dev);
cr_status cr_set_theta(cr_ctx* ctx, const void* theta_dev);

/* Copy the ALCC starting point (the affine fit) to FP64 device arrays. */
cr_status cr_get_start(cr_ctx* ctx, void* y_dev, void* xi_dev);

/* Host-synchronous: constants of the context and, after a CR_THETA_UPDATE
 * pass or a run, the KKT scalars of the last multiplier step. */
cr_status cr_get_info(cr_ctx* ctx, cr_info* info);

/* Per-ALCC-iteration record of the last cr_run (Fig. 3): the MAPG iterations
 * of ALCC iteration k (the step at which Fig. 4's alpha test or l_max ended
 * it) and the KKT measure after its multiplier step, k = 0 .. count - 1.
 * Writes min(cap, count) entries to the host arrays and the total to *count.
 * Errors: CR_ERR_ARG (NULL ctx or count, cap < 0, NULL arrays with cap > 0). */
cr_status cr_get_outer_history(cr_ctx* ctx, int32_t cap, int64_t* inner_iters, double* kkt, int32_t* count);

/* Pure host arithmetic: the pair-pass launch layout cr_init would choose for
 * (N, n, params): out[0] Nrow (rows of theta, N rounded up to 64), out[1] ld
 * (its leading dimension), out[2] rows per workgroup chunk, out[3] chunks,
 * out[4] column strips (16 TW columns each; TW = 2 in FP64, 4 otherwise),
 * out[5] 1 if MAPG steps complete inside the next pass.  For tests of the
 * pass's buffer-view offsets.  Errors as cr_workspace_bytes. */
cr_status cr_pass_layout(int64_t N, int32_t n, const cr_params* params, int64_t* out);

/* Host-synchronous: average device time in milliseconds of the gradient pair
 * pass that cr_run launches, run reps times back to back on the context's
 * internal stream with cr_run's launch configuration, bracketed by HIP events.
 * When cr_run completes each MAPG step inside the next pass (chunk heights
 * whose LDS allows it), the timed kernel is that form at MAPG iteration 2: the
 * call first restarts MAPG at the ALCC starting point and takes one step
 * there (pass and reduction) to give it inputs, so the context's MAPG state
 * is overwritten; otherwise the plain pass at the current operands is timed.
 * theta is unchanged either way; a later cr_run starts afresh.  Only CR_GRAD
 * is accepted.  Errors: CR_ERR_ARG (NULL, reps < 1, mode other than CR_GRAD),
 * CR_ERR_HIP. */
cr_status cr_time_pass(cr_ctx* ctx, int32_t mode, int32_t reps, double* avg_ms);

#ifdef __cplusplus
}
#endif
#endif /* CR_H */
