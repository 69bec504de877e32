// Shared definitions of the gfx950 kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

namespace cr {

constexpr int kBlock = 256;          // threads per workgroup of every kernel
constexpr int kTileRows = 16;        // rows (i) of one MFMA tile
constexpr int kWaves = 4;            // waves per pair-pass workgroup, split over rows
constexpr int kMaxDim = 31;          // n + 1 <= 32 output columns of W^T [X 1]
constexpr int kMaxRowsPerChunk = 4096;  // rows of one pass workgroup (row sums staged in LDS)

// Scalars the host sets once per ALCC iteration (Fig. 3 steps 1-2, 5-6).
struct OuterArgs {
    double mu;            // mu_k
    double gamma;         // Tikhonov weight
    double sy, sxi;       // MAPG block steps step_scale / L^y_k, step_scale / L^xi_k
    double alpha_y, alpha_xi;
    double By, Bxi;       // ball radii of Q_y (centre ybar) and Q_xi (centre 0)
    double theta_scale;   // mu_k / mu_{k+1}
    int64_t lmax;         // l^max_k
    int32_t adaptive;     // 1: alpha tests of Fig. 4 active
    int32_t skip;         // 1: problem already converged (batched form); MAPG does not run
};

// ALCC (Fig. 3) carried on the device.  The host writes the constants once
// (cr_init); k_alcc_start, k_alcc_gate and k_alcc_step advance the state, so
// a whole solve is enqueued with no read-back between ALCC iterations: the
// schedule's scalars (mu_k, tau_k, alpha_k, l^max_k), the decision that a MAPG
// run is over, the multiplier step that follows it and the KKT test all run
// inside the captured graph.
struct AlccSched {
    // constants of the context
    double mu1, c, kappa, tau1, ay1, axi1, gamma, step_scale, kkt_tol;
    double Ly_ovr, Lxi_ovr, By_ovr, Bxi_ovr, sigma2_A1;
    int64_t inner_iters, max_inner;
    int32_t max_outer, pad0;
    int64_t* hist_inner;      // max_outer entries: MAPG iterations of ALCC iteration k
    double* hist_kkt;         // and the KKT measure after its multiplier step
    // state of the current run
    double mu, tau, ay, axi;
    int64_t total_inner;
    int32_t k;                // ALCC iterations begun
    int32_t phase;            // 0 MAPG running, 1 multiplier step due, 2 done
    int32_t converged, nonfinite;
};

// Device-side state.  Written by kernels only (the host reads it back).
struct DevState {
    // problem constants (set up once)
    double ybar_mean, ybar_inf, sigma2_A2, Bbar, aff_b, pad_c;
    int32_t nonfinite, one;           // `one` stays 1: the activity flag of stand-alone passes
    // MAPG loop
    int64_t base;                     // iterations launched before the current graph replay
    int64_t it;                       // MAPG iterations done in this ALCC iteration (set at the stop)
    int32_t active, stopped_by_alpha;
    double dy, dxi;                   // ||y1 - y2||, ||xi1 - xi2|| of the last step
    // KKT of the last multiplier step
    double stat_y, stat_xi, infeas, compl_, infeas_sq, gap, obj, xi_sq;
    int32_t iterate_nonfinite;
    int32_t step_due;                 // 1 from the end of a MAPG run until its multiplier step is done
    // arrival counters of the last-block reductions
    unsigned int cnt[4];
};

// Packed per-lane X operands of one 16-row tile: for lane l = 16 g + c,
//   q <  KS           : A operand of R = [X 1] Xi_aug^T, element X_aug[i0 + c][4 q + g]
//   KS <= q < KS+4NKB : B operand of C = W^T X_aug,      element X_aug[i0 + rmap(g, s)][16 kb + c]
//                        with s = (q - KS) % 4, kb = (q - KS) / 4
// where X_aug[i] = [x_i, 1, 0, ...] (zero rows for i >= N) and rmap is the
// accumulator row map of the pass precision (4 g + s for FP32, g + 4 s for FP64).
__host__ __device__ constexpr int ks_of(int n) { return (n + 1 + 3) / 4; }
__host__ __device__ constexpr int nkb_of_ks(int ks) { return ks <= 4 ? 1 : 2; }
__host__ __device__ constexpr int q_of_ks(int ks) { return ks + 4 * nkb_of_ks(ks); }
__host__ __device__ constexpr int qp_of_ks(int ks, int elem) {
    // padded to whole 16-byte vectors
    return ((q_of_ks(ks) * elem + 15) / 16) * 16 / elem;
}
// Mixed precision: K = 3n BF16 slots of the residual contraction in blocks of 32.
__host__ __device__ constexpr int mixed_kb(int n) { return (3 * n + 31) / 32; }

// Lazy MAPG step.  In a captured MAPG run the gradient pass of iteration l >= 2
// first completes step l - 1 (Fig. 4 steps 1-2 and 4) for the points it touches:
// from the unprojected steps v = (vy, vxi) that the reduce kernel wrote and the
// two norms ||vy - ybar||, ||vxi|| (summed from that kernel's block records),
//   y1 = Proj_{Q_y}(vy),  y2 = y1 + beta_{l-1} (y1 - y1_{l-2})   (xi alike),
// and takes its operands from (y2, xi2) directly.  Iterate y1_m lives in
// y1p[m & 1] (y1_0, the start, in y1p[0]).  Workgroups of strip 0 write the
// state (y1, y2) of their rows, workgroups of chunk 0 that of their columns'
// xi, together with the pieces of the stopping test ||y1 - y2_{l-1}||^2
// (spart[chunk]) and ||xi1 - xi2_{l-1}||^2 (spart[chunks + strip]).  At l = 1
// the operands come from xiaug / ycol (set by k_set_point).
struct LazyStep {
    int32_t on, q;            // q: position of the iteration in the captured replay
    int32_t lfix, n;          // lfix > 0: iteration number to use instead of base + q + 1
    int32_t nblk, chunks;     // records in npart; chunk count of the pass grid
    const double* vy;         // N
    const double* vxi;        // N x n
    const double* X;          // N x n
    const double* ybar;       // N
    double* y1p[2];           // N each
    double* xi1p[2];          // N x n each
    double* y2;               // y^(2)_l (N), read by the reduce kernel
    double* xi2;              // xi^(2)_l (N x n)
    const double* beta;       // beta[l] = (t_l - 1) / t_{l+1}
    const double* npart;      // reduce block records: fields 0, 1 = pieces of ||vy - ybar||^2, ||vxi||^2
    double* spart;            // chunks + strips stopping-test pieces
    const OuterArgs* oa;
    DevState* st;
    const double* shift;      // slope shift c (N x n, null: none): column operands from xi2 + c
};

struct PassArgs {
    int64_t N, Nrow, ld;      // points, padded rows (x16), theta row stride (x64)
    int32_t nc;               // n + 1
    int32_t rows_per_chunk;   // multiple of 64
    int32_t mode;             // 0 gradient pass, 1 multiplier (theta) pass
    int32_t check_first;      // 1: test the activity flag before any tile load (batched adaptive runs)
    void* theta;              // Nrow x ld, pass precision
    const void* xp;           // packed X operands, (Nrow/16) x 64 x QP
    const void* xiaug;        // ld x KP: [-xi_j, d_j - y_j, 0..]
    const void* ycol;         // Nrow: y_i
    void* rowpart;            // strips x Nrow
    void* cpart;              // chunks x ld x nc
    double* kktpart;          // (strips*chunks) x 4
    double theta_scale;       // mu_k / mu_{k+1} (multiplier pass)
    const double* theta_scale_p;   // non-null: read mu_k / mu_{k+1} here instead (device schedule)
    const int32_t* active;
    const float* cvec;        // mixed precision: c_j = x_j^T xi_j - y_j in FP32 (ld)
    LazyStep lz;              // gradient passes of a captured MAPG run (lz.on = 1)
};

// Sum of the pass partials for point j, then the gradient (mode 1), the MAPG
// gradient step (mode 0) or the KKT residuals of a multiplier step (mode 2).
struct ReduceArgs {
    int64_t N, Nrow, ld;
    int32_t n, nc, strips, chunks, mode, npass;   // mode 0 MAPG step, 1 gradient out, 2 KKT
    int32_t q;                // mode 0: position of the iteration in the captured replay
    int32_t mu_dev;           // mode 2: 1 = mu_k from oa->mu (device schedule), 0 = from `mu`
    int32_t check_first, pad; // check_first as in PassArgs
    const void* rowpart;
    const void* cpart;
    const double* X;
    const double* ybar;
    const double* y;
    const double* xi;
    double* out_y;
    double* out_xi;
    double* blockpart;        // gridDim.x x 4 (one record per block)
    const double* kktpart;    // npass x 4 (mode 2)
    const OuterArgs* oa;
    DevState* st;
    double mu, gamma;         // modes 1 and 2
    // mode 0 after lazy passes: the stopping-test pieces of the pass
    // (spart[0 .. chunks) for y, spart[chunks .. chunks + strips) for xi);
    // null: fields 2 and 3 of the update kernel's block records
    const double* spart;
    const int32_t* gate;      // mode 2, non-null: run only while *gate != 0
};

// Completion of a MAPG step (Fig. 4): projections, momentum, stopping test.
struct UpdateArgs {
    int64_t N, ld;
    int32_t n, kp;
    int32_t q, pad;           // position of the iteration in the captured replay
    const double* beta;       // beta[l] = (t_l - 1) / t_{l+1}, l = 1, 2, ... (momentum of Fig. 4)
    const double* X;
    const double* ybar;
    const double* vy;
    const double* vxi;
    double* y1p;     // y^(1)_{l-1} in, y^(1)_l out
    double* y2;      // y^(2)_l in, y^(2)_{l+1} out
    double* xi1p;
    double* xi2;
    void* xiaug;     // pass precision (mixed: BF16 hi/lo slots)
    void* ycol;
    float* cvec;     // mixed precision only
    double* blockpart;
    const OuterArgs* oa;
    DevState* st;
    // optional copies for the adjoint (null otherwise): the pass point y^(2)_l,
    // xi^(2)_l, the unprojected step v_l, and the two norms ||v - centre||
    double* sv_y2;
    double* sv_xi2;
    double* sv_vy;
    double* sv_vxi;
    double* sv_nrm;
    // slope shift c (N x n, null: none): the operands of the next pass are
    // built from xi + c (problems posed in shifted slopes, see k_su_shift)
    const double* shift;
};

// Operands of the next pass at (y, xi), optionally restarting MAPG there.
struct PointArgs {
    int64_t N, Nrow, ld;
    int32_t n, kp, write_state, pad;
    const double* X;
    const double* y;
    const double* xi;
    double* y1p;
    double* y2;
    double* xi1p;
    double* xi2;
    void* xiaug;
    void* ycol;
    float* cvec;     // mixed precision only
    const double* shift;   // slope shift c (null: none); operands from xi + c
    const int32_t* gate;   // non-null: run only while *gate != 0
};

// Message for cr_last_error(NULL) (context-free calls outside cr_api.hip).
void set_last_error(const std::string& msg);

// prec: 0 FP64, 1 FP32, 2 mixed BF16 (the pass precision of cr.h)
hipError_t launch_pair_pass(int prec, int n, const PassArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_reduce(bool f64, const ReduceArgs& a, hipStream_t s);
hipError_t launch_update(int prec, const UpdateArgs& a, hipStream_t s);
hipError_t launch_set_point(int prec, const PointArgs& a, hipStream_t s);
hipError_t launch_begin_outer(const OuterArgs& args, OuterArgs* dst, DevState* st, hipStream_t s,
                              int64_t base = 0);
// launched < 0: the iteration base st->base (device schedule); gate non-null:
// only while *gate != 0.
hipError_t launch_mapg_end(const double* blockpart, int nblk, int64_t launched, DevState* st, hipStream_t s,
                           const int32_t* gate = nullptr);
// After a run of lazy passes: y1_it (xi1_it) into y1p[0] (xi1p[0]); if the run
// ended at l^max with no pass after the last step, that step's projection.
hipError_t launch_mapg_finish(const LazyStep& lz, int64_t N, hipStream_t s, const int32_t* gate = nullptr);
// The same over the problems of a batch whose multiplier step is due (lazy
// gradient-pass table `args`, block table of G lanes per point).
hipError_t launch_mapg_finish_batched(int G, const PassArgs* args, const void* blocks, int nblocks, hipStream_t s);
// Device schedule (AlccSched): start of a run (first ALCC iteration begun),
// end of a graph replay of `iters` MAPG iterations (the run is over once MAPG
// stopped or l^max iterations ran: the multiplier step becomes due), and the
// step after the multiplier step (history, KKT test, next ALCC iteration).
hipError_t launch_alcc_start(AlccSched* s, OuterArgs* oa, DevState* st, hipStream_t strm);
hipError_t launch_alcc_gate(AlccSched* s, DevState* st, const OuterArgs* oa, int iters, hipStream_t strm);
hipError_t launch_alcc_step(AlccSched* s, DevState* st, OuterArgs* oa, hipStream_t strm);
// The same over P problems (tables of per-problem pointers); the gate also
// writes whether any problem is not done.
hipError_t launch_alcc_start_batched(AlccSched* const* s, OuterArgs* const* oa, DevState* const* st, int P,
                                     hipStream_t strm);
hipError_t launch_alcc_gate_batched(AlccSched* const* s, DevState* const* st, OuterArgs* const* oa, int P,
                                    int iters, int32_t* running, hipStream_t strm);
hipError_t launch_alcc_step_batched(AlccSched* const* s, DevState* const* st, OuterArgs* const* oa, int P,
                                    hipStream_t strm);
// Batched multiplier-step pieces (device schedule), each gated per problem on
// its step_due flag: the MAPG end, the set point, the multiplier pass of one
// operand class (mode-1 PassArgs table) and the KKT reduction (mode-2
// ReduceArgs table).
hipError_t launch_mapg_end_batched(const double* const* blockparts, const int32_t* nblk, DevState* const* st, int P,
                                   hipStream_t strm);
hipError_t launch_set_point_batched(bool f64, int G, const PointArgs* args, const void* blocks, const int32_t* nblk,
                                    int nblocks, hipStream_t strm);
hipError_t launch_theta_pass_batched(bool f64, int ks, const PassArgs* args, const int32_t* nstrips,
                                     const void* items, int nitems, hipStream_t strm);
// Largest rows per chunk for which a lazy pass's LDS (row sums, y operands and
// staged column operands) fits the pass workgroup's 32 KiB area.
bool lazy_fits(int prec, int64_t rows_per_chunk);
// Start of a problem posed in shifted slopes xi = xi' + c: xi0 <- xi0 - c and
// st->Bbar = sqrt(||y0 - ybar||^2 + gamma ||xi0 - c||^2) (one workgroup).
hipError_t launch_setup_shift(const double* y0, const double* ybar, double* xi0, const double* shift, int64_t N,
                              int n, double gamma, DevState* st, hipStream_t s);

// Rows per workgroup of the set-up sums (means, centred scatter, X_c^T ybar_c).
constexpr int64_t kSuRows = 64;
// The set-up again for new data ybar on the same points: means, the affine fit
// from the eigen-decomposition the full set-up left in su, the start point and
// Bbar; sigma_max(A2)^2 (a function of X alone) is kept.
// Re-fit of up to kMaxRefit problems in one launch per step (launch_refit's
// kernels, then the slope shift where a problem has one); the table travels in
// the kernel arguments.
constexpr int kMaxRefit = 16;
struct RefitArgs {
    const double* X;
    const double* ybar;
    int64_t N;
    int32_t n, pad;
    double gamma;
    double* su;
    double* part;
    double* y0;
    double* xi0;
    DevState* st;
    const double* shift;      // null: no slope shift
};
struct RefitTable { RefitArgs p[kMaxRefit]; int32_t K; };
hipError_t launch_refit_batched(const RefitTable& t, hipStream_t s);
hipError_t launch_refit(const double* X, const double* ybar, int64_t N, int n, double gamma, double* su,
                        double* part, double* y0, double* xi0, DevState* st, hipStream_t s);

// P-APG (Fig. 2) kernels, see cr_papg.hip.
struct PapgArgs {
    int64_t N, Nbar;
    int32_t n, it;            // it: 0-based iteration (row of the trace)
    double beta;              // (t_{l-1} - 1) / t_l: theta2 = tc + beta (tc - tp)
    double L, gamma, yshift, B;   // step constant of Fig. 2 step 2, Tikhonov weight, data shift, ball radius
    const double* X;
    const double* ybar;
    double* tc;               // theta^(1)_{l-1}, N x N (cross entries; diagonal blocks 0)
    double* tp;               // theta^(1)_{l-2} in, theta^(1)_l out
    double* tyc;              // the same for the y >= 0 multipliers (N)
    double* typ;
    double* ybs;              // block data ybar + yshift + u (N)
    double* shift;            // block slope centres v / gamma (N x n)
    const double* y;          // step-1 output y (N)
    const double* xis;        // step-1 output in shifted slopes xi' (N x n)
    double* part;             // per-workgroup partial sums of k_papg_step2 (3 each)
    double* cpart;            // column partials of k_papg_colsum: [row chunk][N][n + 1]
    double* scal;             // [scale, ||theta||, ||(r_cross)_-||, theta2^T C eta, power: ||C v||^2, ||w||]
    double* trace;            // per iteration: ||theta||, ||(r_cross)_-||, theta2^T C eta
};
constexpr int kPapgStepRows = 32;     // rows per workgroup of k_papg_step2
__host__ __device__ inline int64_t papg_step_parts(int64_t N) { return ((N + kBlock - 1) / kBlock) * ((N + kPapgStepRows - 1) / kPapgStepRows); }
// Rows per workgroup of k_papg_colsum: 64, or more once that would give more
// than 64 row chunks (the partials hold chunks x N x (n + 1) doubles).
__host__ __device__ inline int64_t papg_col_rows(int64_t N) { return N <= 64 * 64 ? 64 : ((N + 63) / 64 + 7) / 8 * 8; }
__host__ __device__ inline int64_t papg_col_chunks(int64_t N) { return (N + papg_col_rows(N) - 1) / papg_col_rows(N); }
hipError_t launch_papg_lin(const PapgArgs& a, hipStream_t s);
hipError_t launch_papg_step2(const PapgArgs& a, hipStream_t s);
hipError_t launch_papg_out(const PapgArgs& a, double* y_out, double* xi_out, hipStream_t s);
// `iters` power iterations on C^T C from a fixed start; afterwards scal[4] is
// ||C v||^2 for the last unit vector v (a lower estimate of sigma_max(C)^2).
// Uses tc as the scratch pair array, ybs/shift as scratch vectors and part.
hipError_t launch_papg_power(const PapgArgs& a, double* vy, double* vxi, const double* zero, int iters,
                             hipStream_t s);
int reduce_blocks(int64_t N, int n);
int reduce_blocks_g(int64_t N, int G);
// Batched form (plain precisions): see cr_batch.hip.
// One pass per operand class ks = ceil((n + 1) / 4), one workgroup per item of
// that class.  lazy: the passes complete the previous MAPG step (LazyStep of
// each table entry) at replay position q.
hipError_t launch_pass_batched(bool f64, int ks, const PassArgs* args, const int32_t* nstrips, const void* items,
                               int nitems, hipStream_t s, bool lazy = false, int q = 0);
hipError_t launch_reduce_batched(bool f64, int G, const ReduceArgs* args, const void* blocks, const int32_t* nblk,
                                 int nblocks, int q, hipStream_t s);
hipError_t launch_update_batched(bool f64, int G, const UpdateArgs* args, const void* blocks, const int32_t* nblk,
                                 int nblocks, int q, hipStream_t s);
hipError_t launch_prep_xp(int prec, const double* X, int64_t N, int n, int64_t Nrow, int ks, int qp, void* xp,
                          hipStream_t s);
hipError_t launch_theta_import(bool f64, const double* src, int64_t N, int64_t Nrow, int64_t ld, void* theta,
                               hipStream_t s);
hipError_t launch_theta_export(bool f64, const void* theta, int64_t N, int64_t ld, double* dst, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_setup(const double* X, const double* ybar, int64_t N, int n, double gamma, double* su,
                        double* part, double* y0, double* xi0, DevState* st, hipStream_t s);

// ---------------------------------------------------------------------------
// Adjoint (reverse-mode) kernels of the fixed-schedule map (cr_adjoint.hip).
// ---------------------------------------------------------------------------
// Pair pass of the adjoint.  Mode 0 (MAPG step): at the pass point (operands
// xiaug, ycol) with theta_k, mask m_ij = [theta_ij - r_ij > 0] (valid pairs),
// W = m (theta - r), and the direction (a, b) (operands diraug, acol) gives
// rho = A1 a + A2 b and z = m rho.  Mode 1 (multiplier step): z = scale m thetabar.
// Outputs (partials, summed by k_adj_reduce):
//   rowpart [strip][i]     sum_j z_ij
//   rowvpart[strip][i][k]  sum_j (W_ij (-b_jk) - z_ij (-xi_jk))
//   cpart   [chunk][j][k]  Z^T [X 1]  (k < n: sum_i z_ij x_ik, k = n: sum_i z_ij)
//   cwpart  [chunk][j]     sum_i W_ij  (mode 0)
// thetabar: mode 0 with tb_mode 1: thetabar += z; mode 1 with tb_mode 2: thetabar = z.
struct AdjPassArgs {
    int64_t N, Nrow, ld;
    int32_t n, nc, rows_per_chunk, kp;
    int32_t mode, tb_mode;
    const void* theta;
    void* thetabar;
    const void* xp;
    const void* xiaug;
    const void* ycol;
    const void* diraug;
    const void* acol;
    void* rowpart;
    void* rowvpart;
    void* cpart;
    void* cwpart;
    double scale;
};

struct AdjReduceArgs {
    int64_t N, Nrow, ld;
    int32_t n, nc, strips, chunks, mode, pad;
    const void* rowpart;
    const void* rowvpart;
    const void* cpart;
    const void* cwpart;
    const double* X;
    const double* xi;          // xi of the pass point
    const double* vb_y;        // mode 0: projected adjoint (v-bar)
    const double* vb_xi;
    double sy, sxi, mu, gamma;
    double* out_y;             // mode 0: q-bar (written); mode 1: adjoint of (y_k, xi_k) (added to)
    double* out_xi;
    double* dybar;             // mode 0: += a / mu
    double* dX;
};

// Momentum and projection adjoints of one MAPG step (vector kernels).
struct AdjVecArgs {
    int64_t N, Nrow, ld;
    int32_t n, kp;
    double beta, sy, sxi, By, Bxi;
    const double* X;
    const double* ybar;
    double* pb_y;              // adjoint of y^(1)_l (in), of y^(1)_{l-1} (out)
    double* pb_xi;
    const double* qb_y;        // adjoint of y^(2)_{l+1}
    const double* qb_xi;
    double* g1_y;              // adjoint of y^(1)_l
    double* g1_xi;
    const double* v_y;         // saved unprojected step v_l
    const double* v_xi;
    const double* nrm;         // saved ||v_y - ybar||, ||v_xi||
    double* vb_y;              // projected adjoint v-bar (out)
    double* vb_xi;
    double* dybar;             // += adjoint of the ball centre
    void* diraug;              // direction operands [-b_j, x_j^T b_j - a_j, 0..], b = sxi vb_xi
    void* acol;                // a = sy vb_y
    double* blockpart;         // per block: dot products (y, xi)
};

hipError_t launch_adj_pass(bool f64, int n, const AdjPassArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_adj_reduce(bool f64, const AdjReduceArgs& a, hipStream_t s);
hipError_t launch_adj_momentum(const AdjVecArgs& a, hipStream_t s);
hipError_t launch_adj_project(bool f64, const AdjVecArgs& a, int nblk, hipStream_t s);
hipError_t launch_add(double* out, const double* a, const double* b, int64_t count, hipStream_t s);
int adj_vec_blocks(int64_t N, int n);

}  // namespace cr
