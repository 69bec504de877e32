// Host driver of the convex-regression pair engine: argument checks, workspace
// layout, set-up, and the ALCC (Fig. 3) / MAPG (Fig. 4) schedule.  The MAPG
// iteration [pair pass -> reduction + step -> projection + momentum] is
// captured once as a hipGraph of kGraphIters iterations and replayed; the
// alpha test of Fig. 4 and the l_max cap are evaluated on the device, which
// turns the remaining iterations of a replay into no-ops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cr.h"
#include "cr_device.h"


namespace {

constexpr int kGraphIters = 32;
thread_local std::string g_last_error;

struct Layout {
    int64_t N = 0, Nrow = 0, ld = 0;
    int n = 0, nc = 0, ks = 0, kp = 0, qp = 0, esz = 8, tw = 2;
    int strips = 0, chunks = 0, rpc = 0, nb = 0, nsu = 0;
    size_t off_theta, off_xp, off_xiaug, off_ycol, off_rowpart, off_cpart, off_kkt;
    size_t off_y1p, off_y2, off_vy, off_y0, off_xi1p, off_xi2, off_vxi, off_xi0;
    size_t off_blockpart, off_supart, off_su, off_oa, off_st, off_beta, off_cvec;
    size_t off_y1p1, off_xi1p1, off_spart;   // second iterate buffers and stopping-test pieces (lazy passes)
    size_t off_sched, off_hist;              // device ALCC schedule and its per-iteration history
    bool lazy = false;                       // MAPG runs use lazy passes (their LDS fits this chunk height)
    int prec = 0;
    int64_t nbeta = 0;
    size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t max_mapg_iters(const cr_params& p);

Layout make_layout(int64_t N, int n, const cr_params& prm, int tile_rows) {
    const int precision = prm.precision;
    const int64_t max_iters = max_mapg_iters(prm);
    Layout L;
    L.N = N;
    L.n = n;
    L.nc = n + 1;
    L.prec = precision;
    L.esz = precision == CR_F64 ? 8 : 4;
    L.tw = L.esz == 8 ? 2 : 4;
    L.Nrow = ((N + 63) / 64) * 64;
    L.ld = ((N + 63) / 64) * 64;
    L.ks = cr::ks_of(n);
    L.kp = 4 * L.ks;
    L.qp = cr::qp_of_ks(L.ks, L.esz);
    size_t xp_bytes = (size_t)(L.Nrow / 16) * 64 * L.qp * L.esz;
    size_t xiaug_bytes = (size_t)L.ld * L.kp * L.esz;
    if (precision == CR_MIXED_BF16) {
        // BF16 operand slots: kp per column, (KB + NKB) 16-byte vectors per lane and tile
        L.kp = 32 * cr::mixed_kb(n);
        L.qp = cr::mixed_kb(n) + (n + 1 + 15) / 16;
        xp_bytes = (size_t)(L.Nrow / 16) * 64 * L.qp * 16;
        xiaug_bytes = (size_t)L.ld * L.kp * 2;
    }
    L.strips = (int)(L.ld / (16 * L.tw));
    // Enough workgroups to fill 256 CUs several times over, but long enough
    // row chunks that the per-chunk column partials stay small.
    int64_t rpc;
    if (tile_rows > 0) {
        rpc = std::min<int64_t>(((int64_t)tile_rows + 63) / 64 * 64, L.Nrow);
    } else {
        int64_t target = 768;
        if (const char* tw = std::getenv("CR_TARGET_WGS")) target = std::max(1L, std::atol(tw));
        int64_t chunks = (target + L.strips - 1) / L.strips;
        chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, L.Nrow / 64));
        rpc = (L.Nrow + chunks - 1) / chunks;
        rpc = ((rpc + 63) / 64) * 64;
    }
    rpc = std::min<int64_t>(rpc, cr::kMaxRowsPerChunk);
    // the pass addresses a workgroup's rows (plus the prefetch overrun of
    // three 64-row steps) through 32-bit buffer offsets
    const int64_t row_bytes = L.ld * L.esz;
    const int64_t rpc_cap = ((((int64_t)1 << 32) - 1) / row_bytes - 256) / 64 * 64;
    rpc = std::max<int64_t>(64, std::min(rpc, rpc_cap));
    L.rpc = (int)rpc;
    L.chunks = (int)((L.Nrow + rpc - 1) / rpc);
    L.nb = (int)((L.ld * 32 + cr::kBlock - 1) / cr::kBlock);  // blocks of the O(N n) kernels (32 lanes per point)
    L.nsu = (int)((N + cr::kSuRows - 1) / cr::kSuRows);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.off_theta = take((size_t)L.Nrow * L.ld * L.esz);
    L.off_xp = take(xp_bytes);
    L.off_xiaug = take(xiaug_bytes);
    L.off_cvec = take((size_t)L.ld * 4);
    L.off_ycol = take((size_t)L.Nrow * L.esz);
    L.off_rowpart = take((size_t)L.strips * L.Nrow * L.esz);
    L.off_cpart = take((size_t)L.chunks * L.ld * L.nc * L.esz);
    L.off_kkt = take((size_t)L.strips * L.chunks * 4 * 8);
    L.off_y1p = take((size_t)L.Nrow * 8);
    L.off_y2 = take((size_t)L.Nrow * 8);
    L.off_vy = take((size_t)L.Nrow * 8);
    L.off_y0 = take((size_t)L.Nrow * 8);
    L.off_xi1p = take((size_t)L.Nrow * n * 8);
    L.off_xi2 = take((size_t)L.Nrow * n * 8);
    L.off_vxi = take((size_t)L.Nrow * n * 8);
    L.off_xi0 = take((size_t)L.Nrow * n * 8);
    L.off_y1p1 = take((size_t)L.Nrow * 8);
    L.off_xi1p1 = take((size_t)L.Nrow * n * 8);
    L.off_spart = take((size_t)(L.chunks + L.strips) * 8);
    L.lazy = cr::lazy_fits(precision, L.rpc);
    L.off_blockpart = take((size_t)std::max<int64_t>(L.nb, 1) * 4 * 8);
    L.off_supart = take((size_t)(std::max<int64_t>((int64_t)L.nsu * (n * n + n + 3), L.nb) + 64) * 8);
    L.off_su = take((size_t)(3 * n + 2 + n * n + 8) * 8);
    L.off_oa = take(sizeof(cr::OuterArgs));
    L.off_st = take(sizeof(cr::DevState));
    L.off_sched = take(sizeof(cr::AlccSched));
    L.off_hist = take((size_t)std::max(prm.max_outer, 1) * 16);
    L.nbeta = max_iters + 2 * kGraphIters + 2;
    L.off_beta = take((size_t)L.nbeta * 8);
    L.total = o + 256;  // slack for re-aligning an unaligned base
    return L;
}

bool check_params(const cr_params* p, std::string& msg) {
    if (!p) { msg = "params is NULL"; return false; }
    if (!(p->gamma > 0) || !std::isfinite(p->gamma)) { msg = "gamma must be finite and > 0"; return false; }
    if (!(p->c > 1) || !std::isfinite(p->c)) { msg = "c must be > 1"; return false; }
    if (!(p->kappa > 0)) { msg = "kappa must be > 0"; return false; }
    if (!(p->tau1 > 0)) { msg = "tau1 must be > 0"; return false; }
    if (!(p->step_scale > 0 && p->step_scale <= 1)) { msg = "step_scale must be in (0, 1]"; return false; }
    if (p->max_outer < 1) { msg = "max_outer must be >= 1"; return false; }
    if (p->inner_iters < 0) { msg = "inner_iters must be >= 0"; return false; }
    if (p->inner_iters == 0 && p->max_inner < 1) { msg = "max_inner must be >= 1"; return false; }
    if (!(p->kkt_tol >= 0)) { msg = "kkt_tol must be >= 0"; return false; }
    if (p->tile_rows < 0) { msg = "tile_rows must be >= 0"; return false; }
    if (p->deterministic != 0 && p->deterministic != 1) { msg = "deterministic must be 0 or 1"; return false; }
    if (p->precision != CR_F64 && p->precision != CR_F32 && p->precision != CR_MIXED_BF16) {
        msg = "unknown precision";
        return false;
    }
    return true;
}

// Longest MAPG run of any ALCC iteration: the length of the momentum table.
int64_t max_mapg_iters(const cr_params& p) { return p.inner_iters > 0 ? p.inner_iters : p.max_inner; }

// MAPG iterations per graph replay: a fixed schedule of at most 64 steps per
// ALCC iteration replays exactly that many (no idle iterations), anything
// else replays kGraphIters and lets the device stop the run inside a replay.
int replay_iters(const cr_params& p) {
    return p.inner_iters > 0 && p.inner_iters <= 2 * kGraphIters ? (int)p.inner_iters : kGraphIters;
}

cr_status check_dims(int64_t N, int32_t n, std::string& msg) {
    if (N < 2) { msg = "N must be >= 2"; return CR_ERR_ARG; }
    if (n < 1) { msg = "n must be >= 1"; return CR_ERR_ARG; }
    if (n > CR_MAX_DIM) { msg = "n above CR_MAX_DIM is not supported"; return CR_ERR_UNSUPPORTED; }
    // beyond 2^20 points a theta row no longer fits the pass's 32-bit buffer
    // offsets (and the N^2 theta would need terabytes)
    if (N > (int64_t)1 << 20) { msg = "N above 2^20 is not supported"; return CR_ERR_UNSUPPORTED; }
    return CR_OK;
}

}  // namespace

struct cr_ctx {
    Layout L;
    cr_params p;
    int64_t N;
    int n;
    bool f64;        // FP64 pass partials (CR_F64); FP32 for CR_F32 and CR_MIXED_BF16
    int prec;
    hipStream_t user_stream = nullptr;
    hipStream_t cs = nullptr;            // internal stream (graph capture needs a non-null stream)
    bool owns_cs = true;                 // false: the stream of the batch this context belongs to
    int dev = 0;                         // device current at creation (its pools take the stream and block back)
    hipGraphExec_t graph = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int32_t* pinned_flag = nullptr;      // 2 slots
    cr::DevState* pinned_state = nullptr;
    const double* X = nullptr;
    const double* ybar = nullptr;
    char* ws = nullptr;
    cr::DevState* st = nullptr;
    cr::OuterArgs* oa = nullptr;
    cr::AlccSched* sched = nullptr;      // device ALCC schedule (constants written at init)
    int replay = 32;                     // MAPG iterations per graph replay
    double sigma2_A1 = 0, sigma2_A2 = 0, Bbar = 0, By = 0, Bxi = 0, ybar_inf = 0;
    std::string err;
    cr::DevState last{};
    std::vector<int64_t> hist_inner;   // MAPG iterations of each ALCC iteration of the last run
    std::vector<double> hist_kkt;      // and its KKT measure after the multiplier step
    bool have_kkt = false;
    bool verbose = false;
    bool lazy = false;   // MAPG iterations use lazy passes (single-problem runs whose chunk height allows them)
    const double* shift = nullptr;   // slope shift c (problems in shifted slopes xi = xi' + c; never lazy)
    char* P(size_t off) const { return ws + off; }
    double* D(size_t off) const { return reinterpret_cast<double*>(ws + off); }
};

static cr_status fail(cr_ctx* ctx, cr_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    g_last_error = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, CR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

// Pinned host blocks (a context's flag slots and state read-back, a batch's
// flag) and internal streams are pooled per device for the life of the
// process: each allocation or creation costs tens of microseconds, and a P-APG
// call builds a batch of contexts every time.  Streams go back idle (their
// owners synchronise them first).
constexpr size_t kPinnedBytes = (64 + sizeof(cr::DevState) + 255) / 256 * 256;
struct HostPools {
    std::mutex mu;
    std::vector<std::vector<void*>> pinned;           // per device
    std::vector<std::vector<hipStream_t>> streams;    // per device
};
static HostPools& pools() {
    static HostPools p;
    return p;
}
static int current_device() {
    int d = 0;
    return hipGetDevice(&d) == hipSuccess && d >= 0 ? d : 0;
}
static hipError_t pinned_get(void** out) {
    const int d = current_device();
    {
        HostPools& P = pools();
        std::lock_guard<std::mutex> g(P.mu);
        if ((int)P.pinned.size() > d && !P.pinned[d].empty()) {
            *out = P.pinned[d].back();
            P.pinned[d].pop_back();
            return hipSuccess;
        }
    }
    return hipHostMalloc(out, kPinnedBytes, hipHostMallocDefault);
}
static void pinned_put(void* p, int d) {
    if (!p) return;
    HostPools& P = pools();
    std::lock_guard<std::mutex> g(P.mu);
    if ((int)P.pinned.size() <= d) P.pinned.resize(d + 1);
    P.pinned[d].push_back(p);
}
static hipError_t stream_get(hipStream_t* out) {
    const int d = current_device();
    {
        HostPools& P = pools();
        std::lock_guard<std::mutex> g(P.mu);
        if ((int)P.streams.size() > d && !P.streams[d].empty()) {
            *out = P.streams[d].back();
            P.streams[d].pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
}
static void stream_put(hipStream_t s, int d) {
    if (!s) return;
    HostPools& P = pools();
    std::lock_guard<std::mutex> g(P.mu);
    if ((int)P.streams.size() <= d) P.streams.resize(d + 1);
    P.streams[d].push_back(s);
}

static cr::PassArgs pass_args(cr_ctx* c, int mode, double theta_scale, const int32_t* active) {
    const Layout& L = c->L;
    cr::PassArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.nc = L.nc; a.rows_per_chunk = L.rpc; a.mode = mode;
    a.theta = c->P(L.off_theta); a.xp = c->P(L.off_xp); a.xiaug = c->P(L.off_xiaug); a.ycol = c->P(L.off_ycol);
    a.rowpart = c->P(L.off_rowpart); a.cpart = c->P(L.off_cpart); a.kktpart = c->D(L.off_kkt);
    a.theta_scale = theta_scale; a.active = active;
    a.cvec = (const float*)c->P(L.off_cvec);
    return a;
}

// Gradient pass of a captured MAPG iteration at replay position q (see LazyStep).
static cr::PassArgs lazy_pass_args(cr_ctx* c, int q, int lfix) {
    const Layout& L = c->L;
    cr::PassArgs a = pass_args(c, 0, 0.0, lfix > 0 ? &c->st->one : &c->st->active);
    cr::LazyStep& z = a.lz;
    z.on = 1; z.q = q; z.lfix = lfix; z.n = L.n;
    z.nblk = cr::reduce_blocks(L.N, L.n); z.chunks = L.chunks;
    z.vy = c->D(L.off_vy); z.vxi = c->D(L.off_vxi); z.X = c->X; z.ybar = c->ybar;
    z.y1p[0] = c->D(L.off_y1p); z.y1p[1] = c->D(L.off_y1p1);
    z.xi1p[0] = c->D(L.off_xi1p); z.xi1p[1] = c->D(L.off_xi1p1);
    z.y2 = c->D(L.off_y2); z.xi2 = c->D(L.off_xi2);
    z.beta = c->D(L.off_beta); z.npart = c->D(L.off_blockpart); z.spart = c->D(L.off_spart);
    z.oa = c->oa; z.st = c->st;
    z.shift = c->shift;
    return a;
}

static dim3 pass_grid(const Layout& L) { return dim3((unsigned)L.strips, (unsigned)L.chunks); }

static cr::ReduceArgs reduce_args(cr_ctx* c, int mode, const double* y, const double* xi, double* oy, double* oxi,
                                  double mu) {
    const Layout& L = c->L;
    cr::ReduceArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.n = L.n; a.nc = L.nc; a.strips = L.strips; a.chunks = L.chunks;
    a.mode = mode; a.npass = L.strips * L.chunks;
    a.rowpart = c->P(L.off_rowpart); a.cpart = c->P(L.off_cpart);
    a.X = c->X; a.ybar = c->ybar; a.y = y; a.xi = xi; a.out_y = oy; a.out_xi = oxi;
    a.blockpart = c->D(L.off_blockpart); a.kktpart = c->D(L.off_kkt);
    a.oa = c->oa; a.st = c->st; a.mu = mu; a.gamma = c->p.gamma;
    return a;
}

static cr::PointArgs point_args(cr_ctx* c, const double* y, const double* xi, int write_state) {
    const Layout& L = c->L;
    cr::PointArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.n = L.n; a.kp = L.kp; a.write_state = write_state;
    a.X = c->X; a.y = y; a.xi = xi;
    a.y1p = c->D(L.off_y1p); a.y2 = c->D(L.off_y2); a.xi1p = c->D(L.off_xi1p); a.xi2 = c->D(L.off_xi2);
    a.xiaug = c->P(L.off_xiaug); a.ycol = c->P(L.off_ycol);
    a.cvec = (float*)c->P(L.off_cvec);
    a.shift = c->shift;
    return a;
}

static cr::UpdateArgs update_args(cr_ctx* c) {
    const Layout& L = c->L;
    cr::UpdateArgs a{};
    a.N = L.N; a.ld = L.ld; a.n = L.n; a.kp = L.kp;
    a.X = c->X; a.ybar = c->ybar; a.vy = c->D(L.off_vy); a.vxi = c->D(L.off_vxi); a.beta = c->D(L.off_beta);
    a.y1p = c->D(L.off_y1p); a.y2 = c->D(L.off_y2); a.xi1p = c->D(L.off_xi1p); a.xi2 = c->D(L.off_xi2);
    a.xiaug = c->P(L.off_xiaug); a.ycol = c->P(L.off_ycol);
    a.cvec = (float*)c->P(L.off_cvec);
    a.blockpart = c->D(L.off_blockpart); a.oa = c->oa; a.st = c->st;
    a.shift = c->shift;
    return a;
}

// One MAPG iteration (position q of a replay): pair pass at (y2, xi2), the
// stopping test of the previous iteration plus the gradient step, then
// projection and momentum.
//
// With lazy passes the update kernel is not needed: the next iteration's pass
// completes the step (projection, momentum) for the points it touches.
static hipError_t enqueue_mapg_iteration(cr_ctx* c, int q, hipStream_t s) {
    const Layout& L = c->L;
    cr::PassArgs pa = c->lazy ? lazy_pass_args(c, q, 0) : pass_args(c, 0, 0.0, &c->st->active);
    hipError_t e = cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), s);
    if (e != hipSuccess) return e;
    cr::ReduceArgs ra = reduce_args(c, 0, c->D(L.off_y2), c->D(L.off_xi2), c->D(L.off_vy), c->D(L.off_vxi), 0.0);
    ra.q = q;
    if (c->lazy) ra.spart = c->D(L.off_spart);
    e = cr::launch_reduce(c->f64, ra, s);
    if (e != hipSuccess || c->lazy) return e;
    cr::UpdateArgs ua = update_args(c);
    ua.q = q;
    return cr::launch_update(c->prec, ua, s);
}

// The multiplier step of the device schedule (Fig. 3 step 4 and the KKT
// residuals), enqueued after every replay and gated on st->step_due: the
// finish of the MAPG run, the point (y_k, xi_k), the multiplier pass, its KKT
// reduction, then k_alcc_step (record, tests, next ALCC iteration).
static hipError_t enqueue_device_step(cr_ctx* c, hipStream_t s) {
    const Layout& L = c->L;
    const int32_t* gate = &c->st->step_due;
    hipError_t e = hipSuccess;
    int nblk = cr::reduce_blocks(c->N, c->n);
    if (c->lazy) {
        if ((e = cr::launch_mapg_finish(lazy_pass_args(c, 0, 0).lz, L.N, s, gate)) != hipSuccess) return e;
        nblk = 0;
    }
    if ((e = cr::launch_mapg_end(c->D(L.off_blockpart), nblk, -1, c->st, s, gate)) != hipSuccess) return e;
    cr::PointArgs pt = point_args(c, c->D(L.off_y1p), c->D(L.off_xi1p), 1);
    pt.gate = gate;
    if ((e = cr::launch_set_point(c->prec, pt, s)) != hipSuccess) return e;
    cr::PassArgs pa = pass_args(c, 1, 0.0, gate);
    pa.theta_scale_p = &c->oa->theta_scale;
    pa.check_first = 1;                          // the gate is closed in most replays
    if ((e = cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), s)) != hipSuccess) return e;
    cr::ReduceArgs ra = reduce_args(c, 2, c->D(L.off_y1p), c->D(L.off_xi1p), nullptr, nullptr, 0.0);
    ra.gate = gate;
    ra.mu_dev = 1;
    ra.check_first = 1;
    if ((e = cr::launch_reduce(c->f64, ra, s)) != hipSuccess) return e;
    return cr::launch_alcc_step(c->sched, c->st, c->oa, s);
}

// One graph replay: c->replay MAPG iterations, the end-of-replay gate of the
// device schedule, and the gated multiplier step.
static cr_status build_graph(cr_ctx* c) {
    if (c->graph) return CR_OK;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int q = 0; q < c->replay && e == hipSuccess; ++q) e = enqueue_mapg_iteration(c, q, c->cs);
    if (e == hipSuccess) e = cr::launch_alcc_gate(c->sched, c->st, c->oa, c->replay, c->cs);
    if (e == hipSuccess) e = enqueue_device_step(c, c->cs);
    hipError_t e2 = hipStreamEndCapture(c->cs, &g);
    if (e != hipSuccess) return fail(c, CR_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(c, CR_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { c->graph = nullptr; return fail(c, CR_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e)); }
    return CR_OK;
}

// ALCC schedule of one problem (Fig. 3 steps 1-2 and 5-6).
struct Schedule {
    double mu, tau, ay, axi;
    int k = 0;
    bool done = false, converged = false;
    int64_t total_inner = 0;
    cr::DevState last{};
    void start(const cr_ctx* c) {
        const cr_params& p = c->p;
        mu = p.mu1 > 0 ? p.mu1 : 1.0 / (2.0 * (double)c->N);
        tau = p.tau1;
        ay = p.alpha_y1 > 0 ? p.alpha_y1 : 1e-2 * c->Bbar;
        axi = p.alpha_xi1 > 0 ? p.alpha_xi1 : 1e-2 * c->Bbar;
        k = 0;
        done = converged = false;
        total_inner = 0;
        last = cr::DevState{};
    }
    // Arguments of ALCC iteration k + 1: L^y, L^xi, l^max and the steps.
    cr::OuterArgs next(const cr_ctx* c) {
        const cr_params& p = c->p;
        ++k;
        const double Ly = p.Ly_override > 0 ? p.Ly_override : 1.0 / mu + c->sigma2_A1;
        const double Lxi = p.Lxi_override > 0 ? p.Lxi_override : p.gamma / mu + c->sigma2_A2;
        int64_t lmax;
        if (p.inner_iters > 0) {
            lmax = p.inner_iters;
        } else {
            const double f = std::ceil(4.0 * std::sqrt((Ly * c->By * c->By + Lxi * c->Bxi * c->Bxi) / tau));
            lmax = (int64_t)std::max(1.0, std::min(f, (double)p.max_inner));
        }
        cr::OuterArgs oa{};
        oa.mu = mu; oa.gamma = p.gamma; oa.sy = p.step_scale / Ly; oa.sxi = p.step_scale / Lxi;
        oa.alpha_y = ay; oa.alpha_xi = axi; oa.By = c->By; oa.Bxi = c->Bxi;
        oa.theta_scale = 1.0 / p.c; oa.lmax = lmax; oa.adaptive = p.inner_iters > 0 ? 0 : 1; oa.skip = 0;
        return oa;
    }
    double mu_next(const cr_ctx* c) const { return c->p.c * mu; }
    // after the multiplier step of iteration k
    void advance(const cr_ctx* c) {
        const cr_params& p = c->p;
        const double decay = std::pow(p.c * std::pow((double)k, 1.0 + p.kappa), 2.0);
        mu = p.c * mu;
        tau /= decay;
        ay /= decay;
        axi /= decay;
    }
};

// The multiplier step at the MAPG output (y_k, xi_k) of one problem, which also
// restarts MAPG there, followed by the KKT residuals; then a state read-back.
// nblk: number of blocks of the update kernel that wrote the last step's norms.
static hipError_t enqueue_multiplier_step(cr_ctx* c, double mu, double mu_next, int64_t launched, int nblk,
                                          hipStream_t cs) {
    const Layout& L = c->L;
    hipError_t e = hipSuccess;
    if (c->lazy) {
        // the run's last iterate into y1p / xi1p; no update-kernel norms to gather
        e = cr::launch_mapg_finish(lazy_pass_args(c, 0, 0).lz, L.N, cs);
        if (e != hipSuccess) return e;
        nblk = 0;
    }
    e = cr::launch_mapg_end(c->D(L.off_blockpart), nblk, launched, c->st, cs);
    if (e != hipSuccess) return e;
    cr::PointArgs pt = point_args(c, c->D(L.off_y1p), c->D(L.off_xi1p), 1);
    if ((e = cr::launch_set_point(c->prec, pt, cs)) != hipSuccess) return e;
    cr::PassArgs pa = pass_args(c, 1, mu / mu_next, &c->st->one);
    if ((e = cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), cs)) != hipSuccess) return e;
    cr::ReduceArgs ra = reduce_args(c, 2, c->D(L.off_y1p), c->D(L.off_xi1p), nullptr, nullptr, mu);
    if ((e = cr::launch_reduce(c->f64, ra, cs)) != hipSuccess) return e;
    return hipMemcpyAsync(c->pinned_state, c->st, sizeof(cr::DevState), hipMemcpyDeviceToHost, cs);
}

extern "C" {

cr_status cr_params_default(cr_params* p) {
    if (!p) return fail(nullptr, CR_ERR_ARG, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1e-3;
    p->mu1 = 0.0;
    p->c = 4.0;
    p->kappa = 0.1;
    p->tau1 = 1.0;
    p->alpha_y1 = 0.0;
    p->alpha_xi1 = 0.0;
    p->step_scale = 0.5;
    p->kkt_tol = 1e-4;
    p->max_outer = 30;
    p->inner_iters = 0;
    p->max_inner = 20000;
    p->precision = CR_F64;
    return CR_OK;
}

const char* cr_status_string(cr_status s) {
    switch (s) {
        case CR_OK: return "CR_OK";
        case CR_ERR_ARG: return "CR_ERR_ARG";
        case CR_ERR_NOMEM: return "CR_ERR_NOMEM";
        case CR_ERR_HIP: return "CR_ERR_HIP";
        case CR_ERR_NONFINITE: return "CR_ERR_NONFINITE";
        case CR_NOT_CONVERGED: return "CR_NOT_CONVERGED";
        case CR_ERR_STATE: return "CR_ERR_STATE";
        case CR_ERR_UNSUPPORTED: return "CR_ERR_UNSUPPORTED";
        default: return "CR_UNKNOWN_STATUS";
    }
}

const char* cr_last_error(const cr_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

cr_status cr_workspace_bytes(int64_t N, int32_t n, const cr_params* params, size_t* bytes) {
    std::string msg;
    if (!bytes) return fail(nullptr, CR_ERR_ARG, "bytes is NULL");
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!check_params(params, msg)) return fail(nullptr, CR_ERR_ARG, msg);
    *bytes = make_layout(N, n, *params, params->tile_rows).total;
    return CR_OK;
}

cr_status cr_pass_layout(int64_t N, int32_t n, const cr_params* params, int64_t* out) {
    std::string msg;
    if (!out) return fail(nullptr, CR_ERR_ARG, "out is NULL");
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!check_params(params, msg)) return fail(nullptr, CR_ERR_ARG, msg);
    const Layout L = make_layout(N, n, *params, params->tile_rows);
    out[0] = L.Nrow;
    out[1] = L.ld;
    out[2] = L.rpc;
    out[3] = L.chunks;
    out[4] = L.strips;
    out[5] = L.lazy && !params->deterministic ? 1 : 0;
    return CR_OK;
}

// shared_cs non-null: the context runs on that stream (a batch's problems) and
// neither creates nor destroys one.
static cr_status ctx_init(cr_ctx** out, int64_t N, int32_t n, const cr_params* params, const void* X_dev,
                          const void* ybar_dev, void* workspace_dev, size_t ws_bytes, void* stream,
                          hipStream_t shared_cs) {
    std::string msg;
    if (!out) return fail(nullptr, CR_ERR_ARG, "out is NULL");
    *out = nullptr;
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!check_params(params, msg)) return fail(nullptr, CR_ERR_ARG, msg);
    if (!X_dev || !ybar_dev || !workspace_dev) return fail(nullptr, CR_ERR_ARG, "X, ybar and workspace must be non-NULL");
    Layout L = make_layout(N, n, *params, params->tile_rows);
    if (ws_bytes < L.total) return fail(nullptr, CR_ERR_NOMEM, "workspace smaller than cr_workspace_bytes()");

    cr_ctx* c = new (std::nothrow) cr_ctx();
    if (!c) return fail(nullptr, CR_ERR_NOMEM, "host allocation failed");
    c->L = L;
    c->p = *params;
    c->N = N;
    c->n = n;
    c->f64 = params->precision == CR_F64;
    c->prec = params->precision;
    c->lazy = L.lazy && !params->deterministic;
    c->user_stream = (hipStream_t)stream;
    {
        const char* v = std::getenv("CR_VERBOSE");
        c->verbose = v && v[0] && v[0] != '0';
    }
    c->X = (const double*)X_dev;
    c->ybar = (const double*)ybar_dev;
    c->ws = (char*)align256((size_t)workspace_dev);
    c->st = reinterpret_cast<cr::DevState*>(c->P(L.off_st));
    c->oa = reinterpret_cast<cr::OuterArgs*>(c->P(L.off_oa));
    c->sched = reinterpret_cast<cr::AlccSched*>(c->P(L.off_sched));
    c->replay = replay_iters(*params);
    auto bad = [&](cr_status st) { cr_destroy(c); return st; };
    c->dev = current_device();
    hipError_t e = hipSuccess;
    if (shared_cs) {
        c->cs = shared_cs;
        c->owns_cs = false;
    } else {
        e = stream_get(&c->cs);
    }
    if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, std::string("stream: ") + hipGetErrorString(e)); return bad(CR_ERR_HIP); }
    for (int q = 0; q < 2; ++q) {
        e = hipEventCreateWithFlags(&c->ev[q], hipEventDisableTiming);
        if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, "event create"); return bad(CR_ERR_HIP); }
    }
    // one pinned block: the two flag slots, then the state read-back
    e = pinned_get((void**)&c->pinned_flag);
    if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, "pinned host allocation"); return bad(CR_ERR_HIP); }
    c->pinned_state = reinterpret_cast<cr::DevState*>(reinterpret_cast<char*>(c->pinned_flag) + 64);

    // order after the caller's prior work on its stream
    hipEvent_t ue = c->ev[0];
    if ((e = hipEventRecord(ue, c->user_stream)) != hipSuccess || (e = hipStreamWaitEvent(c->cs, ue, 0)) != hipSuccess) {
        fail(nullptr, CR_ERR_HIP, std::string("stream join: ") + hipGetErrorString(e));
        return bad(CR_ERR_HIP);
    }
    hipStream_t cs = c->cs;
    e = cr::launch_zero(c->P(L.off_st), (sizeof(cr::DevState) + 15) / 16 * 16, cs);
    if (e == hipSuccess) e = cr::launch_zero(c->P(L.off_theta), (size_t)L.Nrow * L.ld * L.esz, cs);
    if (e == hipSuccess) e = cr::launch_zero(c->P(L.off_y0), (size_t)L.Nrow * 8, cs);
    if (e == hipSuccess) e = cr::launch_zero(c->P(L.off_xi0), (size_t)L.Nrow * n * 8, cs);
    if (e == hipSuccess)
        e = cr::launch_setup(c->X, c->ybar, N, n, params->gamma, c->D(L.off_su), c->D(L.off_supart), c->D(L.off_y0),
                             c->D(L.off_xi0), c->st, cs);
    if (e == hipSuccess) e = cr::launch_prep_xp(c->prec, c->X, N, n, L.Nrow, L.ks, L.qp, c->P(L.off_xp), cs);
    if (e == hipSuccess) {
        // momentum weights of Fig. 4: t_1 = 1, t_{l+1} = (1 + sqrt(1 + 4 t_l^2)) / 2,
        // beta_l = (t_l - 1) / t_{l+1}; entry 0 is unused.  The copy is from
        // pageable memory: the runtime stages it before the call returns.
        std::vector<double> hb((size_t)L.nbeta);
        double t = 1.0;
        hb[0] = 0.0;
        for (int64_t l = 1; l < L.nbeta; ++l) {
            const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
            hb[l] = (t - 1.0) / tn;
            t = tn;
        }
        e = hipMemcpyAsync(c->P(L.off_beta), hb.data(), (size_t)L.nbeta * 8, hipMemcpyHostToDevice, cs);
    }
    {
        // constants of the device ALCC schedule (the state is set by k_alcc_start)
        cr::AlccSched sc{};
        sc.mu1 = params->mu1 > 0 ? params->mu1 : 1.0 / (2.0 * (double)N);
        sc.c = params->c; sc.kappa = params->kappa; sc.tau1 = params->tau1;
        sc.ay1 = params->alpha_y1; sc.axi1 = params->alpha_xi1; sc.gamma = params->gamma;
        sc.step_scale = params->step_scale; sc.kkt_tol = params->kkt_tol;
        sc.Ly_ovr = params->Ly_override; sc.Lxi_ovr = params->Lxi_override;
        sc.By_ovr = params->By_override; sc.Bxi_ovr = params->Bxi_override;
        sc.sigma2_A1 = 2.0 * (double)N;
        sc.inner_iters = params->inner_iters; sc.max_inner = params->max_inner; sc.max_outer = params->max_outer;
        sc.hist_inner = reinterpret_cast<int64_t*>(c->P(L.off_hist));
        sc.hist_kkt = reinterpret_cast<double*>(c->P(L.off_hist) + (size_t)std::max(params->max_outer, 1) * 8);
        sc.phase = 2;
        // staged from pageable memory; complete at the stream synchronisation below
        if (e == hipSuccess) e = hipMemcpyAsync(c->sched, &sc, sizeof(sc), hipMemcpyHostToDevice, cs);
    }
    if (e == hipSuccess) {
        cr::PointArgs pa = point_args(c, c->D(L.off_y0), c->D(L.off_xi0), 1);
        e = cr::launch_set_point(c->prec, pa, cs);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(c->pinned_state, c->st, sizeof(cr::DevState), hipMemcpyDeviceToHost, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, std::string("set-up: ") + hipGetErrorString(e)); return bad(CR_ERR_HIP); }
    const cr::DevState& h = *c->pinned_state;
    if (h.nonfinite) { fail(nullptr, CR_ERR_NONFINITE, "X or ybar holds NaN or Inf"); return bad(CR_ERR_NONFINITE); }
    c->sigma2_A1 = 2.0 * (double)N;
    c->sigma2_A2 = h.sigma2_A2;
    c->Bbar = h.Bbar;
    c->By = params->By_override > 0 ? params->By_override : h.Bbar;
    c->Bxi = params->Bxi_override > 0 ? params->Bxi_override : h.Bbar / std::sqrt(params->gamma);
    c->ybar_inf = h.ybar_inf;
    if (!std::isfinite(c->sigma2_A2) || !std::isfinite(c->Bbar)) {
        fail(nullptr, CR_ERR_NONFINITE, "non-finite problem constants");
        return bad(CR_ERR_NONFINITE);
    }
    *out = c;
    return CR_OK;
}

cr_status cr_init(cr_ctx** out, int64_t N, int32_t n, const cr_params* params, const void* X_dev,
                  const void* ybar_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
    return ctx_init(out, N, n, params, X_dev, ybar_dev, workspace_dev, ws_bytes, stream, nullptr);
}

cr_status cr_destroy(cr_ctx* c) {
    if (!c) return CR_OK;
    if (c->cs) hipStreamSynchronize(c->cs);
    if (c->graph) hipGraphExecDestroy(c->graph);
    for (int q = 0; q < 2; ++q)
        if (c->ev[q]) hipEventDestroy(c->ev[q]);
    pinned_put(c->pinned_flag, c->dev);                // the state read-back shares its block
    if (c->owns_cs) stream_put(c->cs, c->dev);
    delete c;
    return CR_OK;
}

cr_status cr_pairwise_step(cr_ctx* c, int32_t mode, const void* y_dev, const void* xi_dev, void* gy_dev,
                           void* gxi_dev, double mu, double mu_next) {
    if (!c) return fail(nullptr, CR_ERR_ARG, "ctx is NULL");
    if (!y_dev || !xi_dev || !gy_dev || !gxi_dev) return fail(c, CR_ERR_ARG, "y, xi, gy and gxi must be non-NULL");
    if (mode != CR_GRAD && mode != CR_THETA_UPDATE) return fail(c, CR_ERR_ARG, "unknown mode");
    if (!(mu > 0) || !std::isfinite(mu)) return fail(c, CR_ERR_ARG, "mu must be > 0");
    if (mode == CR_THETA_UPDATE && (!(mu_next > 0) || !std::isfinite(mu_next)))
        return fail(c, CR_ERR_ARG, "mu_next must be > 0");
    const Layout& L = c->L;
    hipStream_t s = c->user_stream;
    cr::PointArgs pt = point_args(c, (const double*)y_dev, (const double*)xi_dev, 0);
    HIPCHK(c, cr::launch_set_point(c->prec, pt, s));
    const double scale = mode == CR_THETA_UPDATE ? mu / mu_next : 0.0;
    cr::PassArgs pa = pass_args(c, mode == CR_THETA_UPDATE ? 1 : 0, scale, &c->st->one);
    HIPCHK(c, cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), s));
    cr::ReduceArgs ra = reduce_args(c, mode == CR_THETA_UPDATE ? 2 : 1, (const double*)y_dev, (const double*)xi_dev,
                                    (double*)gy_dev, (double*)gxi_dev, mu);
    HIPCHK(c, cr::launch_reduce(c->f64, ra, s));
    if (mode == CR_THETA_UPDATE) c->have_kkt = true;
    return CR_OK;
}

static void fill_info(cr_ctx* c, const cr::DevState& h, cr_info* info) {
    info->objective = h.obj;
    const double scale = 1.0 + h.ybar_inf;
    info->stat_y = h.stat_y;
    info->stat_xi = h.stat_xi;
    info->infeas = h.infeas;
    info->compl_ = h.compl_;
    info->kkt = std::max(std::max(h.stat_y, h.stat_xi), std::max(h.infeas, h.compl_)) / scale;
    const double np = (double)c->N * (double)(c->N - 1);
    info->infeas_norm = std::sqrt(h.infeas_sq) / std::sqrt(np);
    info->gap_norm = h.gap / np;
    info->sigma2_A1 = c->sigma2_A1;
    info->sigma2_A2 = h.sigma2_A2;
    info->Bbar_y = c->p.By_override > 0 ? c->p.By_override : h.Bbar;
    info->Bbar_xi = c->p.Bxi_override > 0 ? c->p.Bxi_override : h.Bbar / std::sqrt(c->p.gamma);
}

cr_status cr_get_info(cr_ctx* c, cr_info* info) {
    if (!c || !info) return fail(c, CR_ERR_ARG, "ctx and info must be non-NULL");
    HIPCHK(c, hipStreamSynchronize(c->user_stream));
    HIPCHK(c, hipStreamSynchronize(c->cs));
    HIPCHK(c, hipMemcpy(c->pinned_state, c->st, sizeof(cr::DevState), hipMemcpyDeviceToHost));
    std::memset(info, 0, sizeof(*info));
    fill_info(c, *c->pinned_state, info);
    return CR_OK;
}

cr_status cr_get_theta(cr_ctx* c, void* theta_dev) {
    if (!c || !theta_dev) return fail(c, CR_ERR_ARG, "ctx and theta must be non-NULL");
    HIPCHK(c, cr::launch_theta_export(c->f64, c->P(c->L.off_theta), c->N, c->L.ld, (double*)theta_dev, c->user_stream));
    return CR_OK;
}

cr_status cr_set_theta(cr_ctx* c, const void* theta_dev) {
    if (!c || !theta_dev) return fail(c, CR_ERR_ARG, "ctx and theta must be non-NULL");
    HIPCHK(c, cr::launch_theta_import(c->f64, (const double*)theta_dev, c->N, c->L.Nrow, c->L.ld, c->P(c->L.off_theta),
                                      c->user_stream));
    return CR_OK;
}

cr_status cr_get_start(cr_ctx* c, void* y_dev, void* xi_dev) {
    if (!c || !y_dev || !xi_dev) return fail(c, CR_ERR_ARG, "ctx, y and xi must be non-NULL");
    HIPCHK(c, hipMemcpyAsync(y_dev, c->D(c->L.off_y0), (size_t)c->N * 8, hipMemcpyDeviceToDevice, c->user_stream));
    HIPCHK(c, hipMemcpyAsync(xi_dev, c->D(c->L.off_xi0), (size_t)c->N * c->n * 8, hipMemcpyDeviceToDevice,
                             c->user_stream));
    return CR_OK;
}

// Host side of a device-scheduled run: enqueue graph replays until the
// schedule is done.  A fixed schedule needs exactly max_outer x ceil(l / replay)
// replays, all enqueued at once; otherwise the phase flag is polled one replay
// behind (the replay in between finds nothing to do).  No read-back between
// ALCC iterations either way.
static cr_status replay_until_done(cr_ctx* c) {
    const cr_params& p = c->p;
    hipStream_t cs = c->cs;
    if (p.inner_iters > 0) {
        const int64_t per = (p.inner_iters + c->replay - 1) / c->replay;
        for (int64_t r = 0; r < per * p.max_outer; ++r) HIPCHK(c, hipGraphLaunch(c->graph, cs));
        return CR_OK;
    }
    // at most max_inner + one replay of MAPG iterations per ALCC iteration
    const int64_t cap = (int64_t)p.max_outer * ((p.max_inner + c->replay - 1) / c->replay + 1) + 2;
    int slot = 0, pending = -1;
    for (int64_t r = 0; r < cap; ++r) {
        HIPCHK(c, hipGraphLaunch(c->graph, cs));
        HIPCHK(c, hipMemcpyAsync(c->pinned_flag + slot, &c->sched->phase, 4, hipMemcpyDeviceToHost, cs));
        HIPCHK(c, hipEventRecord(c->ev[slot], cs));
        if (pending >= 0) {
            HIPCHK(c, hipEventSynchronize(c->ev[pending]));
            if (c->pinned_flag[pending] == 2) return CR_OK;
        }
        pending = slot;
        slot ^= 1;
    }
    return CR_OK;
}

cr_status cr_run(cr_ctx* c, void* y_dev, void* xi_dev, cr_info* info) {
    if (!c) return fail(nullptr, CR_ERR_ARG, "ctx is NULL");
    if (!y_dev || !xi_dev) return fail(c, CR_ERR_ARG, "y and xi must be non-NULL");
    const Layout& L = c->L;
    const cr_params& p = c->p;
    hipStream_t cs = c->cs;
    HIPCHK(c, hipEventRecord(c->ev[0], c->user_stream));
    HIPCHK(c, hipStreamWaitEvent(cs, c->ev[0], 0));
    cr_status bs = build_graph(c);
    if (bs != CR_OK) return bs;

    const auto t0 = std::chrono::steady_clock::now();
    // theta_1 = 0 and (y_0, xi_0) = the affine fit; ALCC iteration 1 begins on the device
    HIPCHK(c, cr::launch_zero(c->P(L.off_theta), (size_t)L.Nrow * L.ld * L.esz, cs));
    cr::PointArgs start = point_args(c, c->D(L.off_y0), c->D(L.off_xi0), 1);
    HIPCHK(c, cr::launch_set_point(c->prec, start, cs));
    HIPCHK(c, cr::launch_alcc_start(c->sched, c->oa, c->st, cs));
    cr_status rs = replay_until_done(c);
    if (rs != CR_OK) return rs;

    const int64_t N = c->N;
    HIPCHK(c, hipMemcpyAsync(y_dev, c->D(L.off_y1p), (size_t)N * 8, hipMemcpyDeviceToDevice, cs));
    HIPCHK(c, hipMemcpyAsync(xi_dev, c->D(L.off_xi1p), (size_t)N * c->n * 8, hipMemcpyDeviceToDevice, cs));
    cr::AlccSched sc{};
    HIPCHK(c, hipMemcpyAsync(c->pinned_state, c->st, sizeof(cr::DevState), hipMemcpyDeviceToHost, cs));
    HIPCHK(c, hipStreamSynchronize(cs));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    HIPCHK(c, hipMemcpy(&sc, c->sched, sizeof(sc), hipMemcpyDeviceToHost));
    const int outer = std::min(sc.k, p.max_outer);
    c->hist_inner.assign((size_t)outer, 0);
    c->hist_kkt.assign((size_t)outer, 0.0);
    if (outer > 0) {
        HIPCHK(c, hipMemcpy(c->hist_inner.data(), sc.hist_inner, (size_t)outer * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(c->hist_kkt.data(), sc.hist_kkt, (size_t)outer * 8, hipMemcpyDeviceToHost));
    }
    const cr::DevState h = *c->pinned_state;
    c->have_kkt = true;
    if (c->verbose)
        for (int k = 0; k < outer; ++k)
            std::fprintf(stderr, "[cr] outer %d inner %lld kkt %.3e\n", k + 1, (long long)c->hist_inner[k],
                         c->hist_kkt[k]);
    cr_status result = CR_OK;
    if (sc.nonfinite) result = CR_ERR_NONFINITE;
    else if (sc.phase != 2) result = CR_ERR_STATE;
    else if (p.inner_iters == 0 && !sc.converged) result = CR_NOT_CONVERGED;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        fill_info(c, h, info);
        info->outer_iters = outer;
        info->inner_iters = sc.total_inner;
        info->seconds = secs;
        info->pair_updates = (double)N * (double)(N - 1) * (double)sc.total_inner;
        info->status = result;
    }
    if (result == CR_ERR_NONFINITE) return fail(c, result, "non-finite iterate");
    if (result == CR_ERR_STATE) return fail(c, result, "the schedule did not finish within its replay cap");
    return result;
}

cr_status cr_get_outer_history(cr_ctx* c, int32_t cap, int64_t* inner_iters, double* kkt, int32_t* count) {
    if (!c || !count) return fail(c, CR_ERR_ARG, "ctx and count must be non-NULL");
    if (cap < 0 || (cap > 0 && (!inner_iters || !kkt))) return fail(c, CR_ERR_ARG, "bad capacity or NULL arrays");
    const int32_t m = (int32_t)c->hist_inner.size();
    *count = m;
    for (int32_t k = 0; k < std::min(cap, m); ++k) {
        inner_iters[k] = c->hist_inner[k];
        kkt[k] = c->hist_kkt[k];
    }
    return CR_OK;
}

cr_status cr_time_pass(cr_ctx* c, int32_t mode, int32_t reps, double* avg_ms) {
    if (!c || !avg_ms) return fail(c, CR_ERR_ARG, "ctx and avg_ms must be non-NULL");
    if (reps < 1 || mode != CR_GRAD) return fail(c, CR_ERR_ARG, "reps must be >= 1 and mode CR_GRAD");
    const Layout& L = c->L;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    cr::PassArgs pa = pass_args(c, 0, 0.0, &c->st->one);
    hipError_t e = hipSuccess;
    if (c->lazy) {
        // The kernel a MAPG run launches: a lazy pass at iteration 2.  Its inputs
        // come from one step at the start point (pass, reduce); the timed passes
        // rewrite the same state (y1_1, y2_2) each time.
        Schedule sch;
        sch.start(c);
        const cr::OuterArgs oa = sch.next(c);
        e = cr::launch_begin_outer(oa, c->oa, c->st, c->cs);
        cr::PointArgs pt = point_args(c, c->D(L.off_y0), c->D(L.off_xi0), 1);
        if (e == hipSuccess) e = cr::launch_set_point(c->prec, pt, c->cs);
        if (e == hipSuccess) e = cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), c->cs);
        cr::ReduceArgs ra = reduce_args(c, 0, c->D(L.off_y2), c->D(L.off_xi2), c->D(L.off_vy), c->D(L.off_vxi), 0.0);
        ra.spart = c->D(L.off_spart);
        if (e == hipSuccess) e = cr::launch_reduce(c->f64, ra, c->cs);
        pa = lazy_pass_args(c, 0, 2);
        if (e != hipSuccess) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return fail(c, CR_ERR_HIP, std::string("time pass set-up: ") + hipGetErrorString(e));
        }
    }
    e = hipEventRecord(e0, c->cs);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = cr::launch_pair_pass(c->prec, c->n, pa, pass_grid(L), c->cs);
    if (e == hipSuccess) e = hipEventRecord(e1, c->cs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return fail(c, CR_ERR_HIP, std::string("time pass: ") + hipGetErrorString(e));
    *avg_ms = (double)ms / reps;
    return CR_OK;
}

cr_status cr_solve(const void* X_dev, const void* ybar_dev, int64_t N, int32_t n, const cr_params* params,
                   void* y_dev, void* xi_dev, void* workspace_dev, size_t ws_bytes, cr_info* info, void* stream) {
    if (!y_dev || !xi_dev) return fail(nullptr, CR_ERR_ARG, "y and xi must be non-NULL");
    cr_ctx* c = nullptr;
    cr_status s = cr_init(&c, N, n, params, X_dev, ybar_dev, workspace_dev, ws_bytes, stream);
    if (s != CR_OK) return s;
    s = cr_run(c, y_dev, xi_dev, info);
    if (s != CR_OK && s != CR_NOT_CONVERGED) g_last_error = c->err;
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
        hipEventRecord(done, c->cs);
        hipStreamWaitEvent((hipStream_t)stream, done, 0);
        hipEventDestroy(done);
    }
    cr_destroy(c);
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: many independent problems advanced in lockstep.  Each problem
// owns a single-problem context in a slice of the batch workspace; one MAPG
// iteration of every problem is [persistent pass per operand class,
// batched reduce, batched update], captured kGraphIters times in one graph.
// Converged problems are frozen (their activity flag stays 0).
// ---------------------------------------------------------------------------
namespace {

struct BatchItemH { int32_t p, strip, chunk, pad; };

struct BatchPlan {
    std::vector<Layout> L;
    std::vector<size_t> off;     // sub-workspace offsets
    size_t hdr = 0, total = 0;
    // O(N n) kernels of the batch run G = 16 or 32 lanes per point by each
    // problem's own n (as a problem solved alone does): its blocks sit in the
    // block table's segment for that G (16 first), nblk blocks per problem.
    int nblocks = 0;
    int gseg_start[2] = {0, 0}, gseg_count[2] = {0, 0};
    std::vector<int32_t> nblk;
    std::vector<int> ks_classes;
    std::vector<BatchItemH> items;          // grouped by class
    std::vector<int> class_off, class_cnt;
    size_t off_pass, off_red, off_upd, off_nstrips, off_blocks, off_nblk, off_sts, off_any, off_items;
    // device-schedule tables: schedules, outer arguments, update block records,
    // and the multiplier step's pass / reduce / set-point arguments
    size_t off_scheds, off_oas, off_bparts, off_pass1, off_red2, off_pt;
    // lazy batches: the gradient-pass table for cr_batch_time_pass (iteration 2,
    // every problem active) and a table of zero block counts (no update-kernel
    // records at the end of a run)
    size_t off_pass_time, off_nblk0;
    bool lazy = false;           // MAPG iterations use lazy passes (every problem's chunk height allows them)
};

cr_status check_batch(const cr_problem* probs, int32_t P, const cr_params* params, std::string& msg) {
    if (!probs || P < 1) { msg = "probs must be non-NULL and P >= 1"; return CR_ERR_ARG; }
    if (!check_params(params, msg)) return CR_ERR_ARG;
    if (params->precision == CR_MIXED_BF16) { msg = "the batched form supports CR_F64 and CR_F32"; return CR_ERR_UNSUPPORTED; }
    for (int p = 0; p < P; ++p) {
        cr_status s = check_dims(probs[p].N, probs[p].n, msg);
        if (s != CR_OK) { msg = "problem " + std::to_string(p) + ": " + msg; return s; }
        if (probs[p].tile_rows < 0) { msg = "problem " + std::to_string(p) + ": tile_rows must be >= 0"; return CR_ERR_ARG; }
    }
    return CR_OK;
}

// Largest problem of a batch that runs lazy passes (see plan_batch).
constexpr int64_t kBatchLazyMaxN = 2048;

// Lanes per point of a problem's O(N n) kernels (lane k < n: xi_k, lane n: y).
int batch_group(int n) { return n + 1 <= 16 ? 16 : 32; }

BatchPlan plan_batch(const cr_problem* probs, int32_t P, const cr_params* params) {
    BatchPlan B;
    for (int p = 0; p < P; ++p) {
        const int tr = probs[p].tile_rows > 0 ? probs[p].tile_rows : params->tile_rows;
        B.L.push_back(make_layout(probs[p].N, probs[p].n, *params, tr));
        const int G = batch_group(probs[p].n);
        const int nb = (int)((probs[p].N * G + cr::kBlock - 1) / cr::kBlock);
        B.nblk.push_back(nb);
        B.nblocks += nb;
        B.gseg_count[G == 16 ? 0 : 1] += nb;
        const int ks = cr::ks_of(probs[p].n);
        if (std::find(B.ks_classes.begin(), B.ks_classes.end(), ks) == B.ks_classes.end()) B.ks_classes.push_back(ks);
    }
    // Lazy passes save the update kernel but add a per-item set-up whose cost
    // grows with the problem; measured on the MI355X: 3.83 against 4.07 ms per
    // P-APG iteration with 1024-point blocks, 2.20 against 2.05 ms per MAPG
    // iteration of 64 problems of 500 to 8000 points.
    B.gseg_start[1] = B.gseg_count[0];
    B.lazy = !params->deterministic;
    for (int p = 0; p < P; ++p) B.lazy = B.lazy && B.L[p].lazy && probs[p].N <= kBatchLazyMaxN;
    std::sort(B.ks_classes.begin(), B.ks_classes.end());
    for (int ks : B.ks_classes) {
        B.class_off.push_back((int)B.items.size());
        for (int p = 0; p < P; ++p) {
            if (cr::ks_of(probs[p].n) != ks) continue;
            for (int h = 0; h < B.L[p].chunks; ++h)
                for (int st = 0; st < B.L[p].strips; ++st) B.items.push_back(BatchItemH{p, st, h, 0});
        }
        B.class_cnt.push_back((int)B.items.size() - B.class_off.back());
    }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    B.off_pass = take((size_t)P * sizeof(cr::PassArgs));
    B.off_red = take((size_t)P * sizeof(cr::ReduceArgs));
    B.off_upd = take((size_t)P * sizeof(cr::UpdateArgs));
    B.off_nstrips = take((size_t)P * 4);
    B.off_blocks = take((size_t)B.nblocks * 8);
    B.off_nblk = take((size_t)P * 4);
    B.off_sts = take((size_t)P * sizeof(void*));
    B.off_any = take(64);
    B.off_items = take(B.items.size() * sizeof(BatchItemH));
    B.off_scheds = take((size_t)P * sizeof(void*));
    B.off_oas = take((size_t)P * sizeof(void*));
    B.off_bparts = take((size_t)P * sizeof(void*));
    B.off_pass1 = take((size_t)P * sizeof(cr::PassArgs));
    B.off_red2 = take((size_t)P * sizeof(cr::ReduceArgs));
    B.off_pt = take((size_t)P * sizeof(cr::PointArgs));
    B.off_pass_time = take((size_t)P * sizeof(cr::PassArgs));
    B.off_nblk0 = take((size_t)P * 4);
    B.hdr = o;
    for (int p = 0; p < P; ++p) B.off.push_back(take(B.L[p].total));
    B.total = o + 256;
    return B;
}

}  // namespace

struct cr_batch {
    int P = 0;
    cr_params p{};
    BatchPlan plan;
    std::vector<cr_problem> probs;
    std::vector<cr_ctx*> sub;
    hipStream_t user_stream = nullptr, cs = nullptr;
    hipGraphExec_t graph = nullptr;        // `replay` MAPG iterations of every problem + the multiplier steps
    int replay = 32;
    bool started = false;                  // between cr_batch_start and cr_batch_finish
    int64_t launched = 0, total = 0;       // replays launched, and the cap (the exact count of a fixed schedule)
    std::chrono::steady_clock::time_point t0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int32_t* pinned_flag = nullptr;
    int dev = 0;                 // device current at creation
    char* ws = nullptr;
    bool f64 = false;
    std::string err;
};

static cr_status bfail(cr_batch* b, cr_status s, const std::string& msg) {
    if (b) b->err = msg;
    g_last_error = msg;
    return s;
}

#define BHIPCHK(b, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return bfail(b, CR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

// One graph replay: b->replay MAPG iterations of every problem (positions q =
// 0 .. replay - 1; pass and reduce, plus the update kernel unless the passes
// are lazy), the end-of-replay gate of every problem's device schedule, and the
// gated multiplier steps (MAPG finish or end, set point, multiplier pass per
// operand class, KKT reduction, schedule step) of the problems whose run is over.
static cr_status capture_batch_graph(cr_batch* b, hipGraphExec_t* out) {
    const BatchPlan& B = b->plan;
    char* h = b->ws;
    const int iters = b->replay;
    // block-table segment of the problems with G = 16 << gs lanes per point
    auto seg = [&](int gs) { return (const void*)(h + B.off_blocks + (size_t)B.gseg_start[gs] * 8); };
    hipGraph_t g = nullptr;
    BHIPCHK(b, hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int q = 0; q < iters && e == hipSuccess; ++q) {
        for (size_t ci = 0; ci < B.ks_classes.size() && e == hipSuccess; ++ci) {
            e = cr::launch_pass_batched(b->f64, B.ks_classes[ci], (const cr::PassArgs*)(h + B.off_pass),
                                        (const int32_t*)(h + B.off_nstrips),
                                        h + B.off_items + (size_t)B.class_off[ci] * sizeof(BatchItemH),
                                        B.class_cnt[ci], b->cs, B.lazy, q);
        }
        for (int gs = 0; gs < 2 && e == hipSuccess; ++gs)
            if (B.gseg_count[gs])
                e = cr::launch_reduce_batched(b->f64, 16 << gs, (const cr::ReduceArgs*)(h + B.off_red), seg(gs),
                                              (const int32_t*)(h + B.off_nblk), B.gseg_count[gs], q, b->cs);
        for (int gs = 0; gs < 2 && e == hipSuccess && !B.lazy; ++gs)
            if (B.gseg_count[gs])
                e = cr::launch_update_batched(b->f64, 16 << gs, (const cr::UpdateArgs*)(h + B.off_upd), seg(gs),
                                              (const int32_t*)(h + B.off_nblk), B.gseg_count[gs], q, b->cs);
    }
    auto scheds = (cr::AlccSched* const*)(h + B.off_scheds);
    auto sts = (cr::DevState* const*)(h + B.off_sts);
    auto oas = (cr::OuterArgs* const*)(h + B.off_oas);
    if (e == hipSuccess)
        e = cr::launch_alcc_gate_batched(scheds, sts, oas, b->P, iters, (int32_t*)(h + B.off_any), b->cs);
    // lazy runs: the last iterate into y1p[0] / xi1p[0] first; the stopping
    // pieces then come from the reduce, not from update-kernel records
    for (int gs = 0; gs < 2 && e == hipSuccess && B.lazy; ++gs)
        if (B.gseg_count[gs])
            e = cr::launch_mapg_finish_batched(16 << gs, (const cr::PassArgs*)(h + B.off_pass), seg(gs),
                                               B.gseg_count[gs], b->cs);
    if (e == hipSuccess)
        e = cr::launch_mapg_end_batched((const double* const*)(h + B.off_bparts),
                                        (const int32_t*)(h + (B.lazy ? B.off_nblk0 : B.off_nblk)), sts, b->P, b->cs);
    for (int gs = 0; gs < 2 && e == hipSuccess; ++gs)
        if (B.gseg_count[gs])
            e = cr::launch_set_point_batched(b->f64, 16 << gs, (const cr::PointArgs*)(h + B.off_pt), seg(gs),
                                             (const int32_t*)(h + B.off_nblk), B.gseg_count[gs], b->cs);
    for (size_t ci = 0; ci < B.ks_classes.size() && e == hipSuccess; ++ci) {
        e = cr::launch_theta_pass_batched(b->f64, B.ks_classes[ci], (const cr::PassArgs*)(h + B.off_pass1),
                                          (const int32_t*)(h + B.off_nstrips),
                                          h + B.off_items + (size_t)B.class_off[ci] * sizeof(BatchItemH),
                                          B.class_cnt[ci], b->cs);
    }
    for (int gs = 0; gs < 2 && e == hipSuccess; ++gs)
        if (B.gseg_count[gs])
            e = cr::launch_reduce_batched(b->f64, 16 << gs, (const cr::ReduceArgs*)(h + B.off_red2), seg(gs),
                                          (const int32_t*)(h + B.off_nblk), B.gseg_count[gs], 0, b->cs);
    if (e == hipSuccess) e = cr::launch_alcc_step_batched(scheds, sts, oas, b->P, b->cs);
    hipError_t e2 = hipStreamEndCapture(b->cs, &g);
    if (e != hipSuccess) return bfail(b, CR_ERR_HIP, std::string("batch capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return bfail(b, CR_ERR_HIP, std::string("batch end capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { *out = nullptr; return bfail(b, CR_ERR_HIP, std::string("batch instantiate: ") + hipGetErrorString(e)); }
    return CR_OK;
}

static cr_status build_batch_graph(cr_batch* b) {
    if (!b->graph) return capture_batch_graph(b, &b->graph);
    return CR_OK;
}

extern "C" {

cr_status cr_batch_workspace_bytes(const cr_problem* probs, int32_t P, const cr_params* params, size_t* bytes) {
    std::string msg;
    if (!bytes) return fail(nullptr, CR_ERR_ARG, "bytes is NULL");
    cr_status s = check_batch(probs, P, params, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    *bytes = plan_batch(probs, P, params).total;
    return CR_OK;
}

cr_status cr_batch_destroy(cr_batch* b) {
    if (!b) return CR_OK;
    if (b->cs) hipStreamSynchronize(b->cs);
    if (b->graph) hipGraphExecDestroy(b->graph);
    for (cr_ctx* c : b->sub) cr_destroy(c);
    for (int q = 0; q < 2; ++q)
        if (b->ev[q]) hipEventDestroy(b->ev[q]);
    pinned_put(b->pinned_flag, b->dev);
    stream_put(b->cs, b->dev);
    delete b;
    return CR_OK;
}

}  // extern "C"

// shifts: per-problem slope shifts (null: none), fixed for the batch's lifetime.
static cr_status batch_init_impl(cr_batch** out, const cr_problem* probs, int32_t P, const cr_params* params,
                                 void* workspace_dev, size_t ws_bytes, void* stream, const double* const* shifts) {
    std::string msg;
    if (!out) return fail(nullptr, CR_ERR_ARG, "out is NULL");
    *out = nullptr;
    cr_status s = check_batch(probs, P, params, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!workspace_dev) return fail(nullptr, CR_ERR_ARG, "workspace must be non-NULL");
    for (int p = 0; p < P; ++p)
        if (!probs[p].X_dev || !probs[p].ybar_dev || !probs[p].y_dev || !probs[p].xi_dev)
            return fail(nullptr, CR_ERR_ARG, "problem " + std::to_string(p) + ": X, ybar, y and xi must be non-NULL");
    BatchPlan B = plan_batch(probs, P, params);
    if (ws_bytes < B.total) return fail(nullptr, CR_ERR_NOMEM, "workspace smaller than cr_batch_workspace_bytes()");
    cr_batch* b = new (std::nothrow) cr_batch();
    if (!b) return fail(nullptr, CR_ERR_NOMEM, "host allocation failed");
    b->P = P;
    b->p = *params;
    b->plan = B;
    b->probs.assign(probs, probs + P);
    b->user_stream = (hipStream_t)stream;
    b->ws = (char*)align256((size_t)workspace_dev);
    b->f64 = params->precision == CR_F64;
    b->replay = replay_iters(*params);
    auto bad = [&](cr_status st) { std::string m = g_last_error; cr_batch_destroy(b); g_last_error = m; return st; };
    b->dev = current_device();
    hipError_t e = stream_get(&b->cs);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&b->ev[q], hipEventDisableTiming);
    if (e == hipSuccess) e = pinned_get((void**)&b->pinned_flag);
    if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, std::string("batch resources: ") + hipGetErrorString(e)); return bad(CR_ERR_HIP); }
    // per-problem contexts (set-up of each problem on its own slice)
    for (int p = 0; p < P; ++p) {
        cr_ctx* c = nullptr;
        cr_params pp = *params;
        if (probs[p].tile_rows > 0) pp.tile_rows = probs[p].tile_rows;
        cr_status st = ctx_init(&c, probs[p].N, probs[p].n, &pp, probs[p].X_dev, probs[p].ybar_dev,
                                b->ws + B.off[p], B.L[p].total, stream, b->cs);
        if (st != CR_OK) { g_last_error = "problem " + std::to_string(p) + ": " + g_last_error; return bad(st); }
        // lazy batches: the next pass completes each MAPG step (no update kernel)
        c->lazy = B.lazy;
        c->shift = shifts ? shifts[p] : nullptr;
        b->sub.push_back(c);
    }
    // device argument tables
    std::vector<cr::PassArgs> pa(P);
    std::vector<cr::ReduceArgs> ra(P);
    std::vector<cr::UpdateArgs> ua(P);
    std::vector<int32_t> nstrips(P);
    std::vector<int32_t> blocks;
    std::vector<void*> sts(P), scheds(P), oas(P), bparts(P);
    std::vector<cr::PassArgs> pa1(P), pat(P);
    std::vector<cr::ReduceArgs> ra2(P);
    std::vector<cr::PointArgs> pt(P);
    std::vector<int32_t> zeros(P, 0);
    for (int p = 0; p < P; ++p) {
        cr_ctx* c = b->sub[p];
        const Layout& L = c->L;
        if (B.lazy) {
            // the reduce blocks of the problem (batch_group(n) lanes per point) leave the norm pieces
            pa[p] = lazy_pass_args(c, 0, 0);
            pa[p].lz.nblk = B.nblk[p];
            pat[p] = lazy_pass_args(c, 0, 2);
            pat[p].lz.nblk = B.nblk[p];
        } else {
            pa[p] = pass_args(c, 0, 0.0, &c->st->active);
            pat[p] = pass_args(c, 0, 0.0, &c->st->active);
        }
        ra[p] = reduce_args(c, 0, c->D(L.off_y2), c->D(L.off_xi2), c->D(L.off_vy), c->D(L.off_vxi), 0.0);
        if (B.lazy) ra[p].spart = c->D(L.off_spart);
        // adaptive schedules freeze problems at different times: their passes
        // and reduces test the activity flag before loading anything
        const int cf = params->inner_iters > 0 ? 0 : 1;
        pa[p].check_first = pat[p].check_first = ra[p].check_first = cf;
        ua[p] = update_args(c);
        nstrips[p] = L.strips;
        sts[p] = c->st;
        scheds[p] = c->sched;
        oas[p] = c->oa;
        bparts[p] = c->D(L.off_blockpart);
        // the multiplier step of the device schedule, gated on the problem's step_due
        pa1[p] = pass_args(c, 1, 0.0, &c->st->step_due);
        pa1[p].theta_scale_p = &c->oa->theta_scale;
        pa1[p].check_first = 1;                  // the gate is closed in most replays
        ra2[p] = reduce_args(c, 2, c->D(L.off_y1p), c->D(L.off_xi1p), nullptr, nullptr, 0.0);
        ra2[p].gate = &c->st->step_due;
        ra2[p].mu_dev = 1;
        ra2[p].check_first = 1;
        pt[p] = point_args(c, c->D(L.off_y1p), c->D(L.off_xi1p), 1);
        pt[p].gate = &c->st->step_due;
    }
    for (int gs = 0; gs < 2; ++gs)
        for (int p = 0; p < P; ++p)
            if ((batch_group(probs[p].n) == 16) == (gs == 0))
                for (int q = 0; q < B.nblk[p]; ++q) { blocks.push_back(p); blocks.push_back(q); }
    char* h = b->ws;
    // tables copied on the batch's stream, ahead of every kernel that reads them
    // (staged from pageable memory before each call returns)
    e = hipMemcpyAsync(h + B.off_pass, pa.data(), P * sizeof(cr::PassArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_red, ra.data(), P * sizeof(cr::ReduceArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_upd, ua.data(), P * sizeof(cr::UpdateArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_nstrips, nstrips.data(), P * 4, hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_blocks, blocks.data(), blocks.size() * 4, hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_nblk, B.nblk.data(), P * 4, hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_sts, sts.data(), P * sizeof(void*), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess && !B.items.empty())
        e = hipMemcpyAsync(h + B.off_items, B.items.data(), B.items.size() * sizeof(BatchItemH), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_scheds, scheds.data(), P * sizeof(void*), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_oas, oas.data(), P * sizeof(void*), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_bparts, bparts.data(), P * sizeof(void*), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_pass1, pa1.data(), P * sizeof(cr::PassArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_red2, ra2.data(), P * sizeof(cr::ReduceArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_pt, pt.data(), P * sizeof(cr::PointArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h + B.off_pass_time, pat.data(), P * sizeof(cr::PassArgs), hipMemcpyHostToDevice, b->cs);
    if (e == hipSuccess) e = hipMemcpyAsync(h + B.off_nblk0, zeros.data(), P * 4, hipMemcpyHostToDevice, b->cs);
    if (e != hipSuccess) { fail(nullptr, CR_ERR_HIP, std::string("batch tables: ") + hipGetErrorString(e)); return bad(CR_ERR_HIP); }
    *out = b;
    return CR_OK;
}

extern "C" {

cr_status cr_batch_init(cr_batch** out, const cr_problem* probs, int32_t P, const cr_params* params,
                        void* workspace_dev, size_t ws_bytes, void* stream) {
    return batch_init_impl(out, probs, P, params, workspace_dev, ws_bytes, stream, nullptr);
}

}  // extern "C"

// Every problem's last ALCC iterate into its caller-owned y and xi (enqueued).
static hipError_t batch_copy_outputs(cr_batch* b) {
    hipError_t e = hipSuccess;
    for (int q = 0; q < b->P && e == hipSuccess; ++q) {
        cr_ctx* c = b->sub[q];
        const Layout& L = c->L;
        e = hipMemcpyAsync(b->probs[q].y_dev, c->D(L.off_y1p), (size_t)c->N * 8, hipMemcpyDeviceToDevice, b->cs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->probs[q].xi_dev, c->D(L.off_xi1p), (size_t)c->N * c->n * 8, hipMemcpyDeviceToDevice,
                               b->cs);
    }
    return e;
}

extern "C" {

cr_status cr_batch_start(cr_batch* b) {
    if (!b) return fail(nullptr, CR_ERR_ARG, "batch is NULL");
    hipStream_t cs = b->cs;
    BHIPCHK(b, hipEventRecord(b->ev[0], b->user_stream));
    BHIPCHK(b, hipStreamWaitEvent(cs, b->ev[0], 0));
    cr_status bs = build_batch_graph(b);
    if (bs != CR_OK) return bs;
    b->t0 = std::chrono::steady_clock::now();
    for (int q = 0; q < b->P; ++q) {
        cr_ctx* c = b->sub[q];
        const Layout& L = c->L;
        BHIPCHK(b, cr::launch_zero(c->P(L.off_theta), (size_t)L.Nrow * L.ld * L.esz, cs));
        cr::PointArgs start = point_args(c, c->D(L.off_y0), c->D(L.off_xi0), 1);
        BHIPCHK(b, cr::launch_set_point(c->prec, start, cs));
    }
    const char* h = b->ws;
    BHIPCHK(b, cr::launch_alcc_start_batched((cr::AlccSched* const*)(h + b->plan.off_scheds),
                                             (cr::OuterArgs* const*)(h + b->plan.off_oas),
                                             (cr::DevState* const*)(h + b->plan.off_sts), b->P, cs));
    const cr_params& p = b->p;
    b->launched = 0;
    if (p.inner_iters > 0) {
        b->total = (int64_t)p.max_outer * ((p.inner_iters + b->replay - 1) / b->replay);
    } else {
        // a problem runs at most max_inner + one replay of MAPG iterations per ALCC iteration
        b->total = (int64_t)p.max_outer * ((p.max_inner + b->replay - 1) / b->replay + 1) + 2;
    }
    b->started = true;
    return CR_OK;
}

cr_status cr_batch_advance(cr_batch* b, int32_t max_replays, int32_t* running) {
    if (!b || !running) return fail(nullptr, CR_ERR_ARG, "batch and running must be non-NULL");
    if (!b->started) return bfail(b, CR_ERR_STATE, "cr_batch_start first");
    if (max_replays < 1) return bfail(b, CR_ERR_ARG, "max_replays must be >= 1");
    hipStream_t cs = b->cs;
    const bool fixed = b->p.inner_iters > 0;
    int32_t* any = (int32_t*)(b->ws + b->plan.off_any);
    *running = 1;
    if (fixed) {
        // the replay count is known: enqueue, nothing to read back
        const int64_t n = std::min<int64_t>(max_replays, b->total - b->launched);
        for (int64_t r = 0; r < n; ++r) BHIPCHK(b, hipGraphLaunch(b->graph, cs));
        b->launched += n;
        if (b->launched >= b->total) *running = 0;
        return CR_OK;
    }
    int slot = 0, pending = -1;
    for (int32_t r = 0; r < max_replays && b->launched < b->total; ++r) {
        BHIPCHK(b, hipGraphLaunch(b->graph, cs));
        b->launched += 1;
        BHIPCHK(b, hipMemcpyAsync(b->pinned_flag + slot, any, 4, hipMemcpyDeviceToHost, cs));
        BHIPCHK(b, hipEventRecord(b->ev[slot], cs));
        if (pending >= 0) {
            BHIPCHK(b, hipEventSynchronize(b->ev[pending]));
            if (b->pinned_flag[pending] == 0) { *running = 0; break; }
        }
        pending = slot;
        slot ^= 1;
    }
    if (*running) {
        BHIPCHK(b, hipStreamSynchronize(cs));
        if (pending >= 0 && b->pinned_flag[pending] == 0) *running = 0;
        if (b->launched >= b->total) *running = 0;
    }
    return CR_OK;
}

cr_status cr_batch_finish(cr_batch* b, cr_info* infos, double* seconds) {
    if (!b) return fail(nullptr, CR_ERR_ARG, "batch is NULL");
    if (!b->started) return bfail(b, CR_ERR_STATE, "cr_batch_start first");
    const int P = b->P;
    const cr_params& p = b->p;
    const bool fixed = p.inner_iters > 0;
    hipStream_t cs = b->cs;
    BHIPCHK(b, batch_copy_outputs(b));
    BHIPCHK(b, hipStreamSynchronize(cs));
    b->started = false;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - b->t0).count();
    if (seconds) *seconds = secs;
    cr_status result = CR_OK;
    for (int q = 0; q < P; ++q) {
        cr_ctx* c = b->sub[q];
        cr::AlccSched sc{};
        cr::DevState h{};
        BHIPCHK(b, hipMemcpy(&sc, c->sched, sizeof(sc), hipMemcpyDeviceToHost));
        BHIPCHK(b, hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost));
        cr_status st = CR_OK;
        if (sc.nonfinite) st = CR_ERR_NONFINITE;
        else if (sc.phase != 2) st = CR_ERR_STATE;
        else if (!fixed && !sc.converged) st = CR_NOT_CONVERGED;
        if (st == CR_ERR_NONFINITE || st == CR_ERR_STATE) result = st;
        else if (st == CR_NOT_CONVERGED && result == CR_OK) result = st;
        if (infos) {
            cr_info& info = infos[q];
            std::memset(&info, 0, sizeof(info));
            fill_info(c, h, &info);
            info.outer_iters = std::min(sc.k, p.max_outer);
            info.inner_iters = sc.total_inner;
            info.seconds = secs;
            info.pair_updates = (double)c->N * (double)(c->N - 1) * (double)sc.total_inner;
            info.status = st;
        }
    }
    if (result == CR_ERR_NONFINITE) return bfail(b, result, "non-finite iterate");
    if (result == CR_ERR_STATE) return bfail(b, result, "a schedule did not finish within its replay cap");
    return result;
}

cr_status cr_batch_run(cr_batch* b, cr_info* infos, double* seconds) {
    cr_status s = cr_batch_start(b);
    if (s != CR_OK) return s;
    int32_t running = 1;
    while (running) {
        s = cr_batch_advance(b, 1 << 30, &running);
        if (s != CR_OK) return s;
    }
    return cr_batch_finish(b, infos, seconds);
}

cr_status cr_batch_time_pass(cr_batch* b, int32_t reps, double* avg_ms) {
    if (!b || !avg_ms) return fail(nullptr, CR_ERR_ARG, "batch and avg_ms must be non-NULL");
    if (reps < 1) return bfail(b, CR_ERR_ARG, "reps must be >= 1");
    const BatchPlan& B = b->plan;
    char* h = b->ws;
    hipStream_t cs = b->cs;
    BHIPCHK(b, hipEventRecord(b->ev[0], b->user_stream));
    BHIPCHK(b, hipStreamWaitEvent(cs, b->ev[0], 0));
    // every problem active, at its current operands (a later cr_batch_run starts afresh)
    for (int q = 0; q < b->P; ++q) {
        cr_ctx* c = b->sub[q];
        Schedule sch;
        sch.start(c);
        BHIPCHK(b, cr::launch_begin_outer(sch.next(c), c->oa, c->st, cs));
    }
    // the kernels a run launches: lazy passes at iteration 2 (every problem
    // active), else the update-kernel form's passes
    auto step = [&]() {
        hipError_t e = hipSuccess;
        for (size_t ci = 0; ci < B.ks_classes.size() && e == hipSuccess; ++ci) {
            e = cr::launch_pass_batched(b->f64, B.ks_classes[ci], (const cr::PassArgs*)(h + B.off_pass_time),
                                        (const int32_t*)(h + B.off_nstrips),
                                        h + B.off_items + (size_t)B.class_off[ci] * sizeof(BatchItemH),
                                        B.class_cnt[ci], cs, B.lazy, 0);
        }
        return e;
    };
    BHIPCHK(b, step());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIPCHK(b, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, cs);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = step();
    if (e == hipSuccess) e = hipEventRecord(e1, cs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return bfail(b, CR_ERR_HIP, std::string("batch time pass: ") + hipGetErrorString(e));
    *avg_ms = (double)ms / reps;
    return CR_OK;
}

cr_status cr_solve_batched(const cr_problem* probs, int32_t P, const cr_params* params, void* workspace_dev,
                           size_t ws_bytes, cr_info* infos, void* stream) {
    cr_batch* b = nullptr;
    cr_status s = cr_batch_init(&b, probs, P, params, workspace_dev, ws_bytes, stream);
    if (s != CR_OK) return s;
    s = cr_batch_run(b, infos, nullptr);
    if (s != CR_OK && s != CR_NOT_CONVERGED) g_last_error = b->err;
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
        hipEventRecord(done, b->cs);
        hipStreamWaitEvent((hipStream_t)stream, done, 0);
        hipEventDestroy(done);
    }
    cr_batch_destroy(b);
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiable form: the fixed-schedule map and its reverse pass.  The
// forward is cr_run's fixed schedule launched iteration by iteration, keeping
// theta_k of every ALCC iteration and the MAPG state every C iterations.  The
// reverse pass walks the ALCC iterations backwards; for each segment of C MAPG
// steps it recomputes the segment from its checkpoint (saving each step's pass
// point, unprojected step and norms), then applies the step adjoints in
// reverse: momentum, projection, pair pass, reduction.
// ---------------------------------------------------------------------------
namespace {

struct DiffLayout {
    int K = 0, Lin = 0, C = 0, nseg = 0;
    size_t vecN = 0;                 // doubles of one (y, xi) pair of vectors: Nrow (n + 1)
    size_t off_thst, off_thbar, off_ckpt, off_sv, off_svn, off_vec, off_diraug, off_acol, off_rowv, off_cw, off_bp;
    size_t total;
};

enum DiffVec { kPB = 0, kQB, kG1, kVB, kYA, kACC, kZERO, kNumVec };

DiffLayout make_diff_layout(const Layout& L, const cr_params& p, int C) {
    DiffLayout D;
    D.K = p.max_outer;
    D.Lin = p.inner_iters;
    D.C = std::max(1, std::min(C, D.Lin));
    D.nseg = (D.Lin + D.C - 1) / D.C;
    D.vecN = (size_t)L.Nrow * (L.n + 1);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t th = (size_t)L.Nrow * L.ld * L.esz;
    D.off_thst = take(th * (size_t)(D.K - 1));
    D.off_thbar = take(D.K > 1 ? th : 0);
    D.off_ckpt = take((size_t)D.K * D.nseg * 2 * D.vecN * 8);
    D.off_sv = take((size_t)D.C * 2 * D.vecN * 8);
    D.off_svn = take((size_t)D.C * 4 * 8);
    D.off_vec = take((size_t)kNumVec * D.vecN * 8);
    D.off_diraug = take((size_t)L.ld * L.kp * L.esz);
    D.off_acol = take((size_t)L.Nrow * L.esz);
    D.off_rowv = take((size_t)L.strips * L.Nrow * L.n * L.esz);
    D.off_cw = take((size_t)L.chunks * L.ld * L.esz);
    D.off_bp = take((size_t)(cr::adj_vec_blocks(L.Nrow, L.n) + 1) * 4 * 8);
    D.total = o + 256;
    return D;
}

bool check_diff(const cr_params* p, int32_t C, std::string& msg, cr_status& st) {
    st = CR_ERR_ARG;
    if (!check_params(p, msg)) return false;
    if (p->inner_iters < 1) { msg = "the differentiable form needs a fixed schedule (inner_iters >= 1)"; return false; }
    if (C < 1) { msg = "checkpoint_every must be >= 1"; return false; }
    if (p->precision == CR_MIXED_BF16) {
        msg = "the differentiable form runs CR_F64 and CR_F32";
        st = CR_ERR_UNSUPPORTED;
        return false;
    }
    return true;
}

}  // namespace

struct cr_diff {
    cr_ctx* c = nullptr;
    DiffLayout D;
    size_t base_bytes = 0;
    char* ws = nullptr;
    bool have_fwd = false, have_bwd = false;
    std::vector<cr::OuterArgs> oas;
    std::vector<double> beta;        // beta_l, l = 1..Lin (index l)
    double* Dp(size_t off) const { return reinterpret_cast<double*>(ws + off); }
    char* Pp(size_t off) const { return ws + off; }
    // pair of vectors: y part (Nrow), then xi part (Nrow n)
    double* vy(int which) const { return Dp(D.off_vec) + (size_t)which * D.vecN; }
    double* vxi(int which) const { return vy(which) + c->L.Nrow; }
    double* ck(int k, int s, int part) const {          // part 0: (y1p, xi1p), 1: (y2, xi2)
        return Dp(D.off_ckpt) + (((size_t)(k - 1) * D.nseg + s) * 2 + part) * D.vecN;
    }
    double* sv(int slot, int part) const {              // part 0: (y2, xi2), 1: (v_y, v_xi)
        return Dp(D.off_sv) + ((size_t)slot * 2 + part) * D.vecN;
    }
    double* svn(int slot) const { return Dp(D.off_svn) + (size_t)slot * 4; }
    void* thst(int k) const {                            // theta_k, k >= 2
        return Pp(D.off_thst + (size_t)(k - 2) * c->L.Nrow * c->L.ld * c->L.esz);
    }
};

static cr_status dfail(cr_diff* d, cr_status s, const std::string& msg) { return fail(d ? d->c : nullptr, s, msg); }

#define DHIPCHK(d, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return dfail(d, CR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

static hipError_t copy_pair(cr_diff* d, double* dst_y, double* dst_xi, const double* src_y, const double* src_xi,
                            hipStream_t s) {
    const cr_ctx* c = d->c;
    hipError_t e = hipMemcpyAsync(dst_y, src_y, (size_t)c->N * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst_xi, src_xi, (size_t)c->N * c->n * 8, hipMemcpyDeviceToDevice, s);
    return e;
}

static cr::AdjPassArgs adj_pass_args(cr_diff* d, int mode, int tb_mode, double scale) {
    cr_ctx* c = d->c;
    const Layout& L = c->L;
    cr::AdjPassArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.n = L.n; a.nc = L.nc; a.rows_per_chunk = L.rpc; a.kp = L.kp;
    a.mode = mode; a.tb_mode = tb_mode;
    a.theta = c->P(L.off_theta); a.thetabar = d->D.K > 1 ? d->Pp(d->D.off_thbar) : nullptr;
    a.xp = c->P(L.off_xp); a.xiaug = c->P(L.off_xiaug); a.ycol = c->P(L.off_ycol);
    a.diraug = d->Pp(d->D.off_diraug); a.acol = d->Pp(d->D.off_acol);
    a.rowpart = c->P(L.off_rowpart); a.rowvpart = d->Pp(d->D.off_rowv);
    a.cpart = c->P(L.off_cpart); a.cwpart = d->Pp(d->D.off_cw);
    a.scale = scale;
    return a;
}

static cr::AdjReduceArgs adj_reduce_args(cr_diff* d, int mode, const double* xi, const cr::OuterArgs& oa) {
    cr_ctx* c = d->c;
    const Layout& L = c->L;
    cr::AdjReduceArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.n = L.n; a.nc = L.nc; a.strips = L.strips; a.chunks = L.chunks;
    a.mode = mode;
    a.rowpart = c->P(L.off_rowpart); a.rowvpart = d->Pp(d->D.off_rowv);
    a.cpart = c->P(L.off_cpart); a.cwpart = d->Pp(d->D.off_cw);
    a.X = c->X; a.xi = xi;
    a.vb_y = d->vy(kVB); a.vb_xi = d->vxi(kVB);
    a.sy = oa.sy; a.sxi = oa.sxi; a.mu = oa.mu; a.gamma = oa.gamma;
    if (mode == 0) { a.out_y = d->vy(kQB); a.out_xi = d->vxi(kQB); }
    else { a.out_y = d->vy(kYA); a.out_xi = d->vxi(kYA); }
    a.dybar = d->vy(kACC); a.dX = d->vxi(kACC);
    return a;
}

static cr::AdjVecArgs adj_vec_args(cr_diff* d, const cr::OuterArgs& oa, double beta, int slot) {
    cr_ctx* c = d->c;
    const Layout& L = c->L;
    cr::AdjVecArgs a{};
    a.N = L.N; a.Nrow = L.Nrow; a.ld = L.ld; a.n = L.n; a.kp = L.kp;
    a.beta = beta; a.sy = oa.sy; a.sxi = oa.sxi; a.By = oa.By; a.Bxi = oa.Bxi;
    a.X = c->X; a.ybar = c->ybar;
    a.pb_y = d->vy(kPB); a.pb_xi = d->vxi(kPB);
    a.qb_y = d->vy(kQB); a.qb_xi = d->vxi(kQB);
    a.g1_y = d->vy(kG1); a.g1_xi = d->vxi(kG1);
    a.v_y = d->sv(slot, 1); a.v_xi = d->sv(slot, 1) + L.Nrow;
    a.nrm = d->svn(slot);
    a.vb_y = d->vy(kVB); a.vb_xi = d->vxi(kVB);
    a.dybar = d->vy(kACC);
    a.diraug = d->Pp(d->D.off_diraug); a.acol = d->Pp(d->D.off_acol);
    a.blockpart = d->Dp(d->D.off_bp);
    return a;
}

extern "C" {

cr_status cr_diff_workspace_bytes(int64_t N, int32_t n, const cr_params* params, int32_t checkpoint_every,
                                  size_t* bytes) {
    std::string msg;
    if (!bytes) return fail(nullptr, CR_ERR_ARG, "bytes is NULL");
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!check_diff(params, checkpoint_every, msg, s)) return fail(nullptr, s, msg);
    Layout L = make_layout(N, n, *params, params->tile_rows);
    *bytes = L.total + make_diff_layout(L, *params, checkpoint_every).total;
    return CR_OK;
}

cr_status cr_diff_init(cr_diff** out, int64_t N, int32_t n, const cr_params* params, int32_t checkpoint_every,
                       const void* X_dev, const void* ybar_dev, void* workspace_dev, size_t ws_bytes,
                       void* stream) {
    std::string msg;
    if (!out) return fail(nullptr, CR_ERR_ARG, "out is NULL");
    *out = nullptr;
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!check_diff(params, checkpoint_every, msg, s)) return fail(nullptr, s, msg);
    if (!X_dev || !ybar_dev || !workspace_dev) return fail(nullptr, CR_ERR_ARG, "X, ybar and workspace must be non-NULL");
    Layout L = make_layout(N, n, *params, params->tile_rows);
    DiffLayout D = make_diff_layout(L, *params, checkpoint_every);
    if (ws_bytes < L.total + D.total) return fail(nullptr, CR_ERR_NOMEM, "workspace smaller than cr_diff_workspace_bytes()");
    cr_diff* d = new (std::nothrow) cr_diff();
    if (!d) return fail(nullptr, CR_ERR_NOMEM, "host allocation failed");
    s = cr_init(&d->c, N, n, params, X_dev, ybar_dev, workspace_dev, L.total, stream);
    if (s != CR_OK) { delete d; return s; }
    // checkpoints hold (y1_{l-1}, y2_l) before each segment, which needs the
    // update kernel to complete every step
    d->c->lazy = false;
    d->D = D;
    d->base_bytes = L.total;
    d->ws = (char*)align256((size_t)workspace_dev + L.total);
    d->beta.assign((size_t)D.Lin + 2, 0.0);
    double t = 1.0;
    for (int l = 1; l <= D.Lin + 1; ++l) {
        const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        d->beta[l] = (t - 1.0) / tn;
        t = tn;
    }
    hipStream_t cs = d->c->cs;
    hipError_t e = cr::launch_zero(d->Pp(D.off_diraug), (size_t)L.ld * L.kp * L.esz, cs);
    if (e == hipSuccess) e = cr::launch_zero(d->Pp(D.off_acol), (size_t)L.Nrow * L.esz, cs);
    if (e == hipSuccess) e = cr::launch_zero(d->Pp(D.off_vec), (size_t)kNumVec * D.vecN * 8, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (e != hipSuccess) {
        fail(nullptr, CR_ERR_HIP, std::string("diff set-up: ") + hipGetErrorString(e));
        cr_diff_destroy(d);
        return CR_ERR_HIP;
    }
    *out = d;
    return CR_OK;
}

cr_status cr_diff_destroy(cr_diff* d) {
    if (!d) return CR_OK;
    cr_destroy(d->c);
    delete d;
    return CR_OK;
}

cr_status cr_diff_forward(cr_diff* d, const void* y0_dev, const void* xi0_dev, void* y_dev, void* xi_dev,
                          cr_info* info) {
    if (!d) return fail(nullptr, CR_ERR_ARG, "diff is NULL");
    if (!y_dev || !xi_dev) return dfail(d, CR_ERR_ARG, "y and xi must be non-NULL");
    cr_ctx* c = d->c;
    const Layout& L = c->L;
    const DiffLayout& D = d->D;
    hipStream_t cs = c->cs;
    d->have_fwd = false;
    d->have_bwd = false;
    DHIPCHK(d, hipEventRecord(c->ev[0], c->user_stream));
    DHIPCHK(d, hipStreamWaitEvent(cs, c->ev[0], 0));
    const auto t0 = std::chrono::steady_clock::now();
    const size_t th_bytes = (size_t)L.Nrow * L.ld * L.esz;

    DHIPCHK(d, cr::launch_zero(c->P(L.off_theta), th_bytes, cs));
    const double* y0 = y0_dev ? (const double*)y0_dev : c->ybar;
    const double* xi0 = xi0_dev ? (const double*)xi0_dev : d->vxi(kZERO);
    cr::PointArgs start = point_args(c, y0, xi0, 1);
    DHIPCHK(d, cr::launch_set_point(c->prec, start, cs));

    Schedule sch;
    sch.start(c);
    d->oas.clear();
    cr::DevState h{};
    for (int k = 1; k <= D.K; ++k) {
        const cr::OuterArgs oa = sch.next(c);
        d->oas.push_back(oa);
        const double mu = sch.mu, mu_next = sch.mu_next(c);
        if (k >= 2) DHIPCHK(d, hipMemcpyAsync(d->thst(k), c->P(L.off_theta), th_bytes, hipMemcpyDeviceToDevice, cs));
        DHIPCHK(d, cr::launch_begin_outer(oa, c->oa, c->st, cs, 0));
        for (int l = 1; l <= D.Lin; ++l) {
            if ((l - 1) % D.C == 0) {
                const int sg = (l - 1) / D.C;
                double* c0 = d->ck(k, sg, 0);
                double* c1 = d->ck(k, sg, 1);
                DHIPCHK(d, copy_pair(d, c0, c0 + L.Nrow, c->D(L.off_y1p), c->D(L.off_xi1p), cs));
                DHIPCHK(d, copy_pair(d, c1, c1 + L.Nrow, c->D(L.off_y2), c->D(L.off_xi2), cs));
            }
            DHIPCHK(d, enqueue_mapg_iteration(c, l - 1, cs));
        }
        DHIPCHK(d, enqueue_multiplier_step(c, mu, mu_next, D.Lin, cr::reduce_blocks(c->N, c->n), cs));
        sch.total_inner += D.Lin;
        sch.advance(c);
    }
    // the fixed schedule needs nothing from the device: one read-back at the end
    // (a non-finite iterate stays non-finite through the later iterations)
    DHIPCHK(d, copy_pair(d, (double*)y_dev, (double*)xi_dev, c->D(L.off_y1p), c->D(L.off_xi1p), cs));
    DHIPCHK(d, hipStreamSynchronize(cs));
    h = *c->pinned_state;
    if (h.iterate_nonfinite) return dfail(d, CR_ERR_NONFINITE, "non-finite iterate");
    c->have_kkt = true;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        fill_info(c, h, info);
        info->outer_iters = D.K;
        info->inner_iters = sch.total_inner;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->pair_updates = (double)c->N * (double)(c->N - 1) * (double)sch.total_inner;
        info->status = CR_OK;
    }
    d->have_fwd = true;
    return CR_OK;
}

cr_status cr_diff_backward(cr_diff* d, const void* gy_dev, const void* gxi_dev, void* dX_dev, void* dybar_dev,
                           void* dy0_dev, void* dxi0_dev) {
    if (!d) return fail(nullptr, CR_ERR_ARG, "diff is NULL");
    if (!gy_dev || !dX_dev || !dybar_dev || !dy0_dev || !dxi0_dev)
        return dfail(d, CR_ERR_ARG, "gy, dX, dybar, dy0 and dxi0 must be non-NULL");
    if (!d->have_fwd) return dfail(d, CR_ERR_STATE, "cr_diff_backward needs a completed cr_diff_forward");
    cr_ctx* c = d->c;
    const Layout& L = c->L;
    const DiffLayout& D = d->D;
    hipStream_t cs = c->cs;
    DHIPCHK(d, hipEventRecord(c->ev[0], c->user_stream));
    DHIPCHK(d, hipStreamWaitEvent(cs, c->ev[0], 0));
    const size_t th_bytes = (size_t)L.Nrow * L.ld * L.esz;
    const size_t pair_bytes = D.vecN * 8;
    const bool f64 = c->f64;
    const dim3 grid = pass_grid(L);
    const int nvb = cr::adj_vec_blocks(c->N, c->n);

    DHIPCHK(d, cr::launch_zero(d->vy(kACC), pair_bytes, cs));
    DHIPCHK(d, cr::launch_zero(d->vy(kYA), pair_bytes, cs));
    DHIPCHK(d, hipMemcpyAsync(d->vy(kYA), gy_dev, (size_t)c->N * 8, hipMemcpyDeviceToDevice, cs));
    if (gxi_dev)
        DHIPCHK(d, hipMemcpyAsync(d->vxi(kYA), gxi_dev, (size_t)c->N * c->n * 8, hipMemcpyDeviceToDevice, cs));
    if (D.K > 1) DHIPCHK(d, cr::launch_zero(d->Pp(D.off_thbar), th_bytes, cs));

    for (int k = D.K; k >= 1; --k) {
        const cr::OuterArgs& oa = d->oas[k - 1];
        if (k >= 2) DHIPCHK(d, hipMemcpyAsync(c->P(L.off_theta), d->thst(k), th_bytes, hipMemcpyDeviceToDevice, cs));
        else DHIPCHK(d, cr::launch_zero(c->P(L.off_theta), th_bytes, cs));

        if (k < D.K) {
            // multiplier step k: theta_{k+1} = s (A1 y_k + A2 xi_k - theta_k)_-, at (y_k, xi_k)
            const double* yk = d->ck(k + 1, 0, 0);
            const double* xik = yk + L.Nrow;
            cr::PointArgs pt = point_args(c, yk, xik, 0);
            DHIPCHK(d, cr::launch_set_point(c->prec, pt, cs));
            cr::AdjPassArgs pa = adj_pass_args(d, 1, k >= 2 ? 2 : 0, oa.theta_scale);
            DHIPCHK(d, cr::launch_adj_pass(f64, c->n, pa, grid, cs));
            cr::AdjReduceArgs ra = adj_reduce_args(d, 1, xik, oa);
            DHIPCHK(d, cr::launch_adj_reduce(f64, ra, cs));
        }

        // MAPG of iteration k, backwards: pb = adjoint of y_k = y^(1)_L, qb = 0
        DHIPCHK(d, hipMemcpyAsync(d->vy(kPB), d->vy(kYA), pair_bytes, hipMemcpyDeviceToDevice, cs));
        DHIPCHK(d, cr::launch_zero(d->vy(kQB), pair_bytes, cs));
        for (int sg = D.nseg - 1; sg >= 0; --sg) {
            const int l0 = sg * D.C + 1, l1 = std::min(D.Lin, l0 + D.C - 1);
            // recompute the segment from its checkpoint, saving every step
            const double* c0 = d->ck(k, sg, 0);
            const double* c1 = d->ck(k, sg, 1);
            DHIPCHK(d, copy_pair(d, c->D(L.off_y1p), c->D(L.off_xi1p), c0, c0 + L.Nrow, cs));
            DHIPCHK(d, copy_pair(d, c->D(L.off_y2), c->D(L.off_xi2), c1, c1 + L.Nrow, cs));
            cr::PointArgs pt = point_args(c, c->D(L.off_y2), c->D(L.off_xi2), 0);
            DHIPCHK(d, cr::launch_set_point(c->prec, pt, cs));
            DHIPCHK(d, cr::launch_begin_outer(oa, c->oa, c->st, cs, l0 - 1));
            for (int l = l0; l <= l1; ++l) {
                const int q = l - l0;
                cr::PassArgs pa = pass_args(c, 0, 0.0, &c->st->active);
                DHIPCHK(d, cr::launch_pair_pass(c->prec, c->n, pa, grid, cs));
                cr::ReduceArgs ra = reduce_args(c, 0, c->D(L.off_y2), c->D(L.off_xi2), c->D(L.off_vy),
                                                c->D(L.off_vxi), 0.0);
                ra.q = q;
                DHIPCHK(d, cr::launch_reduce(c->f64, ra, cs));
                cr::UpdateArgs ua = update_args(c);
                ua.q = q;
                ua.sv_y2 = d->sv(q, 0); ua.sv_xi2 = d->sv(q, 0) + L.Nrow;
                ua.sv_vy = d->sv(q, 1); ua.sv_vxi = d->sv(q, 1) + L.Nrow;
                ua.sv_nrm = d->svn(q);
                DHIPCHK(d, cr::launch_update(c->prec, ua, cs));
            }
            // step adjoints in reverse
            for (int l = l1; l >= l0; --l) {
                const int q = l - l0;
                cr::AdjVecArgs va = adj_vec_args(d, oa, d->beta[l], q);
                DHIPCHK(d, cr::launch_adj_momentum(va, cs));
                DHIPCHK(d, cr::launch_adj_project(f64, va, nvb, cs));
                const double* qy = d->sv(q, 0);
                const double* qxi = qy + L.Nrow;
                cr::PointArgs pq = point_args(c, qy, qxi, 0);
                DHIPCHK(d, cr::launch_set_point(c->prec, pq, cs));
                cr::AdjPassArgs pa = adj_pass_args(d, 0, k >= 2 ? 1 : 0, 0.0);
                DHIPCHK(d, cr::launch_adj_pass(f64, c->n, pa, grid, cs));
                cr::AdjReduceArgs ra = adj_reduce_args(d, 0, qxi, oa);
                DHIPCHK(d, cr::launch_adj_reduce(f64, ra, cs));
            }
        }
        // adjoint of y_{k-1} = y^(1)_0 = y^(2)_1
        DHIPCHK(d, cr::launch_add(d->vy(kYA), d->vy(kPB), d->vy(kQB), (int64_t)D.vecN, cs));
    }
    DHIPCHK(d, copy_pair(d, (double*)dy0_dev, (double*)dxi0_dev, d->vy(kYA), d->vxi(kYA), cs));
    DHIPCHK(d, copy_pair(d, (double*)dybar_dev, (double*)dX_dev, d->vy(kACC), d->vxi(kACC), cs));
    DHIPCHK(d, hipStreamSynchronize(cs));
    d->have_bwd = true;
    return CR_OK;
}

cr_status cr_diff_time_adjoint_pass(cr_diff* d, int32_t reps, double* avg_ms) {
    if (!d || !avg_ms) return fail(d ? d->c : nullptr, CR_ERR_ARG, "diff and avg_ms must be non-NULL");
    if (reps < 1) return dfail(d, CR_ERR_ARG, "reps must be >= 1");
    if (!d->have_bwd) return dfail(d, CR_ERR_STATE, "cr_diff_time_adjoint_pass needs a completed cr_diff_backward");
    cr_ctx* c = d->c;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DHIPCHK(d, hipEventCreate(&e0));
    DHIPCHK(d, hipEventCreate(&e1));
    cr::AdjPassArgs pa = adj_pass_args(d, 0, d->D.K > 1 ? 1 : 0, 0.0);
    hipError_t e = hipEventRecord(e0, c->cs);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = cr::launch_adj_pass(c->f64, c->n, pa, pass_grid(c->L), c->cs);
    if (e == hipSuccess) e = hipEventRecord(e1, c->cs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return dfail(d, CR_ERR_HIP, std::string("time adjoint pass: ") + hipGetErrorString(e));
    *avg_ms = (double)ms / reps;
    return CR_OK;
}

}  // extern "C"

namespace cr {
// Message of a failed context-free call in another source file (cr_last_error(NULL)).
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace cr

// ---------------------------------------------------------------------------
// P-APG (Fig. 2): the K block problems of step 1 are one batch of shifted-slope
// problems whose data (ybar_i + u_i) and slope centres (v_i / gamma) are
// rewritten in place before every iteration; each problem's set-up (affine
// fit, Bbar) is redone for its new data.  Step 2 and the data of the next
// step 1 are the O(N^2) kernels of cr_papg.hip.
// ---------------------------------------------------------------------------
namespace {

struct PapgLayout {
    int64_t N = 0, Nbar = 0;
    int n = 0, K = 0;
    size_t th[2], ty[2], ybs, shift, y, xis, part, cpart, scal, trace, pvy, pvxi, pzero, su, supart, y0, xi0, st,
        batch;
    size_t batch_bytes = 0, total = 0;
};

cr_status check_papg(int64_t N, int32_t n, const cr_params* alcc, const cr_papg_params* pp, std::string& msg) {
    if (!alcc || !pp) { msg = "alcc and pp must be non-NULL"; return CR_ERR_ARG; }
    cr_status s = check_dims(N, n, msg);
    if (s != CR_OK) return s;
    if (!check_params(alcc, msg)) return CR_ERR_ARG;
    if (pp->K < 1 || N % pp->K != 0 || N / pp->K < 2) { msg = "K must divide N with N / K >= 2"; return CR_ERR_ARG; }
    if (pp->iters < 1) { msg = "iters must be >= 1"; return CR_ERR_ARG; }
    if (pp->method != CR_PAPG_ACCELERATED && pp->method != CR_PAPG_GRADIENT) { msg = "unknown method"; return CR_ERR_ARG; }
    if (pp->power_iters < 0) { msg = "power_iters must be >= 0"; return CR_ERR_ARG; }
    if (alcc->precision == CR_MIXED_BF16) { msg = "P-APG block solves run CR_F64 or CR_F32"; return CR_ERR_UNSUPPORTED; }
    return CR_OK;
}

// Rows per chunk of the block solves when the caller leaves tile_rows at 0: the
// batched pass runs a persistent grid of about 2 workgroups per CU (512 on
// MI355X) over (problem, strip, chunk) items, so the chunks are sized for about
// that many items in total instead of the single-problem default.
int papg_block_tile_rows(int64_t nb, int K, const cr_params* alcc) {
    if (alcc->tile_rows > 0) return alcc->tile_rows;
    const int tw = alcc->precision == CR_F64 ? 2 : 4;
    const int64_t ld = (nb + 63) / 64 * 64;
    const int64_t strips = ld / (16 * tw);
    const int64_t target = 512;
    int64_t chunks = (target + (int64_t)K * strips / 2) / ((int64_t)K * strips);
    chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, ld / 64));
    const int64_t rpc = ((ld + chunks - 1) / chunks + 63) / 64 * 64;
    return (int)rpc;
}

std::vector<cr_problem> papg_problems(int64_t N, int n, int K, const double* X, double* ybs, double* y, double* xis,
                                      const cr_params* alcc) {
    const int64_t nb = N / K;
    std::vector<cr_problem> pr(K);
    const int tr = papg_block_tile_rows(nb, K, alcc);
    for (int i = 0; i < K; ++i) {
        pr[i].N = nb;
        pr[i].n = n;
        pr[i].tile_rows = tr;
        pr[i].X_dev = X ? X + i * nb * n : nullptr;
        pr[i].ybar_dev = ybs ? ybs + i * nb : nullptr;
        pr[i].y_dev = y ? y + i * nb : nullptr;
        pr[i].xi_dev = xis ? xis + i * nb * n : nullptr;
    }
    return pr;
}

PapgLayout papg_layout(int64_t N, int n, const cr_params* alcc, const cr_papg_params* pp) {
    PapgLayout P;
    P.N = N; P.n = n; P.K = pp->K; P.Nbar = N / pp->K;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    for (int q = 0; q < 2; ++q) P.th[q] = take((size_t)N * N * 8);
    for (int q = 0; q < 2; ++q) P.ty[q] = take((size_t)N * 8);
    P.ybs = take((size_t)N * 8);
    P.shift = take((size_t)N * n * 8);
    P.y = take((size_t)N * 8);
    P.xis = take((size_t)N * n * 8);
    P.part = take((size_t)cr::papg_step_parts(N) * 3 * 8);
    P.cpart = take((size_t)cr::papg_col_chunks(N) * N * (n + 1) * 8);
    P.scal = take(64);
    P.trace = take((size_t)pp->iters * 3 * 8);
    P.pvy = take((size_t)N * 8);
    P.pvxi = take((size_t)N * n * 8);
    P.pzero = take((size_t)N * 8);
    // set-up of the whole point set, for sigma_max(A2)^2 of the default L
    const int64_t ld = (N + 63) / 64 * 64;
    const int64_t nsu = (N + cr::kSuRows - 1) / cr::kSuRows, nbk = (ld * 32 + cr::kBlock - 1) / cr::kBlock;
    P.supart = take((size_t)(std::max<int64_t>(nsu * (n * n + n + 3), nbk) + 64) * 8);
    P.su = take((size_t)(3 * n + 2 + n * n + 8) * 8);
    P.y0 = take((size_t)N * 8);
    P.xi0 = take((size_t)N * n * 8);
    P.st = take(sizeof(cr::DevState));
    std::vector<cr_problem> pr = papg_problems(N, n, pp->K, nullptr, nullptr, nullptr, nullptr, alcc);
    P.batch_bytes = plan_batch(pr.data(), pp->K, alcc).total;
    P.batch = take(P.batch_bytes);
    P.total = o + 256;
    return P;
}

}  // namespace

// Redo a problem's set-up for new data in its ybar buffer on the same points
// (affine fit from the stored eigen-decomposition, Bbar, then the shifted
// start); the host constants follow after a sync.
static hipError_t ctx_resetup(cr_ctx* c, hipStream_t cs) {
    const Layout& L = c->L;
    hipError_t e = cr::launch_refit(c->X, c->ybar, c->N, c->n, c->p.gamma, c->D(L.off_su), c->D(L.off_supart),
                                    c->D(L.off_y0), c->D(L.off_xi0), c->st, cs);
    if (e == hipSuccess && c->shift)
        e = cr::launch_setup_shift(c->D(L.off_y0), c->ybar, c->D(L.off_xi0), c->shift, c->N, c->n, c->p.gamma, c->st,
                                   cs);
    return e;
}

// The re-fit of every block problem, one launch per step for all of them
// (the per-problem sequence of ctx_resetup when there are more than
// kMaxRefit blocks).
static bool refit_table(const std::vector<cr_ctx*>& sub, cr::RefitTable& t) {
    if (sub.size() > (size_t)cr::kMaxRefit) return false;
    t = cr::RefitTable{};
    t.K = (int32_t)sub.size();
    for (size_t p = 0; p < sub.size(); ++p) {
        const cr_ctx* c = sub[p];
        const Layout& L = c->L;
        cr::RefitArgs& a = t.p[p];
        a.X = c->X; a.ybar = c->ybar; a.N = c->N; a.n = c->n; a.gamma = c->p.gamma;
        a.su = c->D(L.off_su); a.part = c->D(L.off_supart); a.y0 = c->D(L.off_y0); a.xi0 = c->D(L.off_xi0);
        a.st = c->st; a.shift = c->shift;
    }
    return true;
}


extern "C" {

cr_status cr_papg_workspace_bytes(int64_t N, int32_t n, const cr_params* alcc, const cr_papg_params* pp,
                                  size_t* bytes) {
    std::string msg;
    if (!bytes) return fail(nullptr, CR_ERR_ARG, "bytes is NULL");
    cr_status s = check_papg(N, n, alcc, pp, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    *bytes = papg_layout(N, n, alcc, pp).total;
    return CR_OK;
}

cr_status cr_papg(const void* X_dev, const void* ybar_dev, int64_t N, int32_t n, const cr_params* alcc,
                  const cr_papg_params* pp, void* y_dev, void* xi_dev, void* theta_dev, void* theta_y_dev,
                  double* trace_host, void* workspace_dev, size_t ws_bytes, cr_papg_info* info, void* stream) {
    std::string msg;
    cr_status s = check_papg(N, n, alcc, pp, msg);
    if (s != CR_OK) return fail(nullptr, s, msg);
    if (!X_dev || !ybar_dev || !y_dev || !xi_dev || !workspace_dev)
        return fail(nullptr, CR_ERR_ARG, "X, ybar, y, xi and the workspace must be non-NULL");
    const PapgLayout P = papg_layout(N, n, alcc, pp);
    if (ws_bytes < P.total) return fail(nullptr, CR_ERR_NOMEM, "workspace smaller than cr_papg_workspace_bytes()");
    const auto t0 = std::chrono::steady_clock::now();
    char* ws = (char*)align256((size_t)workspace_dev);
    auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
    hipStream_t us = (hipStream_t)stream;
    const double* X = (const double*)X_dev;
    const double gamma = alcc->gamma;

#define PCHK(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return fail(nullptr, CR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

    // constants: y_shift from ybar's range, L from sigma_max(A2)^2 of all points
    std::vector<double> hy((size_t)N);
    PCHK(hipMemcpyAsync(hy.data(), ybar_dev, (size_t)N * 8, hipMemcpyDeviceToHost, us));
    PCHK(hipStreamSynchronize(us));
    double ymin = hy[0], ymax = hy[0];
    for (double v : hy) {
        if (!std::isfinite(v)) return fail(nullptr, CR_ERR_NONFINITE, "ybar holds NaN or Inf");
        ymin = std::min(ymin, v);
        ymax = std::max(ymax, v);
    }
    const double yshift = pp->y_shift >= 0 ? pp->y_shift : std::max(0.0, ymax - 2.0 * ymin);
    double L = pp->L;
    if (!(L > 0)) {
        cr::DevState hs{};
        PCHK(cr::launch_zero(ws + P.st, (sizeof(cr::DevState) + 15) / 16 * 16, us));
        PCHK(cr::launch_setup(X, (const double*)ybar_dev, N, n, gamma, D(P.su), D(P.supart), D(P.y0), D(P.xi0),
                              reinterpret_cast<cr::DevState*>(ws + P.st), us));
        PCHK(hipMemcpyAsync(&hs, ws + P.st, sizeof(cr::DevState), hipMemcpyDeviceToHost, us));
        PCHK(hipStreamSynchronize(us));
        if (hs.nonfinite || !std::isfinite(hs.sigma2_A2)) return fail(nullptr, CR_ERR_NONFINITE, "X holds NaN or Inf");
        L = (2.0 * (double)N + hs.sigma2_A2 + 1.0) / gamma;
    }

    cr::PapgArgs a{};
    a.N = N; a.Nbar = P.Nbar; a.n = n;
    a.L = L; a.gamma = gamma; a.yshift = yshift;
    a.B = pp->B_theta > 0 ? pp->B_theta : INFINITY;
    a.X = X; a.ybar = (const double*)ybar_dev;
    double* th[2] = {D(P.th[0]), D(P.th[1])};
    double* ty[2] = {D(P.ty[0]), D(P.ty[1])};
    a.ybs = D(P.ybs); a.shift = D(P.shift); a.y = D(P.y); a.xis = D(P.xis);
    a.part = D(P.part); a.cpart = D(P.cpart); a.scal = D(P.scal); a.trace = D(P.trace);
    if (!(pp->L > 0) && pp->power_iters > 0) {
        // sigma_max(C)^2 estimated by power iteration (th[0] and the block-data
        // buffers serve as scratch before they are initialised below)
        a.tc = th[0];
        PCHK(cr::launch_zero(ws + P.pzero, (size_t)N * 8, us));
        PCHK(cr::launch_papg_power(a, D(P.pvy), D(P.pvxi), D(P.pzero), pp->power_iters, us));
        double sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        PCHK(hipMemcpyAsync(sc, a.scal, sizeof(sc), hipMemcpyDeviceToHost, us));
        PCHK(hipStreamSynchronize(us));
        if (!std::isfinite(sc[4]) || !(sc[4] > 0)) return fail(nullptr, CR_ERR_NONFINITE, "power iteration failed");
        L = std::min(L, 1.05 * sc[4] / gamma);
        a.L = L;
    }
    for (int q = 0; q < 2; ++q) {
        PCHK(cr::launch_zero(th[q], (size_t)N * N * 8, us));
        PCHK(cr::launch_zero(ty[q], (size_t)N * 8, us));
    }
    int cur = 0;                 // th[cur] = theta^(1)_{l-1}, th[cur ^ 1] = theta^(1)_{l-2}
    auto set_theta = [&]() { a.tc = th[cur]; a.tp = th[cur ^ 1]; a.tyc = ty[cur]; a.typ = ty[cur ^ 1]; };
    set_theta();
    a.beta = 0.0;
    PCHK(cr::launch_papg_lin(a, us));      // theta^(2)_1 = 0: the blocks' own data, zero centres

    std::vector<cr_problem> pr = papg_problems(N, n, pp->K, X, D(P.ybs), D(P.y), D(P.xis), alcc);
    std::vector<const double*> shifts(pp->K);
    for (int i = 0; i < pp->K; ++i) shifts[i] = D(P.shift) + (int64_t)i * P.Nbar * n;
    cr_batch* b = nullptr;
    s = batch_init_impl(&b, pr.data(), pp->K, alcc, ws + P.batch, P.batch_bytes, stream, shifts.data());
    if (s != CR_OK) return s;
    struct Guard { cr_batch* b; ~Guard() { cr_batch_destroy(b); } } guard{b};
    hipStream_t cs = b->cs;
    hipEvent_t ev = b->ev[0];
#define PBCHK(call)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return bfail(b, CR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
    // everything above ran on the caller's stream: order the batch's stream after it
    PBCHK(hipEventRecord(ev, us));
    PBCHK(hipStreamWaitEvent(cs, ev, 0));

    double t = 1.0;
    int64_t inner = 0;
    cr_status result = CR_OK;
    // Each iteration is enqueued behind the previous one: the block re-set-ups
    // and the block solves' schedules run on the device, so with a fixed block
    // schedule nothing is read back until the end (an adaptive one polls its
    // replays' activity flag).
    const bool fixed_blocks = alcc->inner_iters > 0;
    cr::RefitTable rt;
    const bool batched_refit = refit_table(b->sub, rt);
    for (int l = 1; l <= pp->iters; ++l) {
        if (l > 1) PBCHK(cr::launch_papg_lin(a, cs));
        if (batched_refit) PBCHK(cr::launch_refit_batched(rt, cs));
        else
            for (cr_ctx* c : b->sub) PBCHK(ctx_resetup(c, cs));
        s = cr_batch_start(b);
        if (s != CR_OK) return s;
        int32_t running = 1;
        while (running) {
            s = cr_batch_advance(b, 1 << 30, &running);
            if (s != CR_OK) return s;
        }
        PBCHK(batch_copy_outputs(b));
        b->started = false;
        if (fixed_blocks) {
            inner += (int64_t)pp->K * alcc->max_outer * alcc->inner_iters;
        } else {
            for (cr_ctx* c : b->sub) {
                int64_t ti = 0;
                PBCHK(hipMemcpy(&ti, &c->sched->total_inner, 8, hipMemcpyDeviceToHost));
                inner += ti;
            }
        }
        a.it = l - 1;
        PBCHK(cr::launch_papg_step2(a, cs));
        cur ^= 1;
        set_theta();
        const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        a.beta = pp->method == CR_PAPG_ACCELERATED ? (t - 1.0) / tn : 0.0;
        t = tn;
    }
    PBCHK(cr::launch_papg_out(a, (double*)y_dev, (double*)xi_dev, cs));
    if (theta_dev) PBCHK(hipMemcpyAsync(theta_dev, a.tc, (size_t)N * N * 8, hipMemcpyDeviceToDevice, cs));
    if (theta_y_dev) PBCHK(hipMemcpyAsync(theta_y_dev, a.tyc, (size_t)N * 8, hipMemcpyDeviceToDevice, cs));
    if (trace_host)
        PBCHK(hipMemcpyAsync(trace_host, a.trace, (size_t)pp->iters * 3 * 8, hipMemcpyDeviceToHost, cs));
    double sc[3] = {0, 0, 0};
    PBCHK(hipMemcpyAsync(sc, a.scal, sizeof(sc), hipMemcpyDeviceToHost, cs));
    PBCHK(hipStreamSynchronize(cs));
    // the caller's stream waits for nothing more: the run is host-synchronous
    for (cr_ctx* c : b->sub) {
        cr::AlccSched bs{};
        PBCHK(hipMemcpy(&bs, c->sched, sizeof(bs), hipMemcpyDeviceToHost));
        if (bs.nonfinite) return bfail(b, CR_ERR_NONFINITE, "non-finite block solve");
        if (bs.phase != 2) return bfail(b, CR_ERR_STATE, "a block schedule did not finish");
        if (!fixed_blocks && !bs.converged) result = CR_NOT_CONVERGED;
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->L = L;
        info->y_shift = yshift;
        info->theta_norm = sc[1];
        info->infeas_cross = sc[2];
        info->inner_iters = inner;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!std::isfinite(sc[1])) return fail(nullptr, CR_ERR_NONFINITE, "non-finite multipliers");
    return result;
#undef PCHK
#undef PBCHK
}

}  // extern "C"
