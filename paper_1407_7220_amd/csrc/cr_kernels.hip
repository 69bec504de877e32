// gfx950 kernels of the convex-regression pair engine.
//
// Notation (Aybat & Wang, Sec. II): points x_l (rows of X, N x n), data ybar,
// unknowns y (N) and xi (N x n).  Pair (i, j), i != j, is the constraint
// y_i >= y_j + xi_j^T (x_i - x_j) (eq. "original"); its residual is
//   r_ij = y_i - y_j - xi_j^T x_i + xi_j^T x_j = (A1 y + A2 xi)_(i,j).
// One MAPG iteration (Fig. 4) needs grad P_k (eq. "subproblem"):
//   w_ij = (r_ij - theta_ij)_- = max(theta_ij - r_ij, 0)
//   grad_y P  = (y - ybar)/mu - (rowsum(W) - colsum(W))
//   grad_xi P = (gamma/mu) xi_j + sum_i w_ij x_i - colsum_j(W) x_j
// and the ALCC multiplier step (Fig. 3 step 4) is
//   theta <- (mu_k / mu_{k+1}) max(theta - r, 0).
//
// The pair pass computes r with one MFMA contraction,
//   R = [X 1] [-Xi  c]^T + y 1^T,   c_j = x_j^T xi_j - y_j,
// streams theta once, and reduces W with a second MFMA contraction,
//   C = W^T [X 1]  (columns 0..n-1: sum_i w_ij x_i, column n: colsum_j),
// plus wavefront shuffles for the row sums.  Partial sums leave each
// workgroup once; a separate O(N n) kernel sums them in a fixed order.
#include "cr_device.h"
#include "cr_ops.h"

namespace cr {


// ---------------------------------------------------------------------------
// The fused pair pass (gradient or multiplier step).
//
// Grid (strips, chunks).  Workgroup (s, h) owns the columns
// [16 TW s, 16 TW (s+1)) and the rows [h rpc, (h+1) rpc); its 4 waves take
// alternate 16-row tiles.  Lane (g, c) of a wave covers, for j-tile t and
// accumulator element v, the pair (i0 + rmap(g, v), J0 + TW c + t), so its
// TW theta values of one row are contiguous (one 16-byte load per row).
// ---------------------------------------------------------------------------
// LDS of one pass workgroup: the 4 waves' column-sum accumulators (at most
// 4 x TW x NKB x 4 x 64 elements = 32 KiB in every precision) and 4 x 4 KKT doubles.
constexpr int kPassLds = 32768 + 256;

// Lazy passes place, inside the 32 KiB area, the row sums at [0, R), the y
// operands of the chunk's rows at [R, 2R) (R = rows x element size, 16-byte
// aligned) and the staged column operands at [2R, 2R + kBsBytes): 16 TW
// columns of 33 slots each (k < n: -xi2_jk, k = n: c_j, then zeros).
constexpr int kBsBytes = 64 * kBsStride * 4;   // 16 TW x 33 x element size, either precision
__host__ __device__ constexpr int64_t lazy_rbytes(int64_t rows, int esz) { return (rows * esz + 15) / 16 * 16; }

// Threads per staged column, and k entries per thread (slots 0 .. KCAP - 1).
template <typename Ops> struct LazyShape {
    static constexpr int COLS = 16 * Ops::TW;
    static constexpr int PT = kBlock / COLS;
    static constexpr int KMAX = (Ops::KCAP + PT - 1) / PT;
};

// Operands of a lazy gradient pass (see LazyStep): the y operands of rows
// [I0, I1) into ylds, the column operands of [J0, J0 + 16 TW) into breg, and
// the state and stopping-test pieces that this workgroup owns.  The pieces
// (per-wave sums) go to `stop` (2 x kWaves doubles) for the epilogue.
// The loads that do not depend on the iteration number l go out before the
// activity flag and the replay base (act_v, base_v, vector loads issued by the
// caller) are waited for; returns false, with nothing written, when the flag
// is 0, else sets l.
template <typename Ops>
__device__ bool lazy_operands(const PassArgs& a, const int strip, const int chunk, const int64_t I0, const int64_t I1,
                              const int64_t J0, char* __restrict__ lds, typename Ops::elem* __restrict__ ylds,
                              typename Ops::Breg& breg, const int g, const int c, double* stop, const int act_v,
                              const u32x2 base_v, const int lq, int64_t& l) {
    typedef typename Ops::elem T;
    typedef LazyShape<Ops> S;
    const LazyStep& z = a.lz;
    const int rows = (int)(I1 - I0);
    const int64_t N = a.N;
    const int n = z.n;
    const bool wrows = strip == 0, wcols = chunk == 0;
    const gp<const double> __restrict__ vy = glob(z.vy);
    const gp<const double> __restrict__ vxi = glob(z.vxi);
    const gp<const double> __restrict__ X = glob(z.X);
    const gp<const double> __restrict__ ybar = glob(z.ybar);
    const gp<double> __restrict__ y2 = glob(z.y2);
    const gp<double> __restrict__ xi2 = glob(z.xi2);

    // Loads independent of l (column j = J0 + jj, k = r0 + PT e; the first
    // rows; the first records of the norm pieces; the ball radii), all in
    // flight together with the flag and the base.
    const int jj = threadIdx.x / S::PT, r0 = threadIdx.x % S::PT;
    const int64_t j = J0 + jj;
    const bool vj = j < N;
    double cv[S::KMAX], cx[S::KMAX], co[S::KMAX];
#pragma unroll
    for (int e = 0; e < S::KMAX; ++e) {
        const int k = r0 + S::PT * e;
        cv[e] = cx[e] = co[e] = 0.0;
        if (vj && k < n) {
            const int64_t q = j * n + k;
            cv[e] = vxi[q]; cx[e] = X[q];
            if (wcols) co[e] = xi2[q];
        }
    }
    double jv = 0.0, jb = 0.0;
    if (vj) { jv = vy[j]; jb = ybar[j]; }
    constexpr int RB = 3;      // rows per thread loaded with the first batch (768-row chunks in one round trip)
    double rv[RB], rb[RB], ro[RB];
#pragma unroll
    for (int e = 0; e < RB; ++e) {
        const int r = threadIdx.x + kBlock * e;
        const int64_t i = I0 + r;
        rv[e] = rb[e] = ro[e] = 0.0;
        if (r < rows && i < N) {
            rv[e] = vy[i]; rb[e] = ybar[i];
            if (wrows) ro[e] = y2[i];
        }
    }
    double u0[4], u1[4];
    gather_issue<1>(z.npart, z.nblk, 0, 1, u0, u1);
    const gp<const OuterArgs> oa = glob(z.oa);
    const double By = oa->By, Bxi = oa->Bxi;
    __builtin_amdgcn_sched_barrier(0);

    if (uniform(act_v) == 0) return false;
    l = z.lfix > 0 ? (int64_t)z.lfix : uniform(base_v) + lq + 1;
    if (l <= 1) {
        // first iteration of the run: the operands k_set_point wrote
        const gp<const T> yc = glob((const T*)a.ycol + I0);
        for (int r = threadIdx.x; r < rows; r += kBlock) ylds[r] = yc[r];
        Ops::load_breg(breg, a, J0 + Ops::TW * c, g);
        __syncthreads();
        return true;
    }
    const int par = (int)(l & 1);                        // y1_{l-2} in y1p[l & 1]
    const gp<const double> __restrict__ y1in = glob((const double*)z.y1p[par]);
    const gp<const double> __restrict__ xi1in = glob((const double*)z.xi1p[par]);
    const gp<double> __restrict__ y1out = glob(z.y1p[par ^ 1]);
    const gp<double> __restrict__ xi1out = glob(z.xi1p[par ^ 1]);
    double cp[S::KMAX];
#pragma unroll
    for (int e = 0; e < S::KMAX; ++e) {
        const int k = r0 + S::PT * e;
        cp[e] = vj && k < n ? xi1in[j * n + k] : 0.0;
    }
    const double jp = vj ? y1in[j] : 0.0;
    double rp[RB];
#pragma unroll
    for (int e = 0; e < RB; ++e) {
        const int r = threadIdx.x + kBlock * e;
        const int64_t i = I0 + r;
        rp[e] = r < rows && i < N ? y1in[i] : 0.0;
    }
    const double beta = glob(z.beta)[l - 1];         // (t_{l-1} - 1) / t_l

    // Fig. 4 steps 1-2 of iteration l - 1: the ball projections' scales
    double ny2, nx2;
    gather_finish<1>(z.npart, z.nblk, 0, 1, u0, u1, ny2, nx2);
    const double ny = sqrt(ny2), nx = sqrt(nx2);
    const bool py = ny > By, px = nx > Bxi;
    const double sy = py ? By / ny : 1.0, sx = px ? Bxi / nx : 1.0;
    double dy = 0.0, dx = 0.0;

    // columns: -xi2_jk, and c_j = x_j^T xi2_j - y2_j from the PT threads' products
    // (with a slope shift, both from the constraint slope xi2 + c)
    T* Bs = reinterpret_cast<T*>(lds + 2 * lazy_rbytes(rows, (int)sizeof(T)));
    T* brow = Bs + jj * kBsStride;
    double prod = 0.0;
#pragma unroll
    for (int e = 0; e < S::KMAX; ++e) {
        const int k = r0 + S::PT * e;
        if (k < n) {
            const double x1 = px ? sx * cv[e] : cv[e];          // projection onto Q_xi
            const double x2n = x1 + beta * (x1 - cp[e]);        // extrapolation
            const double xo = z.shift && vj ? x2n + glob(z.shift)[j * n + k] : x2n;
            prod += cx[e] * xo;
            brow[k] = vj ? (T)(-xo) : (T)0;
            if (wcols && vj) {
                const int64_t q = j * n + k;
                dx += (x1 - co[e]) * (x1 - co[e]);
                xi1out[q] = x1;
                xi2[q] = x2n;
            }
        }
    }
    for (int k = n + 1 + r0; k < kBsStride; k += S::PT) brow[k] = (T)0;
    prod = lane_group_sum<S::PT>(prod);
    {
        const double y1 = py ? jb + sy * (jv - jb) : jv;
        const double y2j = y1 + beta * (y1 - jp);
        if (r0 == 0) brow[n] = vj ? (T)(prod - y2j) : (T)0;
    }

    // rows: y2_i, and the state of this workgroup's rows when it owns them
    auto row = [&](int r, double v, double b, double p, double o) {
        const int64_t i = I0 + r;
        T yv = (T)0;
        if (i < N) {
            const double y1 = py ? b + sy * (v - b) : v;       // projection onto Q_y
            const double y2n = y1 + beta * (y1 - p);
            yv = (T)y2n;
            if (wrows) {
                dy += (y1 - o) * (y1 - o);
                y1out[i] = y1;
                y2[i] = y2n;
            }
        }
        ylds[r] = yv;
    };
#pragma unroll
    for (int e = 0; e < RB; ++e) {
        const int r = threadIdx.x + kBlock * e;
        if (r < rows) row(r, rv[e], rb[e], rp[e], ro[e]);
    }
    // taller chunks: the further rows RB at a time, each batch's loads together
    for (int q0 = threadIdx.x + kBlock * RB; q0 < rows; q0 += kBlock * RB) {
        double v[RB], b[RB], p[RB], o[RB];
#pragma unroll
        for (int e = 0; e < RB; ++e) {
            const int r = q0 + kBlock * e;
            const int64_t i = I0 + r;
            v[e] = b[e] = p[e] = o[e] = 0.0;
            if (r < rows && i < N) {
                v[e] = vy[i]; b[e] = ybar[i]; p[e] = y1in[i];
                if (wrows) o[e] = y2[i];
            }
        }
#pragma unroll
        for (int e = 0; e < RB; ++e) {
            const int r = q0 + kBlock * e;
            if (r < rows) row(r, v[e], b[e], p[e], o[e]);
        }
    }
    if (wrows || wcols) {
        dy = wave_sum(dy);
        dx = wave_sum(dx);
        if ((threadIdx.x & 63) == 0) { stop[threadIdx.x >> 6] = dy; stop[kWaves + (threadIdx.x >> 6)] = dx; }
    }
    __syncthreads();
    Ops::load_breg_lds(breg, Bs, Ops::TW * c, g, n);
    return true;
}

// lq: replay position of a lazy gradient pass (LazyStep).  The workgroup
// returns after issuing its first tile loads when the activity flag is 0 (the
// flag and the replay base are read together with those loads, so that the
// pass's start waits on one round trip instead of three).  With
// a.check_first (batched adaptive runs, where many problems sit frozen for
// most of a solve) it returns before any tile load instead, so that a frozen
// problem's workgroups cost no memory traffic.
template <typename Ops, int THETA_MODE, int LAZY = 0>
__device__ void pair_pass_item(const PassArgs& a, const int strip, const int chunk, const int nstrips,
                               char* __restrict__ lds, const int lq) {
    typedef typename Ops::elem T;
    typedef typename Ops::acc_t acc_t;
    constexpr int TW = Ops::TW;
    constexpr int NKB = Ops::NKB;
    constexpr int EV = 16 / (int)sizeof(T);
    // check_first: a plain (scalar) read of the flag before anything else, the
    // cheapest exit for the many workgroups of frozen problems
    if (a.check_first && *a.active == 0) return;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t J0 = (int64_t)strip * (16 * TW);
    const int64_t I0 = (int64_t)chunk * a.rows_per_chunk;
    const int64_t I1 = min(I0 + (int64_t)a.rows_per_chunk, a.Nrow);
    const int64_t jl = J0 + TW * c;
    const T* __restrict__ ycol = (const T*)a.ycol;
    T* __restrict__ theta = (T*)a.theta;
    constexpr bool theta_mode = THETA_MODE != 0;
    // row sums of the chunk, staged in the column-sum area (free until the epilogue)
    T* srow = reinterpret_cast<T*>(lds);
    static_assert(kMaxRowsPerChunk * 8 <= 32768, "row staging");

    // lazy passes: y operands of the chunk's rows in LDS, after the row sums
    T* ylds = reinterpret_cast<T*>(lds + lazy_rbytes(I1 - I0, (int)sizeof(T)));
    double* stop = reinterpret_cast<double*>(lds + 32768);
    typename Ops::Breg breg;
    if constexpr (!LAZY) Ops::load_breg(breg, a, jl, g);

    acc_t cacc[TW][NKB];
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) cacc[t][kb] = acc_t{0, 0, 0, 0};

    double k_rneg_max = 0.0, k_rneg_sq = 0.0, k_wr_max = 0.0, k_wr_sum = 0.0;
    double theta_scale = 0.0;
    if constexpr (theta_mode) theta_scale = a.theta_scale_p ? *glob(a.theta_scale_p) : a.theta_scale;

    constexpr int64_t step = 16 * kWaves;
    constexpr int NSET = Ops::NSET;   // staging sets (tiles in flight per wave)
    // Tiles of this wave: rows I0 + 16 wave + step m < I1 (at least one, since
    // I1 - I0 >= 64).  Prefetches are unconditional (past the last tile they
    // read zeros from the buffer views), so the compiler can count
    // outstanding loads exactly.
    const int64_t first = I0 + 16 * wave;
    const int ntile = (int)((I1 - first + step - 1) / step);
    auto row_of = [&](int m) { return first + step * (int64_t)m; };

    // Operands of one 16-row tile: packed X (L2-resident), y_i, and the
    // wave's 16 x 16TW block of theta (HBM stream).  NSET register sets rotate
    // so that each tile's loads are issued NSET - 1 tiles ahead of its use.
    // Buffer views of this workgroup's rows: the per-lane offsets are fixed,
    // tile m of the wave adds m times a per-view scalar step, and the loads
    // past the last tile return zeros.
    const uint32_t rows = (uint32_t)(I1 - I0);
    const uint32_t row_bytes = (uint32_t)a.ld * (uint32_t)sizeof(T);
    const rsrc_t th_r = make_rsrc(theta + I0 * a.ld + J0, rows * row_bytes);
    const rsrc_t xp_r = make_rsrc((const char*)a.xp + (I0 >> 4) * 64 * Ops::XPB, (rows >> 4) * 64u * Ops::XPB);
    const rsrc_t y_r = make_rsrc(ycol + I0, rows * (uint32_t)sizeof(T));
    uint32_t th_vo[4], y_vo[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        th_vo[v] = (uint32_t)(16 * wave + orow<Ops>(g, v)) * row_bytes + (uint32_t)(TW * c) * (uint32_t)sizeof(T);
        y_vo[v] = (uint32_t)(16 * wave + orow<Ops>(g, v)) * (uint32_t)sizeof(T);
    }
    const uint32_t xp_vo = (uint32_t)(wave * 64 + lane) * (uint32_t)Ops::XPB;
    const uint32_t th_step = 16u * kWaves * row_bytes;
    const uint32_t xp_step = (uint32_t)kWaves * 64u * (uint32_t)Ops::XPB;
    const uint32_t y_step = 16u * kWaves * (uint32_t)sizeof(T);
    auto load_tile = [&](int m, typename Ops::Xop& xop, T* yv, V16<T>* th) {
        const uint32_t mm = (uint32_t)m;
        Ops::load_xop_b(xop, xp_r, xp_vo, mm * xp_step);
        if constexpr (LAZY) {
            (void)yv;
        } else if (sizeof(T) == 4) {
            // rows 4g .. 4g + 3 of the tile
            V16<T> tv = bld16<T>(y_r, y_vo[0], mm * y_step);
#pragma unroll
            for (int e = 0; e < 4; ++e) yv[e] = tv.v[e];
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) yv[v] = (T)bld8(y_r, y_vo[v], mm * y_step);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) th[v] = bld16<T>(th_r, th_vo[v], mm * th_step);
    };

    auto process = [&](const int m, const typename Ops::Xop& xop, const T* yv, const V16<T>* th) {
        const int64_t i0 = row_of(m);
        // residual tiles R_t
        acc_t R[TW];
        if constexpr (LAZY) {
            T yl[4];
            const T* yr = ylds + (i0 - I0);
            if (sizeof(T) == 4) {
                const V16<T> tv = *reinterpret_cast<const V16<T>*>(yr + 4 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e) yl[e] = tv.v[e];
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) yl[v] = yr[orow<Ops>(g, v)];
            }
            Ops::residual(R, xop, breg, yl);
        } else {
            Ops::residual(R, xop, breg, yv);
        }

        // w = max(theta - r, 0); explicit zero off the constraint set
        T W[TW][4];
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T d = th[v].v[t] - R[t][v];
                W[t][v] = d > (T)0 ? d : (T)0;
            }
        const bool edge = (i0 < J0 + 16 * TW && i0 + 16 > J0) || (J0 + 16 * TW > a.N) || (i0 + 16 > a.N);
        // tile-relative 32-bit indices: pair (i0 + r, J0 + q) is a constraint
        // iff r < rlim, q < qlim and r + dij != q
        const int rlim = (int)min((int64_t)16, a.N - i0);
        const int qlim = (int)min((int64_t)(16 * TW), a.N - J0);
        const int dij = (int)max((int64_t)-64, min((int64_t)64, i0 - J0));   // |i0 - J0| >= 64: no diagonal
        if (edge) {
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = orow<Ops>(g, v), q = TW * c + t;
                    if (!(r < rlim && q < qlim && r + dij != q)) W[t][v] = (T)0;
                }
        }

        if constexpr (theta_mode) {
            // Fig. 3 step 4 in place, and the pair terms of the KKT residual
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                V16<T> o;
#pragma unroll
                for (int t = 0; t < TW; ++t) o.v[t] = (T)(theta_scale * (double)W[t][v]);
                st16(theta + (i0 + orow<Ops>(g, v)) * a.ld + jl, o);
            }
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = orow<Ops>(g, v), q = TW * c + t;
                    if (r < rlim && q < qlim && r + dij != q) {
                        const double r = (double)R[t][v];
                        const double rn = r < 0.0 ? -r : 0.0;
                        const double wr = (double)W[t][v] * r;
                        k_rneg_max = fmax(k_rneg_max, rn);
                        k_rneg_sq += rn * rn;
                        k_wr_max = fmax(k_wr_max, fabs(wr));
                        k_wr_sum += wr;
                    }
                }
        }

        Ops::colsums(cacc, W, xop);

        // row sums over this workgroup's columns: the TW j-tiles in the lane,
        // then the 16 lanes of the row group by exchange (lane c ends with row
        // orow(g, c >> 2))
        T rs4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            T s = W[0][v];
#pragma unroll
            for (int t = 1; t < TW; ++t) s += W[t][v];
            rs4[v] = s;
        }
        const T rsum = row16_sum4(rs4, c);
        if ((c & 3) == 0) {
            // staged in LDS (no global store inside the tile loop, so that the
            // prefetched loads stay in flight across iterations); written once
            // per workgroup after the loop
            srow[(i0 - I0) + orow<Ops>(g, c >> 2)] = rsum;
        }
    };

    typename Ops::Xop xs[NSET];
    T ys[NSET][4];
    V16<T> ts[NSET][4];
    // The scheduling barriers keep each staging set's loads together and in
    // program order, so the prologue leaves the same pending-load sequence as
    // the loop's back edge; otherwise the wait-count merge at the loop head
    // drains nearly every prefetched load once per NSET tiles.
    const int act_v = vld_i32(a.active);
    u32x2 base_v = {0u, 0u};
    if constexpr (LAZY) base_v = vld_i64(&a.lz.st->base);
    __builtin_amdgcn_sched_barrier(0);
    int64_t l = 0;
    if constexpr (LAZY) {
        // one tile in flight during the operand set-up (more would spill)
        load_tile(0, xs[0], ys[0], ts[0]);
        __builtin_amdgcn_sched_barrier(0);
        if (!lazy_operands<Ops>(a, strip, chunk, I0, I1, J0, lds, ylds, breg, g, c, stop, act_v, base_v, lq, l)) return;
#pragma unroll
        for (int b = 1; b < NSET; ++b) {
            load_tile(b, xs[b], ys[b], ts[b]);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int b = 0; b < NSET; ++b) {
            load_tile(b, xs[b], ys[b], ts[b]);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (uniform(act_v) == 0) return;
    }
#pragma nounroll
    for (int m = 0; m < ntile; m += NSET) {
#pragma unroll
        for (int b = 0; b < NSET; ++b) {
            if (m + b < ntile) process(m + b, xs[b], ys[b], ts[b]);
            __builtin_amdgcn_sched_barrier(0);
            load_tile(m + b + NSET, xs[b], ys[b], ts[b]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // rowpart[strip][i] of this chunk's rows, from the LDS staging area
    __syncthreads();
    if constexpr (LAZY) {
        if (threadIdx.x == 0 && l > 1 && (strip == 0 || chunk == 0)) {
            double sy2 = stop[0], sx2 = stop[kWaves];
            for (int w = 1; w < kWaves; ++w) { sy2 += stop[w]; sx2 += stop[kWaves + w]; }
            if (strip == 0) glob(a.lz.spart)[chunk] = sy2;
            if (chunk == 0) glob(a.lz.spart)[a.lz.chunks + strip] = sx2;
        }
    }
    {
        const gp<T> dst = glob((T*)a.rowpart + (int64_t)strip * a.Nrow + I0);
        for (int r = threadIdx.x; r < (int)(I1 - I0); r += kBlock) dst[r] = srow[r];
    }
    __syncthreads();

    // Combine the 4 waves' column sums (fixed order) and write this chunk's partial.
    static_assert(sizeof(T) * kWaves * TW * NKB * 4 * 64 <= 32768, "pass LDS");
    typedef T cl_t[TW][NKB][4][64];
    cl_t* cl = reinterpret_cast<cl_t*>(lds);
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) cl[wave][t][kb][v][lane] = cacc[t][kb][v];
    __syncthreads();
    const gp<T> cpart = glob((T*)a.cpart);
    for (int e = threadIdx.x; e < TW * NKB * 4 * 64; e += kBlock) {
        const int ln = e & 63, v = (e >> 6) & 3, rest = e >> 8;
        const int kb = rest % NKB, t = rest / NKB;
        const T s = ((cl[0][t][kb][v][ln] + cl[1][t][kb][v][ln]) + cl[2][t][kb][v][ln]) + cl[3][t][kb][v][ln];
        const int64_t j = J0 + TW * orow<Ops>(ln >> 4, v) + t;
        const int kk = 16 * kb + (ln & 15);
        // cpart[chunk][j][k]: this workgroup's columns are one contiguous range
        if (kk < a.nc) cpart[((int64_t)chunk * a.ld + j) * a.nc + kk] = s;
    }

    if constexpr (theta_mode) {
        double (*kr)[kWaves] = reinterpret_cast<double (*)[kWaves]>(lds + 32768);
        double q0 = wave_max(k_rneg_max), q1 = wave_sum(k_rneg_sq);
        double q2 = wave_max(k_wr_max), q3 = wave_sum(k_wr_sum);
        if (lane == 0) { kr[0][wave] = q0; kr[1][wave] = q1; kr[2][wave] = q2; kr[3][wave] = q3; }
        __syncthreads();
        if (threadIdx.x == 0) {
            const gp<double> o = glob(a.kktpart + ((int64_t)chunk * nstrips + strip) * 4);
            double m0 = kr[0][0], s1 = kr[1][0], m2 = kr[2][0], s3 = kr[3][0];
            for (int w = 1; w < kWaves; ++w) {
                m0 = fmax(m0, kr[0][w]); s1 += kr[1][w]; m2 = fmax(m2, kr[2][w]); s3 += kr[3][w];
            }
            o[0] = m0; o[1] = s1; o[2] = m2; o[3] = s3;
        }
    }
}

// WAVES: minimum waves per SIMD the register allocation must allow (the
// largest count at which the gradient pass of the class needs no spills:
// 4 for FP32 with KS <= 3, 3 for FP32 KS = 4 and FP64 KS <= 4, 2 otherwise).
template <typename Ops, int THETA_MODE, int WAVES, int LAZY = 0>
__global__ __launch_bounds__(kBlock, WAVES) void k_pair_pass(PassArgs a) {
    __shared__ __align__(16) char lds[kPassLds];
    pair_pass_item<Ops, THETA_MODE, LAZY>(a, blockIdx.x, blockIdx.y, gridDim.x, lds, a.lz.q);
}

// Batched pass: workgroup b takes item b of the (problem, strip, chunk) list
// and returns after its first loads when that problem's MAPG has stopped.  Each item is one
// workgroup tile of the single-problem pass; LAZY gradient passes complete
// each problem's previous MAPG step (LazyStep of its table entry, replay
// position q).  (A persistent grid walking the items held some 20-40 more
// VGPRs per lane across its item loop, which cost a wave per SIMD.)
struct BatchItem { int32_t p, strip, chunk, pad; };

template <typename T, int KS, int THETA_MODE, int WAVES, int LAZY = 0>
__global__ __launch_bounds__(kBlock, WAVES) void k_pair_pass_batched(const PassArgs* __restrict__ args,
                                                              const int32_t* __restrict__ nstrips_of_p,
                                                              const BatchItem* __restrict__ items, int q) {
    __shared__ __align__(16) char lds[kPassLds];
    const BatchItem item = items[blockIdx.x];
    const PassArgs& a = args[item.p];
    pair_pass_item<PlainOps<T, KS>, THETA_MODE, LAZY>(a, item.strip, item.chunk, nstrips_of_p[item.p], lds, q);
}

// A group of G lanes (G >= n + 1, a power of two dividing 64) owns one point j:
// lane k < n handles xi_jk, lane n handles y_j; the partial sums of point j are
// contiguous, so every group reads them with unit stride.
// Sum (op 0) or max (op 1) of field q of the first `count` 4-double records,
// by all threads of the block in a fixed order.
__device__ double block_gather(const double* part, int count, int q, int op) {
    double v = 0.0;
    for (int b = threadIdx.x; b < count; b += kBlock) {
        const double x = ld_coherent(part + (int64_t)b * 4 + q);
        v = op == 0 ? v + x : fmax(v, x);
    }
    return block_reduce(v, op);
}

// a.check_first: return before loading partial sums when the problem is
// frozen (see pair_pass_item).
template <typename T, int G>
__device__ void reduce_block(const ReduceArgs& a, const int blk, const int nblk) {
    // The activity flag, the gate and the replay base are read together with
    // the partial sums (every load below stays inside its array), and the
    // block returns once they arrive if there is nothing to do: the kernel's
    // start then waits on one round trip of loads instead of two.
    DevState* st = a.st;
    const bool m0 = a.mode == 0;
    if (a.check_first && ((m0 && st->active == 0) || (a.gate && *a.gate == 0))) return;
    const int act_v = vld_i32(&st->active, m0);
    const u32x2 base_v = vld_i64(&st->base, m0);
    const int gate_v = vld_i32(a.gate, a.gate != nullptr);
    // mu, gamma and the block steps (the first four fields of OuterArgs) where
    // they come from the device schedule
    const bool use_oa = m0 || a.mu_dev;
    const rsrc_t oar = make_rsrc(a.oa, use_oa ? 32u : 0u);
    const V16<double> o01 = bld16<double>(oar, 0, 0), o23 = bld16<double>(oar, 16, 0);
    __builtin_amdgcn_sched_barrier(0);
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t j = (int64_t)blk * PER + threadIdx.x / G;
    const bool valid = j < a.N;
    const T* rowpart = (const T*)a.rowpart;
    const T* cpart = (const T*)a.cpart;
    const int n = a.n, nc = a.nc;
    // Every load of this point first, so that they are in flight together.
    // Lane k of a point sums the strips k, k + G, ... and (k < n + 1) column k
    // over the chunks, each in index order.  Buffer views of 12 strips x G (16
    // chunks) per batch: entries past the last strip (chunk) read as zeros, so
    // there is no per-entry branch.  One batch covers 192 strips at G = 16 (N up
    // to 6144 in FP64, 12288 otherwise).  The strip sums are loaded by thread
    // (point t % PER, strip group t / PER), so that the threads of a wave read
    // whole runs of consecutive points of a few strips, and handed to lane k of
    // their point through LDS.
    constexpr int URS = 12, UCK = 16;
    const int p = (threadIdx.x & 63) / G;
    const int64_t j0 = __builtin_amdgcn_readfirstlane((int)(j - p));   // the same in every lane of the wave
    const int64_t jb = (int64_t)blk * PER;                             // the block's first point
    const int pr = threadIdx.x % PER, kr = threadIdx.x / PER;
    const uint32_t rvo = ((uint32_t)kr * (uint32_t)a.Nrow + (uint32_t)pr) * (uint32_t)sizeof(T);
    const uint32_t rso = (uint32_t)G * (uint32_t)a.Nrow * (uint32_t)sizeof(T);
    const uint32_t cvo = ((uint32_t)p * (uint32_t)nc + (uint32_t)k) * (uint32_t)sizeof(T);
    const uint32_t cso = (uint32_t)(a.ld * nc) * (uint32_t)sizeof(T);
    auto rs_view = [&](int s0) {
        const uint64_t rem = (uint64_t)(a.strips - s0) * (uint64_t)a.Nrow * sizeof(T);
        return make_rsrc(rowpart + (int64_t)s0 * a.Nrow + jb, (uint32_t)min(rem, (uint64_t)0xffffffffu));
    };
    auto ck_view = [&](int h0) {
        const uint64_t rem = (uint64_t)(a.chunks - h0) * (uint64_t)(a.ld * nc) * sizeof(T);
        return make_rsrc(cpart + ((int64_t)h0 * a.ld + j0) * nc, (uint32_t)min(rem, (uint64_t)0xffffffffu));
    };
    // Block 0 takes the stopping decision of iteration l - 1 (below); the
    // first record of each of its two sums is loaded here with the rest.
    const bool may_decide = a.mode == 0 && blk == 0;
    const int tid = threadIdx.x;
    const int d0 = a.spart ? a.chunks : nblk, d1 = a.spart ? a.strips : nblk;
    const rsrc_t dr = make_rsrc(a.spart ? (const double*)a.spart : a.blockpart,
                                may_decide ? (uint32_t)(a.spart ? (d0 + d1) * 8 : nblk * 32) : 0u);
    const uint32_t t0 = (uint32_t)min(tid, d0 - 1), t1 = (uint32_t)min(tid, d1 - 1);
    const double x0 = bld8(dr, a.spart ? 8 * t0 : 8 * (4 * t0 + 2), 0);
    const double x1 = bld8(dr, a.spart ? 8 * (d0 + t1) : 8 * (4 * t1 + 3), 0);
    // first batches and the point's own values, all issued before any sum
    T ur[URS], uc[UCK];
    {
        const rsrc_t r = rs_view(0), c = ck_view(0);
#pragma unroll
        for (int e = 0; e < URS; ++e) ur[e] = bld_t<T>(r, rvo, (uint32_t)e * rso);
#pragma unroll
        for (int e = 0; e < UCK; ++e) uc[e] = bld_t<T>(c, cvo, (uint32_t)e * cso);
    }
    const int64_t jc = valid ? j : a.N - 1;
    const int kk = min(k, n - 1);
    const double y_l = glob(a.y)[jc], yb_l = glob(a.ybar)[jc], x_l = glob(a.X)[jc * n + kk];
    const double xi_l = glob(a.xi)[jc * n + kk];
    __builtin_amdgcn_sched_barrier(0);   // keeps the loads above ahead of the test
    if ((m0 && uniform(act_v) == 0) || (a.gate && uniform(gate_v) == 0)) return;
    const int64_t l = a.mode == 0 ? uniform(base_v) + a.q + 1 : 0;
    const bool decide = may_decide && l > 1;
    const double mu = use_oa ? o01.v[0] : a.mu, gamma = m0 ? o01.v[1] : a.gamma;
    const double sy = m0 ? o23.v[0] : 0.0, sxi = m0 ? o23.v[1] : 0.0;
    double rs = 0.0, ck = 0.0;
#pragma unroll
    for (int e = 0; e < URS; ++e) rs += (double)ur[e];
    for (int s0 = G * URS; s0 < a.strips; s0 += G * URS) {
        const rsrc_t r = rs_view(s0);
#pragma unroll
        for (int e = 0; e < URS; ++e) ur[e] = bld_t<T>(r, rvo, (uint32_t)e * rso);
#pragma unroll
        for (int e = 0; e < URS; ++e) rs += (double)ur[e];
    }
    {
        // (point pr, strips kr + G m) -> lane kr of point pr
        __shared__ double rsl[kBlock];
        rsl[kr * PER + pr] = rs;
        __syncthreads();
        rs = rsl[k * PER + threadIdx.x / G];
    }
#pragma unroll
    for (int e = 0; e < UCK; ++e) ck += (double)uc[e];
    for (int h0 = UCK; h0 < a.chunks; h0 += UCK) {
        const rsrc_t c = ck_view(h0);
#pragma unroll
        for (int e = 0; e < UCK; ++e) uc[e] = bld_t<T>(c, cvo, (uint32_t)e * cso);
#pragma unroll
        for (int e = 0; e < UCK; ++e) ck += (double)uc[e];
    }
    if (k >= nc) ck = 0.0;
    const bool own_y = valid && k == n, own_x = valid && k < n;
    const double yj = own_y ? y_l : 0.0, ybj = own_y ? yb_l : 0.0;
    const double xjk = own_x ? x_l : 0.0, xik = own_x ? xi_l : 0.0;
    if (decide) {
        // Fig. 4 steps 6-9 for the previous iteration l - 1, from the pieces
        // that this iteration's lazy pass (spart: chunks y pieces, then strips
        // xi pieces) or k_update (fields 2, 3 of its block records) left.
        // Block 0 decides; the other blocks go on, since nothing reads this
        // step's output once MAPG has stopped.
        double g0 = tid < d0 ? x0 : 0.0, g1 = tid < d1 ? x1 : 0.0;
        for (int b = tid + kBlock; b < max(d0, d1); b += kBlock) {
            if (b < d0) g0 += a.spart ? glob(a.spart)[b] : glob(a.blockpart)[(int64_t)b * 4 + 2];
            if (b < d1) g1 += a.spart ? glob(a.spart)[d0 + b] : glob(a.blockpart)[(int64_t)b * 4 + 3];
        }
        double dy2 = g0, dx2 = g1;
        block_sum2(dy2, dx2);
        const double dy = sqrt(dy2), dxi = sqrt(dx2);
        const gp<const OuterArgs> oa = glob(a.oa);
        const bool alpha_stop = oa->adaptive && dy <= oa->alpha_y && dxi <= oa->alpha_xi;
        if ((alpha_stop || l - 1 >= oa->lmax) && threadIdx.x == 0) {
            const gp<DevState> sg = glob(st);
            sg->active = 0;
            sg->it = l - 1;
            sg->stopped_by_alpha = alpha_stop ? 1 : 0;
            sg->dy = dy;
            sg->dxi = dxi;
        }
    }
    rs = group_sum<G>(rs);
    const int base = (threadIdx.x & 63) & ~(G - 1);
    const double cs = __shfl(ck, base + n);      // colsum_j = sum_i w_ij
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    bool bad = false;
    if (valid && k == n) {
        if (a.mode == 0) {
            const double gy = (yj - ybj) / mu - rs + cs;
            const double vy = yj - sy * gy;
            glob(a.out_y)[j] = vy;
            acc0 = (vy - ybj) * (vy - ybj);
        } else if (a.mode == 1) {
            glob(a.out_y)[j] = (yj - ybj) / mu - rs + cs;
        } else {
            const double sty = yj - ybj - mu * (rs - cs);
            if (a.out_y) glob(a.out_y)[j] = sty;
            acc0 = fabs(sty);
            acc2 = (yj - ybj) * (yj - ybj);
            bad = !isfinite(yj);
        }
    } else if (valid && k < n) {
        const double aw = ck - cs * xjk;          // -(A2^T w)_jk
        if (a.mode == 0) {
            const double gx = (gamma / mu) * xik + aw;
            const double vx = xik - sxi * gx;
            glob(a.out_xi)[j * n + k] = vx;
            acc1 = vx * vx;
        } else if (a.mode == 1) {
            glob(a.out_xi)[j * n + k] = (gamma / mu) * xik + aw;
        } else {
            const double stx = gamma * xik + mu * aw;
            if (a.out_xi) glob(a.out_xi)[j * n + k] = stx;
            acc1 = fabs(stx);
            acc3 = xik * xik;
            bad = !isfinite(xik);
        }
    }
    if (a.mode == 1) return;
    if (a.mode == 0) {
        // per-block pieces of ||v_y - ybar||^2 and ||v_xi||^2; k_update combines them
        block_sum2(acc0, acc1);
        if (threadIdx.x == 0) { glob(a.blockpart)[blk * 4 + 0] = acc0; glob(a.blockpart)[blk * 4 + 1] = acc1; }
        return;
    }
    // mode 2: KKT residuals of the multiplier step
    const double b0 = block_reduce(acc0, 1), b1 = block_reduce(acc1, 1);
    const double b2 = block_reduce(acc2, 0), b3 = block_reduce(acc3, 0);
    const double bb = block_reduce(bad ? 1.0 : 0.0, 1);
    if (threadIdx.x == 0) {
        glob(a.blockpart)[blk * 4 + 0] = b0;
        glob(a.blockpart)[blk * 4 + 1] = b1;
        glob(a.blockpart)[blk * 4 + 2] = b2;
        glob(a.blockpart)[blk * 4 + 3] = bb > 0.0 ? INFINITY : b3;
    }
    if (last_block(&st->cnt[1], (unsigned int)nblk)) {
        const double m0 = block_gather(a.blockpart, nblk, 0, 1);
        const double m1 = block_gather(a.blockpart, nblk, 1, 1);
        const double s2 = block_gather(a.blockpart, nblk, 2, 0);
        const double s3 = block_gather(a.blockpart, nblk, 3, 0);
        const double p0 = block_gather(a.kktpart, a.npass, 0, 1);
        const double p1 = block_gather(a.kktpart, a.npass, 1, 0);
        const double p2 = block_gather(a.kktpart, a.npass, 2, 1);
        const double p3 = block_gather(a.kktpart, a.npass, 3, 0);
        if (threadIdx.x == 0) {
            st->stat_y = m0;
            st->stat_xi = m1;
            st->obj = 0.5 * s2;
            st->xi_sq = s3;
            st->infeas = p0;
            st->infeas_sq = p1;
            st->compl_ = mu * p2;
            st->gap = mu * p3;
            st->iterate_nonfinite = isfinite(m0) && isfinite(m1) && isfinite(s2) && isfinite(s3) ? 0 : 1;
        }
    }
}

// ---------------------------------------------------------------------------
// MAPG step completion (Fig. 4 steps 1-9): ball projections, momentum,
// stopping test, and the pass-precision operands of the next pass.
// ---------------------------------------------------------------------------

// Pass operands of column j from xi2 (value of lane k) and c_j.  Plain: the
// pass-precision slots [-xi, c, 0..].  Mixed: BF16 slots -xi_hi at k and n + k,
// -xi_lo at 2n + k, and c_j in FP32.
__device__ __forceinline__ void bf16_split(float v, __bf16& hi, __bf16& lo) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

template <typename T, int G, int MIX, bool CHECK_FIRST = false>
__device__ void update_block(const UpdateArgs& a, const int blk, const int nblk) {
    // Everything that does not depend on the iteration number is loaded with
    // the activity flag and the replay base (the point's state, the norm pieces
    // of up to 4096 reduce blocks, the ball radii), before the first wait.
    DevState* st = a.st;
    if (CHECK_FIRST && st->active == 0) return;
    const int act_v = vld_i32(&st->active);
    const u32x2 base_v = vld_i64(&st->base);
    __builtin_amdgcn_sched_barrier(0);
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t j = (int64_t)blk * PER + threadIdx.x / G;
    const bool valid = j < a.N;
    const int n = a.n;
    // branch-free: every lane loads its point's y entries (one address per
    // point) and its xi entries at a clamped index, then keeps what it owns
    const int64_t e = j * n + k;
    const bool isy = valid && k == n, isx = valid && k < n;
    const int64_t jc = valid ? j : 0, ec = isx ? e : 0;
    const double yv = glob(a.vy)[jc], y2v = glob(a.y2)[jc], y1v = glob(a.y1p)[jc], ybv = glob(a.ybar)[jc];
    const double xv = glob(a.vxi)[ec], x2v = glob(a.xi2)[ec], x1v = glob(a.xi1p)[ec], Xv = glob(a.X)[ec];
    const double v = isy ? yv : isx ? xv : 0.0, c2 = isy ? y2v : isx ? x2v : 0.0;
    const double c1p = isy ? y1v : isx ? x1v : 0.0, cb = isy ? ybv : 0.0, xe = isx ? Xv : 0.0;
    double u0[16], u1[16];
    gather_issue<4>(a.blockpart, nblk, 0, 1, u0, u1);
    const gp<const OuterArgs> oa = glob(a.oa);
    const double By = oa->By, Bxi = oa->Bxi;
    __builtin_amdgcn_sched_barrier(0);
    if (uniform(act_v) == 0) return;
    const double beta = glob(a.beta)[uniform(base_v) + a.q + 1];   // (t_l - 1) / t_{l+1}
    // ball projections (Fig. 4 steps 1-2): every block forms the same norms
    double ny2, nx2;
    gather_finish<4>(a.blockpart, nblk, 0, 1, u0, u1, ny2, nx2);
    const double ny = sqrt(ny2), nx = sqrt(nx2);
    const double sc_y = ny > By ? By / ny : 1.0;
    const double sc_xi = nx > Bxi ? Bxi / nx : 1.0;
    double dy2 = 0.0, dx2 = 0.0, prod = 0.0, y2n = 0.0;
    const gp<T> xa = glob((T*)a.xiaug + j * a.kp);
    if (a.sv_nrm && blk == 0 && threadIdx.x == 0) { glob(a.sv_nrm)[0] = ny; glob(a.sv_nrm)[1] = nx; }
    if (valid && k == n) {
        const double y1 = ny > By ? cb + sc_y * (v - cb) : v;   // projection onto Q_y
        if (a.sv_y2) { glob(a.sv_y2)[j] = c2; glob(a.sv_vy)[j] = v; }
        dy2 = (y1 - c2) * (y1 - c2);
        y2n = y1 + beta * (y1 - c1p);                       // extrapolation
        glob(a.y1p)[j] = y1;
        glob(a.y2)[j] = y2n;
    } else if (valid && k < n) {
        const double x1 = sc_xi * v;                        // projection onto Q_xi
        if (a.sv_y2) { glob(a.sv_xi2)[e] = c2; glob(a.sv_vxi)[e] = v; }
        dx2 = (x1 - c2) * (x1 - c2);
        const double x2n = x1 + beta * (x1 - c1p);
        glob(a.xi1p)[e] = x1;
        glob(a.xi2)[e] = x2n;
        const double xo = a.shift ? x2n + glob(a.shift)[e] : x2n;   // slope of the next pass's operands
        if (MIX) {
            const gp<__bf16> xb = glob((__bf16*)a.xiaug + j * a.kp);
            __bf16 hi, lo;
            bf16_split((float)(-xo), hi, lo);
            xb[k] = hi;
            xb[n + k] = hi;
            xb[2 * n + k] = lo;
        } else {
            xa[k] = (T)(-xo);
        }
        prod = xe * xo;
    }
    const double d = group_sum<G>(prod);                    // x_j^T xi_j
    if (valid && k == n) {
        if (MIX) glob(a.cvec)[j] = (float)(d - y2n);
        else xa[n] = (T)(d - y2n);
        glob((T*)a.ycol)[j] = (T)y2n;
    }
    block_sum2(dy2, dx2);
    if (threadIdx.x == 0) { glob(a.blockpart)[blk * 4 + 2] = dy2; glob(a.blockpart)[blk * 4 + 3] = dx2; }
}

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_reduce(ReduceArgs a) {
    reduce_block<T, G>(a, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

template <typename T, int G, int MIX>
__global__ __launch_bounds__(kBlock) void k_update(UpdateArgs a) {
    update_block<T, G, MIX>(a, blockIdx.x, gridDim.x);
}

// Batched O(N n) kernels: block b of the launch is local block blocks[b].y of
// problem blocks[b].x (blocks never straddle problems), nblk_of_p its count.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_reduce_batched(const ReduceArgs* args, const int2* blocks,
                                                           const int32_t* nblk_of_p, int q) {
    // no XCD remap here: a problem's blocks stay spread over all XCDs, so the
    // last problems still running in an adaptive batch use the whole chip
    const int2 bp = blocks[blockIdx.x];
    ReduceArgs a = args[bp.x];
    a.q = q;
    reduce_block<T, G>(a, bp.y, nblk_of_p[bp.x]);
}

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_update_batched(const UpdateArgs* args, const int2* blocks,
                                                           const int32_t* nblk_of_p, int q) {
    const int2 bp = blocks[blockIdx.x];
    UpdateArgs a = args[bp.x];
    a.q = q;
    update_block<T, G, 0, true>(a, bp.y, nblk_of_p[bp.x]);
}

// After the last replay of an ALCC iteration: if no reduce kernel has stopped
// MAPG yet, the run ended at exactly `launched` = l_max iterations.
__global__ __launch_bounds__(kBlock) void k_mapg_end(const double* blockpart, int nblk, int64_t launched,
                                                     DevState* st, const int32_t* gate) {
    if (gate && *gate == 0) return;
    if (st->active == 0) return;
    if (launched < 0) launched = st->base;
    double dy2, dx2;
    gather_sum2(blockpart, nblk, 2, 3, dy2, dx2);
    const double dy = sqrt(dy2), dxi = sqrt(dx2);
    if (threadIdx.x == 0) {
        st->active = 0;
        st->it = launched;
        st->stopped_by_alpha = 0;
        st->dy = dy;
        st->dxi = dxi;
    }
}

// End of a run of lazy passes (see LazyStep).  If no reduce kernel stopped the
// run, it ended at l^max = the launched count after the reduce of step l^max,
// and that step's projections (Fig. 4 steps 1-2) give (y1, xi1); otherwise the
// stopping iteration `it` left y1_it in y1p[it & 1].  Either way the result
// goes to y1p[0] / xi1p[0].  `active` is read here and cleared afterwards by
// k_mapg_end.
template <int G>
__device__ void mapg_finish_block(const LazyStep& z, const int64_t N, const int blk) {
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t j = (int64_t)blk * PER + threadIdx.x / G;
    const int n = z.n;
    const bool valid = j < N;
    const DevState* st = z.st;
    if (st->active) {
        double ny2, nx2;
        gather_sum2(z.npart, z.nblk, 0, 1, ny2, nx2);
        const double ny = sqrt(ny2), nx = sqrt(nx2);
        const bool py = ny > z.oa->By, px = nx > z.oa->Bxi;
        const double sy = py ? z.oa->By / ny : 1.0, sx = px ? z.oa->Bxi / nx : 1.0;
        if (valid && k == n) {
            const double v = z.vy[j], b = z.ybar[j];
            z.y1p[0][j] = py ? b + sy * (v - b) : v;
        } else if (valid && k < n) {
            const double v = z.vxi[j * n + k];
            z.xi1p[0][j * n + k] = px ? sx * v : v;
        }
    } else if (st->it & 1) {
        if (valid && k == n) z.y1p[0][j] = z.y1p[1][j];
        else if (valid && k < n) z.xi1p[0][j * n + k] = z.xi1p[1][j * n + k];
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_mapg_finish(LazyStep z, int64_t N, const int32_t* gate) {
    if (gate && *gate == 0) return;
    mapg_finish_block<G>(z, N, blockIdx.x);
}

// Batched: block b is local block blocks[b].y of problem blocks[b].x, run only
// when that problem's multiplier step is due.
template <int G>
__global__ __launch_bounds__(kBlock) void k_mapg_finish_batched(const PassArgs* args, const int2* blocks) {
    const int2 bp = blocks[blockIdx.x];
    const LazyStep& z = args[bp.x].lz;
    if (z.st->step_due == 0) return;
    mapg_finish_block<G>(z, args[bp.x].N, bp.y);
}

// Set the point of the next pass (and optionally restart MAPG there):
// pass-precision operands from (y, xi); with write_state, also
// y^(1)_0 = y^(2)_1 = y and likewise xi.

template <typename T, int G, int MIX>
__device__ void set_point_block(const PointArgs& a, const int blk) {
    if (a.gate && *a.gate == 0) return;
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t j = (int64_t)blk * PER + threadIdx.x / G;
    const int n = a.n;
    double prod = 0.0, x = 0.0;
    const bool valid = j < a.N;
    if (valid && k < n) {
        const double xs = a.xi[j * n + k];
        if (a.write_state) { a.xi1p[j * n + k] = xs; a.xi2[j * n + k] = xs; }
        x = a.shift ? xs + a.shift[j * n + k] : xs;     // operands from the constraint slope
        prod = a.X[j * n + k] * x;
    }
    const double d = group_sum<G>(prod);
    if (j >= a.ld) return;
    const double yj = valid ? a.y[j] : 0.0;
    if (valid && k == n) {
        ((T*)a.ycol)[j] = (T)yj;
        if (a.write_state) { a.y1p[j] = yj; a.y2[j] = yj; }
    } else if (!valid && k == 0 && j < a.Nrow) {
        ((T*)a.ycol)[j] = (T)0;
    }
    if (MIX) {
        // every BF16 slot of the column, lanes striding over them
        __bf16* xb = (__bf16*)a.xiaug + j * a.kp;
        for (int q = k; q < a.kp; q += G) {
            __bf16 val = (__bf16)0.0f;
            if (valid && q < 3 * n) {
                const int kk = q % n;
                __bf16 hi, lo;
                bf16_split((float)(-(a.shift ? a.xi[j * n + kk] + a.shift[j * n + kk] : a.xi[j * n + kk])), hi, lo);
                val = q < 2 * n ? hi : lo;
            }
            xb[q] = val;
        }
        if (k == 0) a.cvec[j] = valid ? (float)(d - yj) : 0.0f;
    } else {
        if (k >= a.kp) return;
        T* xa = (T*)a.xiaug + j * a.kp;
        xa[k] = !valid ? (T)0 : (k < n ? (T)(-x) : (k == n ? (T)(d - yj) : (T)0));
    }
}

template <typename T, int G, int MIX>
__global__ __launch_bounds__(kBlock) void k_set_point(PointArgs a) {
    set_point_block<T, G, MIX>(a, blockIdx.x);
}

// Batched set point: block b is local block blocks[b].y of problem blocks[b].x.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_set_point_batched(const PointArgs* args, const int2* blocks) {
    const int2 bp = blocks[blockIdx.x];
    set_point_block<T, G, 0>(args[bp.x], bp.y);
}

__global__ void k_begin_outer(OuterArgs args, OuterArgs* dst, DevState* st, int64_t base) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *dst = args;
        st->base = base;
        st->it = 0;
        st->active = args.skip ? 0 : 1;
        st->stopped_by_alpha = 0;
        st->one = 1;
        for (int q = 0; q < 4; ++q) st->cnt[q] = 0u;
    }
}

// ---------------------------------------------------------------------------
// ALCC schedule on the device (Fig. 3; AlccSched).  One thread per problem.
// ---------------------------------------------------------------------------

// Begin ALCC iteration k + 1: L^y_k = 1/mu_k + sigma_max(A1)^2, L^xi_k =
// gamma/mu_k + sigma_max(A2)^2, the radii of Q_y and Q_xi, l^max_k =
// ceil(4 sqrt((L^y By^2 + L^xi Bxi^2)/tau_k)) (capped; a fixed count for a
// fixed schedule), the steps and thresholds; MAPG restarts (t = 1) at the
// current iterate, whose operands the previous multiplier step left in place.
__device__ void alcc_begin(AlccSched* s, OuterArgs* oa, DevState* st) {
    s->k += 1;
    const double Ly = s->Ly_ovr > 0 ? s->Ly_ovr : 1.0 / s->mu + s->sigma2_A1;
    const double Lxi = s->Lxi_ovr > 0 ? s->Lxi_ovr : s->gamma / s->mu + st->sigma2_A2;
    const double By = s->By_ovr > 0 ? s->By_ovr : st->Bbar;
    const double Bxi = s->Bxi_ovr > 0 ? s->Bxi_ovr : st->Bbar / sqrt(s->gamma);
    int64_t lmax;
    if (s->inner_iters > 0) {
        lmax = s->inner_iters;
    } else {
        const double f = ceil(4.0 * sqrt((Ly * By * By + Lxi * Bxi * Bxi) / s->tau));
        lmax = (int64_t)fmax(1.0, fmin(f, (double)s->max_inner));
    }
    OuterArgs a;
    a.mu = s->mu; a.gamma = s->gamma; a.sy = s->step_scale / Ly; a.sxi = s->step_scale / Lxi;
    a.alpha_y = s->ay; a.alpha_xi = s->axi; a.By = By; a.Bxi = Bxi;
    a.theta_scale = 1.0 / s->c; a.lmax = lmax; a.adaptive = s->inner_iters > 0 ? 0 : 1; a.skip = 0;
    *oa = a;
    st->base = 0;
    st->it = 0;
    st->active = 1;
    st->stopped_by_alpha = 0;
    st->step_due = 0;
    st->one = 1;
    for (int q = 0; q < 4; ++q) st->cnt[q] = 0u;
    s->phase = 0;
}

// Start of a run: mu_1, tau_1 and the alpha thresholds (1e-2 Bbar unless
// given), then ALCC iteration 1.
__device__ void alcc_start(AlccSched* s, OuterArgs* oa, DevState* st) {
    s->mu = s->mu1;
    s->tau = s->tau1;
    s->ay = s->ay1 > 0 ? s->ay1 : 1e-2 * st->Bbar;
    s->axi = s->axi1 > 0 ? s->axi1 : 1e-2 * st->Bbar;
    s->k = 0;
    s->total_inner = 0;
    s->converged = 0;
    s->nonfinite = 0;
    alcc_begin(s, oa, st);
}

// End of a replay of `iters` MAPG iterations: the run is over once MAPG has
// stopped (alpha test or l^max, decided by a reduce kernel) or l^max
// iterations have run (the stop of the last one is then not yet decided;
// k_mapg_end takes it).  Then the multiplier step is due.
__device__ void alcc_gate(AlccSched* s, DevState* st, const OuterArgs* oa, int iters) {
    st->base += iters;
    if (s->phase == 0 && (st->active == 0 || st->base >= oa->lmax)) {
        s->phase = 1;
        st->step_due = 1;
    }
}

// After the multiplier step (Fig. 3 step 4) and its KKT reduction: record the
// ALCC iteration, stop on the KKT test (adaptive schedules), on max_outer or
// on a non-finite iterate; otherwise mu_{k+1} = c mu_k, tau and both alpha
// thresholds divided by (c k^{1+kappa})^2, and the next ALCC iteration begins.
__device__ void alcc_step(AlccSched* s, DevState* st, OuterArgs* oa) {
    if (s->phase != 1) return;
    const double kkt = fmax(fmax(st->stat_y, st->stat_xi), fmax(st->infeas, st->compl_)) / (1.0 + st->ybar_inf);
    const int idx = s->k - 1;
    if (idx >= 0 && idx < s->max_outer) {
        s->hist_inner[idx] = st->it;
        s->hist_kkt[idx] = kkt;
    }
    s->total_inner += st->it;
    st->step_due = 0;
    if (st->iterate_nonfinite) { s->nonfinite = 1; s->phase = 2; return; }
    if (s->inner_iters == 0 && kkt <= s->kkt_tol) { s->converged = 1; s->phase = 2; return; }
    if (s->k >= s->max_outer) { s->phase = 2; return; }
    const double decay = pow(s->c * pow((double)s->k, 1.0 + s->kappa), 2.0);
    s->mu = s->c * s->mu;
    s->tau /= decay;
    s->ay /= decay;
    s->axi /= decay;
    alcc_begin(s, oa, st);
}

__global__ void k_alcc_start(AlccSched* s, OuterArgs* oa, DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) alcc_start(s, oa, st);
}
__global__ void k_alcc_gate(AlccSched* s, DevState* st, const OuterArgs* oa, int iters) {
    if (threadIdx.x == 0 && blockIdx.x == 0) alcc_gate(s, st, oa, iters);
}
__global__ void k_alcc_step(AlccSched* s, DevState* st, OuterArgs* oa) {
    if (threadIdx.x == 0 && blockIdx.x == 0) alcc_step(s, st, oa);
}
__global__ void k_alcc_start_batched(AlccSched* const* s, OuterArgs* const* oa, DevState* const* st, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) alcc_start(s[p], oa[p], st[p]);
}
__global__ void k_alcc_gate_batched(AlccSched* const* s, DevState* const* st, OuterArgs* const* oa, int P, int iters,
                                    int32_t* running) {
    int any = 0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        alcc_gate(s[p], st[p], oa[p], iters);
        any |= s[p]->phase != 2;
    }
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    if (any) atomicOr(&s_any, 1);
    __syncthreads();
    if (threadIdx.x == 0) *running = s_any;
}
__global__ void k_alcc_step_batched(AlccSched* const* s, DevState* const* st, OuterArgs* const* oa, int P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) alcc_step(s[p], st[p], oa[p]);
}

// k_mapg_end of every problem whose multiplier step is due (block p: problem p).
__global__ __launch_bounds__(kBlock) void k_mapg_end_batched(const double* const* blockparts, const int32_t* nblk,
                                                             DevState* const* sts) {
    DevState* st = sts[blockIdx.x];
    if (st->step_due == 0 || st->active == 0) return;
    double dy2, dx2;
    gather_sum2(blockparts[blockIdx.x], nblk[blockIdx.x], 2, 3, dy2, dx2);
    const double dy = sqrt(dy2), dxi = sqrt(dx2);
    if (threadIdx.x == 0) {
        st->active = 0;
        st->it = st->base;
        st->stopped_by_alpha = 0;
        st->dy = dy;
        st->dxi = dxi;
    }
}

// Packed X operands (see cr_device.h): one thread per (16-row tile, lane).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prep_xp(const double* X, int64_t N, int n, int64_t Nrow, int ks,
                                                    int qp, T* xp) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= (Nrow / 16) * 64) return;
    const int64_t tile = gid / 64;
    const int lane = (int)(gid % 64), g = lane >> 4, c = lane & 15;
    const int64_t i0 = tile * 16;
    const int q_used = ks + 4 * nkb_of_ks(ks);
    for (int q = 0; q < qp; ++q) {
        int64_t i;
        int k;
        if (q < ks) {
            i = i0 + c; k = 4 * q + g;
        } else if (q < q_used) {
            const int s = (q - ks) % 4, kb = (q - ks) / 4;
            i = i0 + rmap<T>(g, s); k = 16 * kb + c;
        } else {
            xp[gid * qp + q] = (T)0;
            continue;
        }
        double val = 0.0;
        if (i < N) val = k < n ? X[i * n + k] : (k == n ? 1.0 : 0.0);
        xp[gid * qp + q] = (T)val;
    }
}

// Packed mixed-precision X operands, one thread per (16-row tile, lane), as
// 16-byte vectors: KB vectors of the residual A operand (slots 32 kb + 8 g + e
// of [x_hi | x_lo | x_hi] for row i0 + c), then per column block kb2 the two
// B operands of C: [X_hi rows 4g..4g+3, X_hi same rows] and [X_lo same rows, 0].
__device__ __forceinline__ double xaug_at(const double* X, int64_t N, int n, int64_t i, int k) {
    if (i >= N) return 0.0;
    return k < n ? X[i * n + k] : (k == n ? 1.0 : 0.0);
}
__global__ __launch_bounds__(kBlock) void k_prep_xp_mixed(const double* X, int64_t N, int n, int64_t Nrow,
                                                           int kb_r, int nkb, bf16x8* xp) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= (Nrow / 16) * 64) return;
    const int64_t i0 = (gid / 64) * 16;
    const int lane = (int)(gid % 64), g = lane >> 4, c = lane & 15;
    bf16x8* out = xp + gid * (kb_r + nkb);
    for (int kb = 0; kb < kb_r; ++kb) {
        bf16x8 v;
        for (int e = 0; e < 8; ++e) {
            const int q = 32 * kb + 8 * g + e;
            __bf16 hi = (__bf16)0.0f, lo = (__bf16)0.0f;
            if (q < 3 * n) bf16_split((float)xaug_at(X, N, n, i0 + c, q % n), hi, lo);
            v[e] = (q >= n && q < 2 * n) ? lo : hi;
        }
        out[kb] = v;
    }
    // column blocks: [x_hi, x_lo] of the lane's rows 4g .. 4g + 3 at feature 16 kb + c
    for (int kb = 0; kb < nkb; ++kb) {
        bf16x8 v;
        for (int e = 0; e < 4; ++e) {
            __bf16 hi, lo;
            bf16_split((float)xaug_at(X, N, n, i0 + 4 * g + e, 16 * kb + c), hi, lo);
            v[e] = hi;
            v[e + 4] = lo;
        }
        out[kb_r + kb] = v;
    }
}

// theta layout conversions (inspection / tests) and clearing.
template <typename T>
__global__ void k_theta_import(const double* src, int64_t N, int64_t Nrow, int64_t ld, T* theta) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= Nrow * ld) return;
    const int64_t i = e / ld, j = e % ld;
    theta[e] = (i < N && j < N && i != j) ? (T)src[i * N + j] : (T)0;
}
template <typename T>
__global__ void k_theta_export(const T* theta, int64_t N, int64_t ld, double* dst) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= N * N) return;
    const int64_t i = e / N, j = e % N;
    dst[e] = i == j ? 0.0 : (double)theta[i * ld + j];
}
__global__ void k_zero16(uint4* p, int64_t n16) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = e; q < n16; q += stride) p[q] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// Set-up (once per context, FP64): means, centred scatter matrix and its
// eigen-decomposition, affine least-squares fit, sigma_max(A2)^2, start point.
// Scratch `su` layout: [0,n) xbar | [n] ybar mean | [n+1,2n+1) a | [2n+1] b |
//   [2n+2, 3n+2) eigenvalues | [3n+2, 3n+2+n^2) eigenvectors (column k = vector k)
// ---------------------------------------------------------------------------
__device__ void su_sums_body(const double* X, const double* ybar, int64_t N, int n, int64_t rows,
                             const double* su, int phase, double* part, const int blk) {
    // phase 0: e < n: sum x_ik; e = n: sum ybar; e = n+1: max |ybar|; e = n+2: # non-finite
    // phase 1: e < n*n: sum u_ik u_il; n*n <= e < n*n+n: sum u_ik (ybar_i - ybar_mean)
    // phase 2: e < n: sum u_ik (ybar_i - ybar_mean) (the entries n*n + e of phase 1)
    // Thread (e, p) owns entry e and the rows r0 + p, r0 + p + P, ... of the
    // workgroup's rows (P = 256 / #entries row lanes, so that the loads of a
    // workgroup are in flight together); the P pieces of an entry are then
    // combined in LDS in index order.  With more entries than threads each
    // thread walks all the rows of its entries (P = 1).
    const int64_t r0 = (int64_t)blk * rows, r1 = min(r0 + rows, N);
    const int ne = phase == 0 ? n + 3 : (phase == 1 ? n * n + n : n);
    const int eq = phase == 2 ? n * n : 0;        // phase 2 computes phase 1's entries n*n + e
    const double ym = phase != 0 ? su[n] : 0.0;
    const int P = ne < (int)blockDim.x ? (int)blockDim.x / ne : 1;
    __shared__ double piece[kBlock];
    for (int e0 = 0; e0 < ne; e0 += (int)blockDim.x / P) {
        const int e = e0 + (int)threadIdx.x % (ne < (int)blockDim.x ? ne : (int)blockDim.x);
        const int p = P > 1 ? (int)threadIdx.x / ne : 0;
        const bool active = e < ne && p < P;
        const bool is_max = phase == 0 && e == n + 1;
        auto term = [&](int64_t i) -> double {
            if (phase == 0) {
                if (e < n) return X[i * n + e];
                if (e == n) return ybar[i];
                if (e == n + 1) return fabs(ybar[i]);
                bool bad = !isfinite(ybar[i]);
                for (int k = 0; k < n; ++k) bad = bad || !isfinite(X[i * n + k]);
                return bad ? 1.0 : 0.0;
            }
            const int ee = e + eq;
            if (ee < n * n) {
                const int k = ee / n, l = ee % n;
                return (X[i * n + k] - su[k]) * (X[i * n + l] - su[l]);
            }
            const int k = ee - n * n;
            return (X[i * n + k] - su[k]) * (ybar[i] - ym);
        };
        double a0 = 0.0, a1 = 0.0;
        if (active) {
            int64_t i = r0 + p;
            for (; i + P < r1; i += 2 * P) {
                const double t0 = term(i), t1 = term(i + P);
                a0 = is_max ? fmax(a0, t0) : a0 + t0;
                a1 = is_max ? fmax(a1, t1) : a1 + t1;
            }
            if (i < r1) { const double t0 = term(i); a0 = is_max ? fmax(a0, t0) : a0 + t0; }
        }
        const double v = is_max ? fmax(a0, a1) : a0 + a1;
        if (P == 1) {
            if (active) part[(int64_t)blk * ne + e] = v;
            continue;
        }
        __syncthreads();
        if (active) piece[p * ne + e] = v;
        __syncthreads();
        if (threadIdx.x < ne) {
            const int ee = threadIdx.x;
            const bool mx = phase == 0 && ee == n + 1;
            double acc = piece[ee];
            for (int q = 1; q < P; ++q) acc = mx ? fmax(acc, piece[q * ne + ee]) : acc + piece[q * ne + ee];
            part[(int64_t)blk * ne + ee] = acc;
        }
    }
}

__global__ void k_su_sums(const double* X, const double* ybar, int64_t N, int n, int64_t rows,
                          const double* su, int phase, double* part) {
    su_sums_body(X, ybar, N, n, rows, su, phase, part, blockIdx.x);
}

__device__ void su_means_final_body(const double* part, int nblk, int64_t N, int n, double* su, DevState* st) {
    // one thread per entry, blocks summed in index order
    const int ne = n + 3;
    const int e = threadIdx.x;
    if (e == 0) st->one = 1;
    if (e >= ne) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc = (e == n + 1) ? fmax(acc, part[b * ne + e]) : acc + part[b * ne + e];
    if (e < n) su[e] = acc / (double)N;
    else if (e == n) { su[n] = acc / (double)N; st->ybar_mean = su[n]; }
    else if (e == n + 1) st->ybar_inf = acc;
    else st->nonfinite = acc > 0.0 ? 1 : 0;
}
__global__ void k_su_means_final(const double* part, int nblk, int64_t N, int n, double* su, DevState* st) {
    su_means_final_body(part, nblk, N, n, su, st);
}

// The affine fit for new data on the same points: q = X_c^T ybar_c from the
// phase-2 partials, then a and b from the eigen-decomposition already in su
// (the same formula and order as k_su_eig_final).  The sums of q, the
// eigen-pairs and the means are staged in LDS by the whole workgroup first,
// so that thread 0's arithmetic reads no global memory between its stores.
__device__ void su_fit_final_body(const double* part, int nblk, int n, double* su) {
    __shared__ double q[kMaxDim], lam[kMaxDim], V[kMaxDim * kMaxDim], xm[kMaxDim + 1], acoef[kMaxDim];
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += part[b * n + e];
        q[e] = acc;
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) lam[e] = su[2 * n + 2 + e];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) V[e] = su[3 * n + 2 + e];
    for (int e = threadIdx.x; e <= n; e += blockDim.x) xm[e] = su[e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double lmax = 0.0;
    for (int k = 0; k < n; ++k) lmax = fmax(lmax, lam[k]);
    for (int l = 0; l < n; ++l) acoef[l] = 0.0;
    for (int k = 0; k < n; ++k) {
        if (!(lam[k] > 1e-12 * lmax)) continue;
        double proj = 0.0;
        for (int l = 0; l < n; ++l) proj += V[l * n + k] * q[l];
        proj /= lam[k];
        for (int l = 0; l < n; ++l) acoef[l] += proj * V[l * n + k];
    }
    double b = xm[n];
    for (int l = 0; l < n; ++l) b -= xm[l] * acoef[l];
    for (int l = 0; l < n; ++l) su[n + 1 + l] = acoef[l];
    su[2 * n + 1] = b;
}
__global__ void k_su_fit_final(const double* part, int nblk, int n, double* su) {
    su_fit_final_body(part, nblk, n, su);
}

// Cyclic Jacobi eigen-decomposition of the centred scatter matrix M0 and the
// affine fit a = M0^+ X_c^T ybar_c, b = mean(ybar) - xbar^T a.  Each rotation's
// column, row and eigenvector updates run with one thread per index k (the
// elements a thread updates are its own, so every value is computed exactly
// as a single thread walking k would); the sweep's stopping test and the
// rotation angle are formed from the same LDS values in the same order.
__global__ void k_su_eig_final(const double* part, int nblk, int n, double* su) {
    __shared__ double A[kMaxDim * kMaxDim], V[kMaxDim * kMaxDim], q[kMaxDim];
    __shared__ int done;
    const int ne = n * n + n;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += part[b * ne + e];
        if (e < n * n) A[e] = acc;
        else q[e - n * n] = acc;
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) V[e] = e / n == e % n ? 1.0 : 0.0;
    __syncthreads();
    const int k = threadIdx.x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        if (threadIdx.x == 0) {
            double off = 0.0, diag = 0.0;
            for (int p = 0; p < n; ++p) {
                diag += A[p * n + p] * A[p * n + p];
                for (int r = p + 1; r < n; ++r) off += A[p * n + r] * A[p * n + r];
            }
            done = off <= 1e-32 * diag || off == 0.0;
        }
        __syncthreads();
        if (done) break;
        for (int p = 0; p < n; ++p)
            for (int r = p + 1; r < n; ++r) {
                const double apr = A[p * n + r];
                const double app = A[p * n + p], arr = A[r * n + r];
                __syncthreads();                     // every thread has read the pivot entries
                if (apr == 0.0) continue;            // the same value in every thread
                const double tau = (arr - app) / (2.0 * apr);
                const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = tt * cs;
                if (k < n) {                         // columns p, r
                    const double akp = A[k * n + p], akr = A[k * n + r];
                    A[k * n + p] = cs * akp - sn * akr;
                    A[k * n + r] = sn * akp + cs * akr;
                }
                __syncthreads();
                if (k < n) {                         // rows p, r; eigenvectors
                    const double apk = A[p * n + k], ark = A[r * n + k];
                    A[p * n + k] = cs * apk - sn * ark;
                    A[r * n + k] = sn * apk + cs * ark;
                    const double vkp = V[k * n + p], vkr = V[k * n + r];
                    V[k * n + p] = cs * vkp - sn * vkr;
                    V[k * n + r] = sn * vkp + cs * vkr;
                }
                __syncthreads();
            }
    }
    if (threadIdx.x != 0) return;
    double lmax = 0.0;
    for (int k = 0; k < n; ++k) lmax = fmax(lmax, A[k * n + k]);
    double* lam = su + 2 * n + 2;
    double* vec = su + 3 * n + 2;
    for (int k = 0; k < n; ++k) lam[k] = A[k * n + k];
    for (int e = 0; e < n * n; ++e) vec[e] = V[e];
    // a = sum_k v_k (v_k^T q) / lam_k over eigenvalues above the rank tolerance
    double* acoef = su + n + 1;
    for (int l = 0; l < n; ++l) acoef[l] = 0.0;
    for (int k = 0; k < n; ++k) {
        if (!(lam[k] > 1e-12 * lmax)) continue;
        double proj = 0.0;
        for (int l = 0; l < n; ++l) proj += V[l * n + k] * q[l];
        proj /= lam[k];
        for (int l = 0; l < n; ++l) acoef[l] += proj * V[l * n + k];
    }
    double b = su[n];
    for (int l = 0; l < n; ++l) b -= su[l] * acoef[l];
    su[2 * n + 1] = b;
}

// lambda_max(S_j) with S_j = M0 + N u u^T, u = x_j - xbar: the largest root of
// the secular equation 1 = sum_k z_k^2 / (lambda - lam_k), z = sqrt(N) V^T u,
// found by bisection on [max lam, max lam + |z|^2].
__global__ __launch_bounds__(kBlock) void k_su_sigma2(const double* X, int64_t N, int n, const double* su,
                                                      double* part) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double best = 0.0;
    if (j < N) {
        const double* lam = su + 2 * n + 2;
        const double* vec = su + 3 * n + 2;
        double z[kMaxDim];
        double zz = 0.0, l1 = lam[0];
        for (int k = 1; k < n; ++k) l1 = fmax(l1, lam[k]);
        for (int k = 0; k < n; ++k) {
            double acc = 0.0;
            for (int l = 0; l < n; ++l) acc += vec[l * n + k] * (X[j * n + l] - su[l]);
            z[k] = sqrt((double)N) * acc;
            zz += z[k] * z[k];
        }
        double lo = l1, hi = l1 + zz;
        for (int itr = 0; itr < 200 && zz > 0.0; ++itr) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            double f = 1.0;
            for (int k = 0; k < n; ++k) f -= z[k] * z[k] / (mid - lam[k]);
            if (f < 0.0) lo = mid; else hi = mid;
        }
        best = zz > 0.0 ? hi : l1;
    }
    const double b = block_reduce(best, 1);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ void k_su_sigma2_final(const double* part, int nblk, DevState* st) {
    if (threadIdx.x != 0) return;
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = fmax(m, part[b]);
    st->sigma2_A2 = m;
}

// Start point (Sec. II-E): yhat = X a + b, xihat_l = a; Bbar^2 = |yhat - ybar|^2 + gamma |xihat|^2.
__device__ void su_start_body(const double* X, const double* ybar, int64_t N, int n, const double* su, double* y0,
                              double* xi0, double* part, const int blk) {
    const int64_t j = (int64_t)blk * kBlock + threadIdx.x;
    const double* acoef = su + n + 1;
    double r2 = 0.0;
    if (j < N) {
        double v = su[2 * n + 1];
        for (int k = 0; k < n; ++k) {
            v += X[j * n + k] * acoef[k];
            xi0[j * n + k] = acoef[k];
        }
        y0[j] = v;
        r2 = (v - ybar[j]) * (v - ybar[j]);
    }
    const double b = block_reduce(r2, 0);
    if (threadIdx.x == 0) part[blk] = b;
}
__global__ __launch_bounds__(kBlock) void k_su_start(const double* X, const double* ybar, int64_t N, int n,
                                                     const double* su, double* y0, double* xi0, double* part) {
    su_start_body(X, ybar, N, n, su, y0, xi0, part, blockIdx.x);
}

__device__ void su_start_final_body(const double* part, int nblk, int64_t N, int n, double gamma, const double* su,
                                    DevState* st) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    double aa = 0.0;
    for (int k = 0; k < n; ++k) aa += su[n + 1 + k] * su[n + 1 + k];
    st->aff_b = su[2 * n + 1];
    st->Bbar = sqrt(s + gamma * (double)N * aa);
}
__global__ void k_su_start_final(const double* part, int nblk, int64_t N, int n, double gamma, const double* su,
                                 DevState* st) {
    su_start_final_body(part, nblk, N, n, gamma, su, st);
}

// Start of a problem in shifted slopes xi = xi' + c: the affine fit (yhat, a)
// is (yhat, a - c) there, still feasible; Bbar is the objective at it.  One
// workgroup; fixed summation order.
__device__ void su_shift_body(const double* y0, const double* ybar, double* xi0, const double* shift, int64_t N, int n,
                              double gamma, DevState* st) {
    double r2 = 0.0, x2 = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kBlock) {
        const double d = y0[j] - ybar[j];
        r2 += d * d;
        for (int k = 0; k < n; ++k) {
            const double x = xi0[j * n + k] - shift[j * n + k];
            xi0[j * n + k] = x;
            x2 += x * x;
        }
    }
    const double R2 = block_reduce(r2, 0), X2 = block_reduce(x2, 0);
    if (threadIdx.x == 0) st->Bbar = sqrt(R2 + gamma * X2);
}
__global__ __launch_bounds__(kBlock) void k_su_shift(const double* y0, const double* ybar, double* xi0,
                                                     const double* shift, int64_t N, int n, double gamma,
                                                     DevState* st) {
    su_shift_body(y0, ybar, xi0, shift, N, n, gamma, st);
}

// The re-fit of several problems (P-APG's blocks) in one launch per step:
// problem blockIdx.y of the table, its blocks past its own count return.
__global__ __launch_bounds__(kBlock) void k_refit_sums_b(RefitTable t, int phase) {
    const RefitArgs& a = t.p[blockIdx.y];
    if ((int64_t)blockIdx.x * kSuRows >= a.N) return;
    su_sums_body(a.X, a.ybar, a.N, a.n, kSuRows, a.su, phase, a.part, blockIdx.x);
}
__global__ void k_refit_means_b(RefitTable t) {
    const RefitArgs& a = t.p[blockIdx.y];
    su_means_final_body(a.part, (int)((a.N + kSuRows - 1) / kSuRows), a.N, a.n, a.su, a.st);
}
__global__ void k_refit_fit_b(RefitTable t) {
    const RefitArgs& a = t.p[blockIdx.y];
    su_fit_final_body(a.part, (int)((a.N + kSuRows - 1) / kSuRows), a.n, a.su);
}
__global__ __launch_bounds__(kBlock) void k_refit_start_b(RefitTable t) {
    const RefitArgs& a = t.p[blockIdx.y];
    if ((int64_t)blockIdx.x * kBlock >= a.N) return;
    su_start_body(a.X, a.ybar, a.N, a.n, a.su, a.y0, a.xi0, a.part, blockIdx.x);
}
__global__ void k_refit_start_final_b(RefitTable t) {
    const RefitArgs& a = t.p[blockIdx.y];
    su_start_final_body(a.part, (int)((a.N + kBlock - 1) / kBlock), a.N, a.n, a.gamma, a.su, a.st);
}
__global__ __launch_bounds__(kBlock) void k_refit_shift_b(RefitTable t) {
    const RefitArgs& a = t.p[blockIdx.y];
    if (!a.shift) return;
    su_shift_body(a.y0, a.ybar, a.xi0, a.shift, a.N, a.n, a.gamma, a.st);
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (called by the driver in cr_api.hip).
// ---------------------------------------------------------------------------
template <typename Ops, int GRAD_WAVES = 2>
static hipError_t launch_pass_ops(const PassArgs& a, dim3 grid, hipStream_t s) {
    if (a.mode == 1) hipLaunchKernelGGL((k_pair_pass<Ops, 1, 2>), grid, dim3(kBlock), 0, s, a);
    else if (a.lz.on) hipLaunchKernelGGL((k_pair_pass<Ops, 0, GRAD_WAVES, 1>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_pair_pass<Ops, 0, GRAD_WAVES>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

bool lazy_fits(int prec, int64_t rows_per_chunk) {
    const int esz = prec == 0 ? 8 : 4;
    return 2 * lazy_rbytes(rows_per_chunk, esz) + kBsBytes <= 32768;
}

template <typename T>
static hipError_t launch_pass_t(int ks, const PassArgs& a, dim3 grid, hipStream_t s) {
    // waves per SIMD the small classes' gradient passes allow without spills
    constexpr int W_SMALL = sizeof(T) == 4 ? 4 : 3;
    switch (ks) {
        case 1: return launch_pass_ops<PlainOps<T, 1>, W_SMALL>(a, grid, s);
        case 2: return launch_pass_ops<PlainOps<T, 2>, W_SMALL>(a, grid, s);
        case 3: return launch_pass_ops<PlainOps<T, 3>, W_SMALL>(a, grid, s);
        case 4: return launch_pass_ops<PlainOps<T, 4>, 3>(a, grid, s);
        case 5: return launch_pass_ops<PlainOps<T, 5>>(a, grid, s);
        case 6: return launch_pass_ops<PlainOps<T, 6>>(a, grid, s);
        case 7: return launch_pass_ops<PlainOps<T, 7>>(a, grid, s);
        case 8: return launch_pass_ops<PlainOps<T, 8>>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// Mixed: KB = ceil(3n / 32) BF16 k-blocks for R, NKB = ceil((n + 1) / 16) column blocks.
static hipError_t launch_pass_mixed(int n, const PassArgs& a, dim3 grid, hipStream_t s) {
    const int kb = mixed_kb(n), nkb = (n + 1 + 15) / 16;
    if (kb == 1 && nkb == 1) return launch_pass_ops<MixedOps<1, 1>>(a, grid, s);
    if (kb == 2 && nkb == 1) return launch_pass_ops<MixedOps<2, 1>>(a, grid, s);
    if (kb == 2 && nkb == 2) return launch_pass_ops<MixedOps<2, 2>>(a, grid, s);
    if (kb == 3 && nkb == 2) return launch_pass_ops<MixedOps<3, 2>>(a, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pair_pass(int prec, int n, const PassArgs& a, dim3 grid, hipStream_t s) {
    if (prec == 2) return launch_pass_mixed(n, a, grid, s);
    const int ks = ks_of(n);
    return prec == 0 ? launch_pass_t<double>(ks, a, grid, s) : launch_pass_t<float>(ks, a, grid, s);
}

// Threads per point of the O(N n) kernels: the smallest of 16, 32 that holds n + 1.
static int group_of(int n) { return n + 1 <= 16 ? 16 : 32; }
static dim3 points_grid(int64_t points, int G) { return dim3((unsigned)((points * G + kBlock - 1) / kBlock)); }

template <typename T>
static void reduce_t(const ReduceArgs& a, hipStream_t s) {
    if (group_of(a.n) == 16) hipLaunchKernelGGL((k_reduce<T, 16>), points_grid(a.N, 16), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_reduce<T, 32>), points_grid(a.N, 32), dim3(kBlock), 0, s, a);
}
template <typename T, int MIX>
static void update_t(const UpdateArgs& a, hipStream_t s) {
    if (group_of(a.n) == 16) hipLaunchKernelGGL((k_update<T, 16, MIX>), points_grid(a.N, 16), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_update<T, 32, MIX>), points_grid(a.N, 32), dim3(kBlock), 0, s, a);
}
template <typename T, int MIX>
static void set_point_t(const PointArgs& a, hipStream_t s) {
    if (group_of(a.n) == 16) hipLaunchKernelGGL((k_set_point<T, 16, MIX>), points_grid(a.ld, 16), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_set_point<T, 32, MIX>), points_grid(a.ld, 32), dim3(kBlock), 0, s, a);
}

hipError_t launch_reduce(bool f64, const ReduceArgs& a, hipStream_t s) {
    if (f64) reduce_t<double>(a, s); else reduce_t<float>(a, s);
    return hipGetLastError();
}

hipError_t launch_update(int prec, const UpdateArgs& a, hipStream_t s) {
    if (prec == 0) update_t<double, 0>(a, s);
    else if (prec == 1) update_t<float, 0>(a, s);
    else update_t<float, 1>(a, s);
    return hipGetLastError();
}

int reduce_blocks(int64_t N, int n) { return (int)points_grid(N, group_of(n)).x; }

hipError_t launch_mapg_finish(const LazyStep& z, int64_t N, hipStream_t s, const int32_t* gate) {
    if (group_of(z.n) == 16) hipLaunchKernelGGL((k_mapg_finish<16>), points_grid(N, 16), dim3(kBlock), 0, s, z, N, gate);
    else hipLaunchKernelGGL((k_mapg_finish<32>), points_grid(N, 32), dim3(kBlock), 0, s, z, N, gate);
    return hipGetLastError();
}
int reduce_blocks_g(int64_t N, int G) { return (int)points_grid(N, G).x; }

hipError_t launch_mapg_finish_batched(int G, const PassArgs* args, const void* blocks, int nblocks, hipStream_t s) {
    const int2* b = (const int2*)blocks;
    if (G == 16) hipLaunchKernelGGL((k_mapg_finish_batched<16>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
    else hipLaunchKernelGGL((k_mapg_finish_batched<32>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
    return hipGetLastError();
}

// One workgroup per item.  WAVES: the waves per SIMD the class's register
// budget allows without spills (the single-problem pass's figures; the lazy
// FP32 KS = 3 class takes one less).
template <typename T, int KS, int MODE, int LAZY>
static void pass_batched_ks(const PassArgs* args, const int32_t* nstrips, const BatchItem* it, int nitems, int q,
                            hipStream_t s) {
    constexpr int W = MODE == 1 ? 2
                    : sizeof(T) == 4 ? (KS <= 2 ? 4 : KS == 3 ? (LAZY ? 3 : 4) : KS == 4 ? 3 : 2)
                                     : (KS <= 4 ? 3 : 2);
    if (nitems < 1) return;
    hipLaunchKernelGGL((k_pair_pass_batched<T, KS, MODE, W, LAZY>), dim3(nitems), dim3(kBlock), 0, s, args, nstrips, it,
                       q);
}
template <typename T, int MODE, int LAZY>
static hipError_t pass_batched_t(int ks, const PassArgs* args, const int32_t* nstrips, const BatchItem* it,
                                 int nitems, int q, hipStream_t s) {
    switch (ks) {
        case 1: pass_batched_ks<T, 1, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 2: pass_batched_ks<T, 2, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 3: pass_batched_ks<T, 3, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 4: pass_batched_ks<T, 4, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 5: pass_batched_ks<T, 5, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 6: pass_batched_ks<T, 6, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 7: pass_batched_ks<T, 7, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        case 8: pass_batched_ks<T, 8, MODE, LAZY>(args, nstrips, it, nitems, q, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass_batched(bool f64, int ks, const PassArgs* args, const int32_t* nstrips, const void* items,
                               int nitems, hipStream_t s, bool lazy, int q) {
    const BatchItem* it = (const BatchItem*)items;
    if (lazy)
        return f64 ? pass_batched_t<double, 0, 1>(ks, args, nstrips, it, nitems, q, s)
                   : pass_batched_t<float, 0, 1>(ks, args, nstrips, it, nitems, q, s);
    return f64 ? pass_batched_t<double, 0, 0>(ks, args, nstrips, it, nitems, q, s)
               : pass_batched_t<float, 0, 0>(ks, args, nstrips, it, nitems, q, s);
}

hipError_t launch_theta_pass_batched(bool f64, int ks, const PassArgs* args, const int32_t* nstrips, const void* items,
                                     int nitems, hipStream_t s) {
    const BatchItem* it = (const BatchItem*)items;
    return f64 ? pass_batched_t<double, 1, 0>(ks, args, nstrips, it, nitems, 0, s)
               : pass_batched_t<float, 1, 0>(ks, args, nstrips, it, nitems, 0, s);
}

hipError_t launch_reduce_batched(bool f64, int G, const ReduceArgs* args, const void* blocks, const int32_t* nblk,
                                 int nblocks, int q, hipStream_t s) {
    const int2* b = (const int2*)blocks;
    if (f64) {
        if (G == 16) hipLaunchKernelGGL((k_reduce_batched<double, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
        else hipLaunchKernelGGL((k_reduce_batched<double, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_reduce_batched<float, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
        else hipLaunchKernelGGL((k_reduce_batched<float, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
    }
    return hipGetLastError();
}

hipError_t launch_update_batched(bool f64, int G, const UpdateArgs* args, const void* blocks, const int32_t* nblk,
                                 int nblocks, int q, hipStream_t s) {
    const int2* b = (const int2*)blocks;
    if (f64) {
        if (G == 16) hipLaunchKernelGGL((k_update_batched<double, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
        else hipLaunchKernelGGL((k_update_batched<double, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_update_batched<float, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
        else hipLaunchKernelGGL((k_update_batched<float, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b, nblk, q);
    }
    return hipGetLastError();
}

hipError_t launch_mapg_end(const double* blockpart, int nblk, int64_t launched, DevState* st, hipStream_t s,
                           const int32_t* gate) {
    hipLaunchKernelGGL(k_mapg_end, dim3(1), dim3(kBlock), 0, s, blockpart, nblk, launched, st, gate);
    return hipGetLastError();
}

hipError_t launch_alcc_start(AlccSched* sc, OuterArgs* oa, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_start, dim3(1), dim3(64), 0, s, sc, oa, st);
    return hipGetLastError();
}
hipError_t launch_alcc_gate(AlccSched* sc, DevState* st, const OuterArgs* oa, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_gate, dim3(1), dim3(64), 0, s, sc, st, oa, iters);
    return hipGetLastError();
}
hipError_t launch_alcc_step(AlccSched* sc, DevState* st, OuterArgs* oa, hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_step, dim3(1), dim3(64), 0, s, sc, st, oa);
    return hipGetLastError();
}
hipError_t launch_alcc_start_batched(AlccSched* const* sc, OuterArgs* const* oa, DevState* const* st, int P,
                                     hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_start_batched, dim3((P + 63) / 64), dim3(64), 0, s, sc, oa, st, P);
    return hipGetLastError();
}
hipError_t launch_alcc_gate_batched(AlccSched* const* sc, DevState* const* st, OuterArgs* const* oa, int P, int iters,
                                    int32_t* running, hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_gate_batched, dim3(1), dim3(kBlock), 0, s, sc, st, oa, P, iters, running);
    return hipGetLastError();
}
hipError_t launch_alcc_step_batched(AlccSched* const* sc, DevState* const* st, OuterArgs* const* oa, int P,
                                    hipStream_t s) {
    hipLaunchKernelGGL(k_alcc_step_batched, dim3((P + 63) / 64), dim3(64), 0, s, sc, st, oa, P);
    return hipGetLastError();
}
hipError_t launch_mapg_end_batched(const double* const* blockparts, const int32_t* nblk, DevState* const* st, int P,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_mapg_end_batched, dim3(P), dim3(kBlock), 0, s, blockparts, nblk, st);
    return hipGetLastError();
}
hipError_t launch_set_point_batched(bool f64, int G, const PointArgs* args, const void* blocks, const int32_t*,
                                    int nblocks, hipStream_t s) {
    const int2* b = (const int2*)blocks;
    if (f64) {
        if (G == 16) hipLaunchKernelGGL((k_set_point_batched<double, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
        else hipLaunchKernelGGL((k_set_point_batched<double, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_set_point_batched<float, 16>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
        else hipLaunchKernelGGL((k_set_point_batched<float, 32>), dim3(nblocks), dim3(kBlock), 0, s, args, b);
    }
    return hipGetLastError();
}

hipError_t launch_set_point(int prec, const PointArgs& a, hipStream_t s) {
    if (prec == 0) set_point_t<double, 0>(a, s);
    else if (prec == 1) set_point_t<float, 0>(a, s);
    else set_point_t<float, 1>(a, s);
    return hipGetLastError();
}

hipError_t launch_begin_outer(const OuterArgs& args, OuterArgs* dst, DevState* st, hipStream_t s, int64_t base) {
    hipLaunchKernelGGL(k_begin_outer, dim3(1), dim3(64), 0, s, args, dst, st, base);
    return hipGetLastError();
}

hipError_t launch_prep_xp(int prec, const double* X, int64_t N, int n, int64_t Nrow, int ks, int qp, void* xp,
                          hipStream_t s) {
    const int64_t total = (Nrow / 16) * 64;
    const dim3 grid((unsigned)((total + kBlock - 1) / kBlock));
    if (prec == 0) hipLaunchKernelGGL(k_prep_xp<double>, grid, dim3(kBlock), 0, s, X, N, n, Nrow, ks, qp, (double*)xp);
    else if (prec == 1) hipLaunchKernelGGL(k_prep_xp<float>, grid, dim3(kBlock), 0, s, X, N, n, Nrow, ks, qp, (float*)xp);
    else hipLaunchKernelGGL(k_prep_xp_mixed, grid, dim3(kBlock), 0, s, X, N, n, Nrow, mixed_kb(n), (n + 1 + 15) / 16,
                            (bf16x8*)xp);
    return hipGetLastError();
}

hipError_t launch_theta_import(bool f64, const double* src, int64_t N, int64_t Nrow, int64_t ld, void* theta,
                               hipStream_t s) {
    const dim3 grid((unsigned)((Nrow * ld + kBlock - 1) / kBlock));
    if (f64) hipLaunchKernelGGL(k_theta_import<double>, grid, dim3(kBlock), 0, s, src, N, Nrow, ld, (double*)theta);
    else hipLaunchKernelGGL(k_theta_import<float>, grid, dim3(kBlock), 0, s, src, N, Nrow, ld, (float*)theta);
    return hipGetLastError();
}

hipError_t launch_theta_export(bool f64, const void* theta, int64_t N, int64_t ld, double* dst, hipStream_t s) {
    const dim3 grid((unsigned)((N * N + kBlock - 1) / kBlock));
    if (f64) hipLaunchKernelGGL(k_theta_export<double>, grid, dim3(kBlock), 0, s, (const double*)theta, N, ld, dst);
    else hipLaunchKernelGGL(k_theta_export<float>, grid, dim3(kBlock), 0, s, (const float*)theta, N, ld, dst);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    int64_t blocks = (n16 + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint4*)p, n16);
    return hipGetLastError();
}

hipError_t launch_setup_shift(const double* y0, const double* ybar, double* xi0, const double* shift, int64_t N,
                              int n, double gamma, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_su_shift, dim3(1), dim3(kBlock), 0, s, y0, ybar, xi0, shift, N, n, gamma, st);
    return hipGetLastError();
}

hipError_t launch_refit(const double* X, const double* ybar, int64_t N, int n, double gamma, double* su,
                        double* part, double* y0, double* xi0, DevState* st, hipStream_t s) {
    const int64_t rows = kSuRows;
    const int nblk = (int)((N + rows - 1) / rows);
    hipLaunchKernelGGL(k_su_sums, dim3(nblk), dim3(kBlock), 0, s, X, ybar, N, n, rows, (const double*)su, 0, part);
    hipLaunchKernelGGL(k_su_means_final, dim3(1), dim3(64), 0, s, (const double*)part, nblk, N, n, su, st);
    hipLaunchKernelGGL(k_su_sums, dim3(nblk), dim3(kBlock), 0, s, X, ybar, N, n, rows, (const double*)su, 2, part);
    hipLaunchKernelGGL(k_su_fit_final, dim3(1), dim3(64), 0, s, (const double*)part, nblk, n, su);
    const int nb = (int)((N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_su_start, dim3(nb), dim3(kBlock), 0, s, X, ybar, N, n, (const double*)su, y0, xi0, part);
    hipLaunchKernelGGL(k_su_start_final, dim3(1), dim3(64), 0, s, (const double*)part, nb, N, n, gamma,
                       (const double*)su, st);
    return hipGetLastError();
}

hipError_t launch_refit_batched(const RefitTable& t, hipStream_t s) {
    if (t.K < 1 || t.K > kMaxRefit) return hipErrorInvalidValue;
    int64_t nmax = 0;
    for (int p = 0; p < t.K; ++p) nmax = std::max(nmax, t.p[p].N);
    const unsigned nblk = (unsigned)((nmax + kSuRows - 1) / kSuRows), nb = (unsigned)((nmax + kBlock - 1) / kBlock);
    const unsigned K = (unsigned)t.K;
    hipLaunchKernelGGL(k_refit_sums_b, dim3(nblk, K), dim3(kBlock), 0, s, t, 0);
    hipLaunchKernelGGL(k_refit_means_b, dim3(1, K), dim3(64), 0, s, t);
    hipLaunchKernelGGL(k_refit_sums_b, dim3(nblk, K), dim3(kBlock), 0, s, t, 2);
    hipLaunchKernelGGL(k_refit_fit_b, dim3(1, K), dim3(64), 0, s, t);
    hipLaunchKernelGGL(k_refit_start_b, dim3(nb, K), dim3(kBlock), 0, s, t);
    hipLaunchKernelGGL(k_refit_start_final_b, dim3(1, K), dim3(64), 0, s, t);
    hipLaunchKernelGGL(k_refit_shift_b, dim3(1, K), dim3(kBlock), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_setup(const double* X, const double* ybar, int64_t N, int n, double gamma, double* su,
                        double* part, double* y0, double* xi0, DevState* st, hipStream_t s) {
    const int64_t rows = kSuRows;
    const int nblk = (int)((N + rows - 1) / rows);
    hipLaunchKernelGGL(k_su_sums, dim3(nblk), dim3(kBlock), 0, s, X, ybar, N, n, rows, (const double*)su, 0, part);
    hipLaunchKernelGGL(k_su_means_final, dim3(1), dim3(64), 0, s, (const double*)part, nblk, N, n, su, st);
    hipLaunchKernelGGL(k_su_sums, dim3(nblk), dim3(kBlock), 0, s, X, ybar, N, n, rows, (const double*)su, 1, part);
    hipLaunchKernelGGL(k_su_eig_final, dim3(1), dim3(kBlock), 0, s, (const double*)part, nblk, n, su);
    const int nb = (int)((N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_su_sigma2, dim3(nb), dim3(kBlock), 0, s, X, N, n, (const double*)su, part);
    hipLaunchKernelGGL(k_su_sigma2_final, dim3(1), dim3(64), 0, s, (const double*)part, nb, st);
    hipLaunchKernelGGL(k_su_start, dim3(nb), dim3(kBlock), 0, s, X, ybar, N, n, (const double*)su, y0, xi0, part);
    hipLaunchKernelGGL(k_su_start_final, dim3(1), dim3(64), 0, s, (const double*)part, nb, N, n, gamma,
                       (const double*)su, st);
    return hipGetLastError();
}

}  // namespace cr
