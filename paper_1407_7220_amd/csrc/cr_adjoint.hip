// gfx950 kernels of the reverse-mode (adjoint) pass through the fixed-schedule
// ALCC/MAPG map (Fig. 3 with a fixed number of Fig. 4 steps per iteration).
//
// One MAPG step maps (y^(1)_{l-1}, y^(2)_l) to (y^(1)_l, y^(2)_{l+1}):
//   v   = y^(2) - S grad P_k(y^(2)),       S = diag(s^y, s^xi)
//   y^(1)_l = Proj(v),  y^(2)_{l+1} = (1 + beta_l) y^(1)_l - beta_l y^(1)_{l-1}
// (the same for xi).  grad P_k = (z-part)/mu - A^T (A z - theta)_- has the
// Jacobian H = diag(1/mu, gamma/mu) + A^T M A with the pair mask
// M = diag(m_ij), m_ij = [theta_ij - r_ij > 0].  Its adjoint, for the adjoint
// v-bar of v, is
//   y^(2)-bar = v-bar - H S v-bar,
//   theta-bar += M A S v-bar,   ybar-bar += s^y vy-bar / mu,
// and the derivative of <S v-bar, grad P_k> in X.  With (a, b) = S v-bar,
// rho = A1 a + A2 b and z = m rho, this is one pass over the pairs:
//   (A^T z)        rowsum(z) - colsum(z);  -sum_i z_ij x_i + colsum_j(z) x_j
//   X-bar_m       += sum_j z_mj xi_j - sum_j w_mj b_j - colsum_m(z) xi_m + colsum_m(W) b_m
// and the multiplier step theta_{k+1} = s (A y_k + A2 xi_k - theta_k)_- gives
// the same structure with z = s m thetabar_{k+1} and W = 0.
//
// The pass keeps the forward pass's tiling and operands: the residual tile R is
// recomputed with the same MFMA chain on the same operands, so the mask is
// bit-identical to the forward's; rho is a second MFMA chain on the direction
// operands; Z^T [X 1] is the forward's column contraction with W replaced by
// Z.  The row-direction terms sum over the column index, which the MFMA
// accumulator layout does not contract: each lane forms its four columns'
// products against the staged xi_j and b_j (LDS, [k][column]) and a 16-lane
// DPP sum finishes the row.
#include "cr_device.h"
#include "cr_ops.h"

namespace cr {

template <typename T> struct AdjTile {
    static constexpr int TW = Tr<T>::TW;
    static constexpr int NW = 16 * TW;            // columns of one workgroup
    static constexpr int kCsum = 32768;           // wave column-sum accumulators (as in the forward pass)
    static constexpr int kCw = kWaves * 4 * NW * (int)sizeof(T);
    static constexpr int kStage = 2 * 32 * NW * (int)sizeof(T);
    static constexpr int kLds = kCsum + kCw + kStage;
};

// NST staging sets of tile operands (2 while the registers allow, else 1).
template <typename T, int KS, int MODE>
__global__ __launch_bounds__(kBlock, 2) void k_adj_pass(AdjPassArgs a) {
    constexpr int NST = (KS <= 3 || (KS == 4 && sizeof(T) == 4)) ? 2 : 1;
    typedef PlainOps<T, KS, 1> Ops;
    typedef typename Ops::acc_t acc_t;
    constexpr int TW = Ops::TW;
    constexpr int NKB = Ops::NKB;
    constexpr int NW = AdjTile<T>::NW;
    constexpr int KX = 4 * KS;                    // staged k slots (>= n + 1)
    __shared__ __align__(16) char lds[AdjTile<T>::kLds];
    T* sx = reinterpret_cast<T*>(lds + AdjTile<T>::kCsum + AdjTile<T>::kCw);   // [KX][NW]  -xi_jk
    T* sb = sx + KX * NW;                                                          // [KX][NW]  -b_jk

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int strip = blockIdx.x, chunk = blockIdx.y;
    const int64_t J0 = (int64_t)strip * NW;
    const int64_t I0 = (int64_t)chunk * a.rows_per_chunk;
    const int64_t I1 = min(I0 + (int64_t)a.rows_per_chunk, a.Nrow);
    const int64_t jl = J0 + TW * c;
    const int n = a.n;

    // stage -xi_j (and -b_j) of this workgroup's columns, k-major
    {
        const T* xa = (const T*)a.xiaug;
        const T* da = (const T*)a.diraug;
        for (int e = threadIdx.x; e < KX * NW; e += kBlock) {
            const int k = e / NW, jj = e - k * NW;
            const int64_t j = J0 + jj;
            T vx = (T)0, vb = (T)0;
            if (k < n) {
                vx = xa[j * a.kp + k];
                if (MODE == 0) vb = da[j * a.kp + k];
            }
            sx[k * NW + jj] = vx;
            sb[k * NW + jj] = vb;
        }
    }

    PassArgs pa{};
    pa.xp = a.xp;
    pa.xiaug = a.xiaug;
    typename Ops::Breg breg, dreg;
    Ops::load_breg(breg, pa, jl, g);
    if (MODE == 0) {
        pa.xiaug = a.diraug;
        Ops::load_breg(dreg, pa, jl, g);
    }

    acc_t cacc[TW][NKB];
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) cacc[t][kb] = acc_t{0, 0, 0, 0};
    T cw[TW];
#pragma unroll
    for (int t = 0; t < TW; ++t) cw[t] = (T)0;

    T* __restrict__ thetabar = (T*)a.thetabar;
    const bool tb_read = (MODE == 1) || a.tb_mode == 1;
    const bool tb_write = a.tb_mode != 0;
    const T scale = (T)a.scale;

    // Buffer views of this workgroup's rows (as in the forward pass): fixed
    // per-lane offsets, the tile step in the scalar offset, zeros past the rows.
    const uint32_t rows = (uint32_t)(I1 - I0);
    const uint32_t row_bytes = (uint32_t)a.ld * (uint32_t)sizeof(T);
    const rsrc_t th_r = make_rsrc((const T*)a.theta + I0 * a.ld + J0, rows * row_bytes);
    const rsrc_t tb_r = make_rsrc(tb_read ? thetabar + I0 * a.ld + J0 : (const T*)a.theta + I0 * a.ld + J0,
                                  rows * row_bytes);
    const rsrc_t xp_r = make_rsrc((const char*)a.xp + (I0 >> 4) * 64 * Ops::XPB, (rows >> 4) * 64u * Ops::XPB);
    const rsrc_t y_r = make_rsrc((const T*)a.ycol + I0, rows * (uint32_t)sizeof(T));
    const rsrc_t a_r = make_rsrc((const T*)a.acol + I0, rows * (uint32_t)sizeof(T));
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
    const int64_t first = I0 + 16 * wave;
    const int ntile = (int)((I1 - first + 16 * kWaves - 1) / (16 * kWaves));

    struct Stage {
        typename Ops::Xop xop;
        T yv[4], av[4];
        V16<T> th[4], tb[4];
    };
    auto load_tile = [&](int m, Stage& S) {
        const uint32_t mm = (uint32_t)m;
        Ops::load_xop_b(S.xop, xp_r, xp_vo, mm * xp_step);
        if constexpr (sizeof(T) == 4) {
            // rows 4g .. 4g + 3 of the tile: one 16-byte load each
            const V16<T> ty = bld16<T>(y_r, y_vo[0], mm * y_step);
            V16<T> ta;
            if (MODE == 0) ta = bld16<T>(a_r, y_vo[0], mm * y_step);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                S.yv[e] = ty.v[e];
                S.av[e] = MODE == 0 ? ta.v[e] : (T)0;
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                S.yv[v] = (T)bld8(y_r, y_vo[v], mm * y_step);
                S.av[v] = MODE == 0 ? (T)bld8(a_r, y_vo[v], mm * y_step) : (T)0;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            S.th[v] = bld16<T>(th_r, th_vo[v], mm * th_step);
            if (tb_read) S.tb[v] = bld16<T>(tb_r, th_vo[v], mm * th_step);
            else {
#pragma unroll
                for (int t = 0; t < TW; ++t) S.tb[v].v[t] = (T)0;
            }
        }
    };

    auto process = [&](int m, const Stage& S) {
        const int64_t i0 = first + 16 * kWaves * (int64_t)m;
        acc_t R[TW];
        Ops::residual(R, S.xop, breg, S.yv);
        acc_t P[TW];
        if (MODE == 0) Ops::residual(P, S.xop, dreg, S.av);

        const bool edge = (i0 < J0 + NW && i0 + 16 > J0) || (J0 + NW > a.N) || (i0 + 16 > a.N);
        // tile-relative indices: pair (i0 + r, J0 + q) is a constraint iff r < rlim, q < qlim, r + dij != q
        const int rlim = (int)min((int64_t)16, a.N - i0);
        const int qlim = (int)min((int64_t)NW, a.N - J0);
        const int dij = (int)max((int64_t)-64, min((int64_t)64, i0 - J0));
        T W[TW][4], Z[TW][4];
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T d = S.th[v].v[t] - R[t][v];
                bool mk = d > (T)0;
                if (edge) {
                    const int r = orow<Ops>(g, v), q = TW * c + t;
                    mk = mk && r < rlim && q < qlim && r + dij != q;
                }
                if (MODE == 0) {
                    W[t][v] = mk ? d : (T)0;
                    Z[t][v] = mk ? P[t][v] : (T)0;
                } else {
                    W[t][v] = (T)0;
                    Z[t][v] = mk ? scale * S.tb[v].v[t] : (T)0;
                }
            }
        if (tb_write) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                V16<T> o;
#pragma unroll
                for (int t = 0; t < TW; ++t) o.v[t] = MODE == 0 ? S.tb[v].v[t] + Z[t][v] : Z[t][v];
                st16(thetabar + (i0 + orow<Ops>(g, v)) * a.ld + jl, o);
            }
        }

        Ops::colsums(cacc, Z, S.xop);
        if (MODE == 0) {
#pragma unroll
            for (int t = 0; t < TW; ++t) cw[t] += (W[t][0] + W[t][1]) + (W[t][2] + W[t][3]);
        }

        if constexpr (sizeof(T) == 4) {
            // Row-direction terms and the row sums of z as one MFMA contraction
            // over the tile's 64 columns: D[i][k] = sum_j W_ij (-b_jk) + Z_ij xi_jk
            // for k < n, and D[i][n] = sum_j Z_ij.  The W and Z tiles go through this
            // wave's LDS rows ([16][NW], row-major) from the accumulator layout
            // (lane (g, c): rows 4g + v, columns TW c .. TW c + 3) to the A layout
            // (lane (g, c): row c, columns 16 g .. 16 g + 15, MFMA step s <-> column
            // 16 g + s); the staged -b (sb) and -xi (sx) give B (feature 16 kb + c).
            static_assert(kWaves * 2 * 16 * NW * 4 <= AdjTile<T>::kCsum, "W/Z staging");
            float* wl = reinterpret_cast<float*>(lds) + wave * (2 * 16 * NW);
            float* zl = wl + 16 * NW;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                V16<T> zo;
#pragma unroll
                for (int t = 0; t < TW; ++t) zo.v[t] = Z[t][v];
                st16(zl + (4 * g + v) * NW + TW * c, zo);
                if (MODE == 0) {
                    V16<T> wo;
#pragma unroll
                    for (int t = 0; t < TW; ++t) wo.v[t] = W[t][v];
                    st16(wl + (4 * g + v) * NW + TW * c, wo);
                }
            }
            V16<T> aw[4], az[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                az[q] = ld16(zl + c * NW + 16 * g + 4 * q);
                if (MODE == 0) aw[q] = ld16(wl + c * NW + 16 * g + 4 * q);
            }
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                const int f = 16 * kb + c;            // feature of this lane's B column
                V16<T> bb[4], bx[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) { bb[q].v[e] = (T)0; bx[q].v[e] = (T)0; }
                    if (f < KX) {
                        bx[q] = ld16(sx + f * NW + 16 * g + 4 * q);
                        if (MODE == 0) bb[q] = ld16(sb + f * NW + 16 * g + 4 * q);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) bx[q].v[e] = f == n ? (T)1 : -bx[q].v[e];
                }
                acc_t dz = acc_t{0, 0, 0, 0}, dw = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        dz = mfma4(az[q].v[e], bx[q].v[e], dz);
                        if (MODE == 0) dw = mfma4(aw[q].v[e], bb[q].v[e], dw);
                    }
                // lane (g, c) holds D[4g + v][f]
                if (f < n) {
                    T* rv = (T*)a.rowvpart;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        rv[((int64_t)strip * a.Nrow + i0 + 4 * g + v) * n + f] = MODE == 0 ? dw[v] + dz[v] : dz[v];
                } else if (f == n) {
                    T* dst = (T*)a.rowpart + (int64_t)strip * a.Nrow + i0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) dst[4 * g + v] = dz[v];
                }
            }
            return;
        }

        // row sums of z
        T rs[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            T sm = Z[0][v];
#pragma unroll
            for (int t = 1; t < TW; ++t) sm += Z[t][v];
            rs[v] = row16_sum(sm);
        }
        if (c == 0) {
            T* dst = (T*)a.rowpart + (int64_t)strip * a.Nrow + i0;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[orow<Ops>(g, v)] = rs[v];
        }

        // row-direction terms sum_j (w_ij (-b_jk) - z_ij (-xi_jk)); lane c keeps k = c and k = 16 + c
        T keep[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) keep[h][v] = (T)0;
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            if (k >= n) break;
            const V16<T> xv = *reinterpret_cast<const V16<T>*>(sx + k * NW + TW * c);
            V16<T> bv;
            if (MODE == 0) bv = *reinterpret_cast<const V16<T>*>(sb + k * NW + TW * c);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T sm = (T)0;
#pragma unroll
                for (int t = 0; t < TW; ++t) {
                    if (MODE == 0) sm += W[t][v] * bv.v[t];
                    sm -= Z[t][v] * xv.v[t];
                }
                sm = row16_sum(sm);
                if (c == (k & 15)) keep[k >> 4][v] = sm;
            }
        }
        T* rv = (T*)a.rowvpart;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 16 * h + c;
            if (k < n) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    rv[((int64_t)strip * a.Nrow + i0 + orow<Ops>(g, v)) * n + k] = keep[h][v];
            }
        }
    };

    __syncthreads();
    // staging sets; the scheduling barriers keep each set's loads together so
    // that one set stays in flight while another is processed
    Stage st[NST];
#pragma unroll
    for (int b = 0; b < NST; ++b) {
        load_tile(b, st[b]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma nounroll
    for (int m = 0; m < ntile; m += NST) {
#pragma unroll
        for (int b = 0; b < NST; ++b) {
            if (m + b < ntile) process(m + b, st[b]);
            __builtin_amdgcn_sched_barrier(0);
            load_tile(m + b + NST, st[b]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // combine the 4 waves' column sums (fixed order) and write this chunk's partials
    // (the FP32 path staged its W and Z tiles in this area: every wave done first)
    if constexpr (sizeof(T) == 4) __syncthreads();
    typedef T cl_t[TW][NKB][4][64];
    cl_t* cl = reinterpret_cast<cl_t*>(lds);
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) cl[wave][t][kb][v][lane] = cacc[t][kb][v];
    T* cwl = reinterpret_cast<T*>(lds + AdjTile<T>::kCsum);   // [wave][g][NW]
    if (MODE == 0) {
#pragma unroll
        for (int t = 0; t < TW; ++t) cwl[(wave * 4 + g) * NW + TW * c + t] = cw[t];
    }
    __syncthreads();
    T* cpart = (T*)a.cpart;
    for (int e = threadIdx.x; e < TW * NKB * 4 * 64; e += kBlock) {
        const int ln = e & 63, v = (e >> 6) & 3, rest = e >> 8;
        const int kb = rest % NKB, t = rest / NKB;
        const T s = ((cl[0][t][kb][v][ln] + cl[1][t][kb][v][ln]) + cl[2][t][kb][v][ln]) + cl[3][t][kb][v][ln];
        const int64_t j = J0 + TW * orow<Ops>(ln >> 4, v) + t;
        const int kk = 16 * kb + (ln & 15);
        if (kk < a.nc) cpart[((int64_t)chunk * a.ld + j) * a.nc + kk] = s;
    }
    if (MODE == 0) {
        T* cwp = (T*)a.cwpart + (int64_t)chunk * a.ld + J0;
        for (int e = threadIdx.x; e < NW; e += kBlock) {
            T s = (T)0;
            for (int q = 0; q < kWaves * 4; ++q) s += cwl[q * NW + e];
            cwp[e] = s;
        }
    }
}

template <int G>
__device__ __forceinline__ double adj_group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sums of the pass partials for point m, then the adjoint formulas (header).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_adj_reduce(AdjReduceArgs a) {
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t m = (int64_t)blockIdx.x * PER + threadIdx.x / G;
    const bool valid = m < a.N;
    const int n = a.n, nc = a.nc;
    const T* rowpart = (const T*)a.rowpart;
    const T* rowvpart = (const T*)a.rowvpart;
    const T* cpart = (const T*)a.cpart;
    const T* cwpart = (const T*)a.cwpart;
    // Partial sums through buffer views based at the wave's first point, in
    // batches whose loads are all issued before any sum (entries past the
    // last strip or chunk read as zeros):
    //   rowpart [strip][i]      lane k: strips k, k + G, ...       (in order)
    //   rowvpart[strip][i][k]   lane k < n: every strip, four sums (strip q into sum q % 4)
    //   cpart   [chunk][j][k]   lane k < n + 1: every chunk        (in order)
    //   cwpart  [chunk][j]      lane n: every chunk                (in order)
    constexpr int URS = 8, URV = 32, UCK = 16;
    const int p = (threadIdx.x & 63) / G;
    const int64_t m0 = __builtin_amdgcn_readfirstlane((int)(m - p));   // the same in every lane of the wave
    const uint32_t esz = (uint32_t)sizeof(T);
    auto view = [&](const T* base, uint64_t bytes) {
        return make_rsrc(base, (uint32_t)min(bytes, (uint64_t)0xffffffffu));
    };
    // this lane's own values (clamped addresses; used only by lanes that own them)
    const int64_t mc = valid ? m : a.N - 1;
    const int64_t ec = mc * n + min(k, n - 1);
    const bool own_y = k == n;
    const double o_vb = a.mode == 0 ? (own_y ? a.vb_y[mc] : a.vb_xi[ec]) : 0.0;
    const double o_acc = own_y ? (a.mode == 0 ? a.dybar[mc] : a.out_y[mc]) : a.dX[ec];
    const double o_out = a.mode == 0 ? 0.0 : (own_y ? 0.0 : a.out_xi[ec]);
    const double o_x = a.X[ec], o_xi = a.xi[ec];
    double rs = 0.0, rv = 0.0, ck = 0.0, cw = 0.0;
    {
        const uint32_t vo = ((uint32_t)k * (uint32_t)a.Nrow + (uint32_t)p) * esz;
        const uint32_t so = (uint32_t)G * (uint32_t)a.Nrow * esz;
        for (int s0 = 0; s0 < a.strips; s0 += G * URS) {
            const rsrc_t r = view(rowpart + (int64_t)s0 * a.Nrow + m0, (uint64_t)(a.strips - s0) * a.Nrow * esz);
            T u[URS];
#pragma unroll
            for (int e = 0; e < URS; ++e) u[e] = bld_t<T>(r, vo, (uint32_t)e * so);
#pragma unroll
            for (int e = 0; e < URS; ++e) rs += (double)u[e];
        }
    }
    {
        const uint32_t vo = ((uint32_t)p * (uint32_t)n + (uint32_t)k) * esz;
        const uint32_t so = (uint32_t)a.Nrow * (uint32_t)n * esz;
        double r4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < a.strips; q0 += URV) {
            // four views of 8 strips each keep the scalar offsets below 2^31
            T u[URV];
#pragma unroll
            for (int sv = 0; sv < URV / 8; ++sv) {
                const int qs = q0 + 8 * sv;
                const rsrc_t r = view(rowvpart + ((int64_t)qs * a.Nrow + m0) * n,
                                      qs < a.strips ? (uint64_t)(a.strips - qs) * a.Nrow * n * esz : 0);
#pragma unroll
                for (int e = 0; e < 8; ++e) u[8 * sv + e] = bld_t<T>(r, vo, (uint32_t)e * so);
            }
#pragma unroll
            for (int e = 0; e < URV; ++e) r4[e & 3] += (double)u[e];
        }
        rv = k < n ? (r4[0] + r4[1]) + (r4[2] + r4[3]) : 0.0;
    }
    {
        const uint32_t vo = ((uint32_t)p * (uint32_t)nc + (uint32_t)k) * esz;
        const uint32_t so = (uint32_t)(a.ld * nc) * esz;
        const uint32_t wvo = (uint32_t)p * esz, wso = (uint32_t)a.ld * esz;
        for (int h0 = 0; h0 < a.chunks; h0 += UCK) {
            const rsrc_t r = view(cpart + ((int64_t)h0 * a.ld + m0) * nc, (uint64_t)(a.chunks - h0) * a.ld * nc * esz);
            T u[UCK], w[UCK];
#pragma unroll
            for (int e = 0; e < UCK; ++e) u[e] = bld_t<T>(r, vo, (uint32_t)e * so);
            if (a.mode == 0) {
                const rsrc_t rw = view(cwpart + (int64_t)h0 * a.ld + m0, (uint64_t)(a.chunks - h0) * a.ld * esz);
#pragma unroll
                for (int e = 0; e < UCK; ++e) w[e] = bld_t<T>(rw, wvo, (uint32_t)e * wso);
            } else {
#pragma unroll
                for (int e = 0; e < UCK; ++e) w[e] = (T)0;
            }
#pragma unroll
            for (int e = 0; e < UCK; ++e) { ck += (double)u[e]; cw += (double)w[e]; }
        }
        if (k >= nc) ck = 0.0;
        if (k != n) cw = 0.0;
    }
    rs = adj_group_sum<G>(rs);
    const int base = (threadIdx.x & 63) & ~(G - 1);
    const double czn = __shfl(ck, base + n);      // colsum_m(z)
    const double cwn = __shfl(cw, base + n);      // colsum_m(W)
    if (!valid) return;
    if (k == n) {
        if (a.mode == 0) {
            const double vb = o_vb;
            const double at = a.sy * vb;
            a.out_y[m] = vb - at / a.mu - (rs - czn);
            a.dybar[m] = o_acc + at / a.mu;
        } else {
            a.out_y[m] = o_acc + -(rs - czn);
        }
    } else if (k < n) {
        const int64_t e = m * n + k;
        const double xmk = o_x;
        if (a.mode == 0) {
            const double vb = o_vb;
            const double bt = a.sxi * vb;
            a.out_xi[e] = vb - a.gamma * bt / a.mu + ck - czn * xmk;
            a.dX[e] = o_acc + (rv - czn * o_xi + cwn * bt);
        } else {
            a.out_xi[e] = o_out + (ck - czn * xmk);
            a.dX[e] = o_acc + (rv - czn * o_xi);
        }
    }
}

// Momentum adjoint: g1 = pb + (1 + beta) qb, pb <- -beta qb, and per-block
// pieces of <v_y - ybar, g1_y> and <v_xi, g1_xi> for the projection adjoint.
template <int G>
__global__ __launch_bounds__(kBlock) void k_adj_momentum(AdjVecArgs a) {
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t m = (int64_t)blockIdx.x * PER + threadIdx.x / G;
    const bool valid = m < a.N;
    const int n = a.n;
    double dy = 0.0, dx = 0.0;
    if (valid && k == n) {
        const double q = a.qb_y[m];
        const double g1 = a.pb_y[m] + (1.0 + a.beta) * q;
        a.g1_y[m] = g1;
        a.pb_y[m] = -a.beta * q;
        dy = (a.v_y[m] - a.ybar[m]) * g1;
    } else if (valid && k < n) {
        const int64_t e = m * n + k;
        const double q = a.qb_xi[e];
        const double g1 = a.pb_xi[e] + (1.0 + a.beta) * q;
        a.g1_xi[e] = g1;
        a.pb_xi[e] = -a.beta * q;
        dx = a.v_xi[e] * g1;
    }
    const double b0 = block_reduce(dy, 0), b1 = block_reduce(dx, 0);
    if (threadIdx.x == 0) { a.blockpart[blockIdx.x * 4 + 0] = b0; a.blockpart[blockIdx.x * 4 + 1] = b1; }
}

// Projection adjoint (ball of radius B around the centre, active when the
// forward norm exceeded B): vb = (B/|d|) (g1 - d <d, g1> / |d|^2), centre
// adjoint g1 - vb; then the direction operands (a, b) = (s^y vb_y, s^xi vb_xi).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_adj_project(AdjVecArgs a, int nblk) {
    constexpr int PER = kBlock / G;
    const int k = threadIdx.x % G;
    const int64_t m = (int64_t)blockIdx.x * PER + threadIdx.x / G;
    const bool valid = m < a.N;
    const int n = a.n;
    double sdy = 0.0, sdx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        sdy += a.blockpart[(int64_t)b * 4 + 0];
        sdx += a.blockpart[(int64_t)b * 4 + 1];
    }
    const double dy = block_reduce(sdy, 0), dx = block_reduce(sdx, 0);
    const double ny = a.nrm[0], nx = a.nrm[1];
    double prod = 0.0, at = 0.0;
    if (valid && k == n) {
        const double g1 = a.g1_y[m];
        double vb = g1;
        if (ny > a.By) {
            const double d = a.v_y[m] - a.ybar[m];
            vb = (a.By / ny) * (g1 - d * (dy / (ny * ny)));
            a.dybar[m] += g1 - vb;
        }
        a.vb_y[m] = vb;
        at = a.sy * vb;
        ((T*)a.acol)[m] = (T)at;
    } else if (valid && k < n) {
        const int64_t e = m * n + k;
        const double g1 = a.g1_xi[e];
        double vb = g1;
        if (nx > a.Bxi) vb = (a.Bxi / nx) * (g1 - a.v_xi[e] * (dx / (nx * nx)));
        a.vb_xi[e] = vb;
        const double bt = a.sxi * vb;
        ((T*)a.diraug)[m * a.kp + k] = (T)(-bt);
        prod = a.X[e] * bt;
    }
    const double d = adj_group_sum<G>(prod);         // x_m^T b_m
    if (valid && k == n) ((T*)a.diraug)[m * a.kp + n] = (T)(d - at);
}

__global__ __launch_bounds__(kBlock) void k_add(double* out, const double* x, const double* y, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) out[i] = x[i] + y[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int adj_group(int n) { return n + 1 <= 16 ? 16 : 32; }

int adj_vec_blocks(int64_t N, int n) {
    const int G = adj_group(n);
    return (int)((N * G + kBlock - 1) / kBlock);
}

template <typename T, int KS>
static void adj_pass_ks(const AdjPassArgs& a, dim3 grid, hipStream_t s) {
    if (a.mode == 0) hipLaunchKernelGGL((k_adj_pass<T, KS, 0>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_adj_pass<T, KS, 1>), grid, dim3(kBlock), 0, s, a);
}

template <typename T>
static hipError_t adj_pass_t(int ks, const AdjPassArgs& a, dim3 grid, hipStream_t s) {
    switch (ks) {
        case 1: adj_pass_ks<T, 1>(a, grid, s); break;
        case 2: adj_pass_ks<T, 2>(a, grid, s); break;
        case 3: adj_pass_ks<T, 3>(a, grid, s); break;
        case 4: adj_pass_ks<T, 4>(a, grid, s); break;
        case 5: adj_pass_ks<T, 5>(a, grid, s); break;
        case 6: adj_pass_ks<T, 6>(a, grid, s); break;
        case 7: adj_pass_ks<T, 7>(a, grid, s); break;
        case 8: adj_pass_ks<T, 8>(a, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj_pass(bool f64, int n, const AdjPassArgs& a, dim3 grid, hipStream_t s) {
    const int ks = ks_of(n);
    return f64 ? adj_pass_t<double>(ks, a, grid, s) : adj_pass_t<float>(ks, a, grid, s);
}

hipError_t launch_adj_reduce(bool f64, const AdjReduceArgs& a, hipStream_t s) {
    const int G = adj_group(a.n);
    const dim3 grid((unsigned)adj_vec_blocks(a.N, a.n));
    if (f64) {
        if (G == 16) hipLaunchKernelGGL((k_adj_reduce<double, 16>), grid, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_adj_reduce<double, 32>), grid, dim3(kBlock), 0, s, a);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_adj_reduce<float, 16>), grid, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_adj_reduce<float, 32>), grid, dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_adj_momentum(const AdjVecArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)adj_vec_blocks(a.N, a.n));
    if (adj_group(a.n) == 16) hipLaunchKernelGGL(k_adj_momentum<16>, grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_adj_momentum<32>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_project(bool f64, const AdjVecArgs& a, int nblk, hipStream_t s) {
    const dim3 grid((unsigned)adj_vec_blocks(a.N, a.n));
    const int G = adj_group(a.n);
    if (f64) {
        if (G == 16) hipLaunchKernelGGL((k_adj_project<double, 16>), grid, dim3(kBlock), 0, s, a, nblk);
        else hipLaunchKernelGGL((k_adj_project<double, 32>), grid, dim3(kBlock), 0, s, a, nblk);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_adj_project<float, 16>), grid, dim3(kBlock), 0, s, a, nblk);
        else hipLaunchKernelGGL((k_adj_project<float, 32>), grid, dim3(kBlock), 0, s, a, nblk);
    }
    return hipGetLastError();
}

hipError_t launch_add(double* out, const double* x, const double* y, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, out, x, y, count);
    return hipGetLastError();
}

}  // namespace cr
