// P-APG on the partial dual (Aybat & Wang, Sec. II-B to II-D, Fig. 2): the
// O(N^2) kernels between the block solves (gfx950).
//
// The points split into K index sets of Nbar consecutive points; pair (i, j)
// is a cross-block pair when i and j lie in different sets.  The multipliers
// of the cross-block rows of C = [A3 A4; I 0] (eq. "C") are the off-diagonal
// blocks of an N x N row-major FP64 array (zero inside the diagonal blocks),
// those of the rows y >= 0 a vector of N.  Two such arrays hold theta^(1)_{l-1}
// (tc) and theta^(1)_{l-2} (tp); the extrapolated point of Fig. 2 step 4,
// theta^(2)_l = tc + beta (tc - tp), is formed on the fly wherever it is read.
//
//  k_papg_colsum, k_papg_lin
//               data of the block problems of step 1 (eq. "g_gamma" after
//               completing the square): ybar + yshift + u and centres v/gamma,
//               u = A3^T theta2 + theta2_y, v = A4^T theta2: column partials
//               over row chunks (thread <-> column), then one workgroup per
//               point for its row sum and the combination.
//  k_papg_step2 step 2 before the ball: theta^(1)_l = max(theta2 - C eta / L, 0)
//               written over tp, with per-workgroup sums of theta^2, of the
//               squared negative parts of the cross residuals and of
//               theta2 * (C eta).  Tiles of 32 rows x 256 columns.
//  k_papg_ball  ||theta||, the scale of the projection onto the ball of Q2.
//  k_papg_scale the scale applied (only when the ball is active).
//  k_papg_capply, k_papg_pnorm, k_papg_pstart
//               optional power iteration for sigma_max(C)^2 (the step constant).
//
// The projection onto Q2 = {theta >= 0, ||theta|| <= B} is the clip at zero
// followed by a radial scale: the ball is centred at the origin and the
// orthant is a cone.
#include "cr_device.h"
#include "cr_ops.h"

namespace cr {

constexpr int kPapgMaxN = 32;
constexpr int kPapgBatch = 8;     // rows whose loads are issued together

__device__ __forceinline__ double theta2_at(const PapgArgs& a, int64_t idx) {
    const double c = a.tc[idx];
    return c + a.beta * (c - a.tp[idx]);
}

// Column sums of theta2 over one chunk of papg_col_rows(N) rows, for every column
// l: c_l = sum_i theta2_il and w_lk = sum_i theta2_il x_ik over the rows i
// outside l's index set.  Thread <-> column, so every row is one coalesced
// read per array; x_i is the same for the whole workgroup.
template <int NM>
__global__ __launch_bounds__(kBlock) void k_papg_colsum(PapgArgs a) {
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t rows = papg_col_rows(N);
    const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(i0 + rows, N);
    const bool vl = l < N;
    const int64_t lb0 = vl ? l / a.Nbar * a.Nbar : -1, lb1 = lb0 + a.Nbar;   // l's index set [lb0, lb1)
    double c = 0.0, w[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) w[k] = 0.0;
    // rows in batches of kPapgBatch: every load of a batch is issued first
    for (int64_t ib = i0; ib < i1; ib += kPapgBatch) {
        double tc[kPapgBatch], tp[kPapgBatch];
#pragma unroll
        for (int u = 0; u < kPapgBatch; ++u) {
            const int64_t i = ib + u;
            const bool ok = vl && i < i1;
            tc[u] = ok ? a.tc[i * N + l] : 0.0;
            tp[u] = ok ? a.tp[i * N + l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPapgBatch; ++u) {
            const int64_t i = ib + u;
            if (!(vl && i < i1) || (i >= lb0 && i < lb1)) continue;
            const double t = tc[u] + a.beta * (tc[u] - tp[u]);
            c += t;
#pragma unroll
            for (int k = 0; k < NM; ++k)
                if (k < n) w[k] += t * a.X[i * n + k];
        }
    }
    if (vl) {
        double* out = a.cpart + ((int64_t)blockIdx.y * N + l) * (n + 1);
        out[0] = c;
#pragma unroll
        for (int k = 0; k < NM; ++k)
            if (k < n) out[1 + k] = w[k];
    }
}

// Block data of step 1 for point l (one workgroup): the row sum of theta2 over
// the columns outside l's set (coalesced), the column sums from the chunk
// partials of k_papg_colsum (chunks in order), then
//   u_l = rowsum_l - colsum_l + theta2_y,l,   v_lk = -(w_lk - x_lk colsum_l).
__global__ __launch_bounds__(kBlock) void k_papg_lin(PapgArgs a) {
    const int64_t l = blockIdx.x;
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t lb0 = l / a.Nbar * a.Nbar, lb1 = lb0 + a.Nbar;    // l's index set
    double su = 0.0;
    for (int64_t m = threadIdx.x; m < N; m += kBlock)
        if (m < lb0 || m >= lb1) su += theta2_at(a, l * N + m);    // pair (l, m): +y_l
    su = block_reduce(su, 0);
    __shared__ double cs[kPapgMaxN + 1];
    const int64_t chunks = papg_col_chunks(N);
    if (threadIdx.x <= n) {
        // chunks in order, kPapgBatch loads in flight
        double t = 0.0;
        for (int64_t q0 = 0; q0 < chunks; q0 += kPapgBatch) {
            double v[kPapgBatch];
#pragma unroll
            for (int u = 0; u < kPapgBatch; ++u)
                v[u] = q0 + u < chunks ? a.cpart[((q0 + u) * N + l) * (n + 1) + threadIdx.x] : 0.0;
#pragma unroll
            for (int u = 0; u < kPapgBatch; ++u) t += v[u];
        }
        cs[threadIdx.x] = t;                                     // [colsum, w_l0 .. w_l(n-1)]
    }
    __syncthreads();
    if (threadIdx.x <= n) {
        const double colsum = cs[0];
        if (threadIdx.x == n) {
            const double ty = a.tyc[l] + a.beta * (a.tyc[l] - a.typ[l]);
            a.ybs[l] = (a.ybar[l] + a.yshift) + ((su - colsum) + ty);
        } else {
            const int k = threadIdx.x;
            a.shift[l * n + k] = -(cs[1 + k] - a.X[l * n + k] * colsum) / a.gamma;
        }
    }
}

// Step 2 over a tile of kPapgStepRows rows and kBlock columns: thread <-> column
// j keeps x_j, y_j and the slope xi'_j + c_j in registers and walks the rows
// (x_i, y_i the same for the whole workgroup), so every theta row segment is
// one coalesced read of each array and one coalesced write.  The workgroups of
// column block 0 also take the rows y >= 0 of their row range.
template <int NM>
__global__ __launch_bounds__(kBlock) void k_papg_step2(PapgArgs a) {
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * kPapgStepRows, i1 = min(i0 + kPapgStepRows, N);
    const bool vj = j < N;
    const int64_t jb0 = vj ? j / a.Nbar * a.Nbar : -1, jb1 = jb0 + a.Nbar;   // j's index set [jb0, jb1)
    // the tile's rows: x_i (n values) and y_i, staged once
    __shared__ double xs[kPapgStepRows][kPapgMaxN + 1];
    for (int e = threadIdx.x; e < kPapgStepRows * (n + 1); e += kBlock) {
        const int r = e / (n + 1), k = e % (n + 1);
        const int64_t i = i0 + r;
        xs[r][k] = i < i1 ? (k < n ? a.X[i * n + k] : a.y[i]) : 0.0;
    }
    __syncthreads();
    double xj[NM], sj[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        xj[k] = (vj && k < n) ? a.X[j * n + k] : 0.0;
        sj[k] = (vj && k < n) ? a.xis[j * n + k] + a.shift[j * n + k] : 0.0;
    }
    const double yj = vj ? a.y[j] : 0.0;
    const double L = a.L;
    double s2 = 0.0, neg2 = 0.0, gap = 0.0;
    // rows in batches of kPapgBatch: the batch's loads are issued before its
    // stores (which overwrite tp in place, element by element)
    for (int64_t ib = i0; ib < i1; ib += kPapgBatch) {
        double tc[kPapgBatch], tq[kPapgBatch];
#pragma unroll
        for (int u = 0; u < kPapgBatch; ++u) {
            const int64_t i = ib + u;
            const bool ok = vj && i < i1;
            tc[u] = ok ? a.tc[i * N + j] : 0.0;
            tq[u] = ok ? a.tp[i * N + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kPapgBatch; ++u) {
            const int64_t i = ib + u;
            if (!(vj && i < i1)) continue;
            double tn = 0.0;
            if (i < jb0 || i >= jb1) {
                // r_ij = y_i - y_j - xi_j^T (x_i - x_j), xi_j = xi'_j + c_j
                const double* xr = xs[ib + u - i0];
                double h = 0.0;
#pragma unroll
                for (int k = 0; k < NM; ++k)
                    if (k < n) h += sj[k] * (xr[k] - xj[k]);
                const double r = (xr[n] - yj) - h;
                const double t2 = tc[u] + a.beta * (tc[u] - tq[u]);
                tn = fmax(t2 - r / L, 0.0);
                if (r < 0.0) neg2 += r * r;
                gap += t2 * r;
            }
            a.tp[i * N + j] = tn;
            s2 += tn * tn;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < i1 - i0) {
        const int64_t i = i0 + threadIdx.x;
        const double yi = a.y[i];
        const double ty = a.tyc[i] + a.beta * (a.tyc[i] - a.typ[i]);
        const double tn = fmax(ty - yi / L, 0.0);
        a.typ[i] = tn;
        s2 += tn * tn;
        gap += ty * yi;
    }
    block_sum2(s2, neg2);
    gap = block_reduce(gap, 0);
    if (threadIdx.x == 0) {
        const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.part[3 * wg] = s2;
        a.part[3 * wg + 1] = neg2;
        a.part[3 * wg + 2] = gap;
    }
}

// sigma_max(C)^2 by power iteration on C^T C (an option of cr_papg).  One
// step: R = C v for v = (y, xi) (this kernel: the cross residuals r_ij into
// the tc array, zero inside the diagonal blocks, with the per-workgroup sums of
// r^2 and, in column block 0, of y^2), then C^T (R, y) by k_papg_colsum and
// k_papg_lin (theta2 = R, theta2_y = y, zero data, gamma = 1), then
// k_papg_pnorm.  Tiles as in k_papg_step2.
template <int NM>
__global__ __launch_bounds__(kBlock) void k_papg_capply(PapgArgs a) {
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * kPapgStepRows, i1 = min(i0 + kPapgStepRows, N);
    const bool vj = j < N;
    const int64_t jb0 = vj ? j / a.Nbar * a.Nbar : -1, jb1 = jb0 + a.Nbar;
    __shared__ double xs[kPapgStepRows][kPapgMaxN + 1];
    for (int e = threadIdx.x; e < kPapgStepRows * (n + 1); e += kBlock) {
        const int r = e / (n + 1), k = e % (n + 1);
        const int64_t i = i0 + r;
        xs[r][k] = i < i1 ? (k < n ? a.X[i * n + k] : a.y[i]) : 0.0;
    }
    __syncthreads();
    double xj[NM], sj[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        xj[k] = (vj && k < n) ? a.X[j * n + k] : 0.0;
        sj[k] = (vj && k < n) ? a.xis[j * n + k] : 0.0;
    }
    const double yj = vj ? a.y[j] : 0.0;
    double s2 = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        if (!vj) continue;
        double r = 0.0;
        if (i < jb0 || i >= jb1) {
            const double* xr = xs[i - i0];
            double h = 0.0;
#pragma unroll
            for (int k = 0; k < NM; ++k)
                if (k < n) h += sj[k] * (xr[k] - xj[k]);
            r = (xr[n] - yj) - h;
        }
        a.tc[i * N + j] = r;
        s2 += r * r;
    }
    if (blockIdx.x == 0 && threadIdx.x < i1 - i0) {
        const double yi = a.y[i0 + threadIdx.x];
        s2 += yi * yi;
    }
    s2 = block_reduce(s2, 0);
    if (threadIdx.x == 0) {
        const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.part[3 * wg] = s2;
        a.part[3 * wg + 1] = 0.0;
        a.part[3 * wg + 2] = 0.0;
    }
}

// One workgroup: w = (ybs, shift) holds C^T C v (or, at the start, any vector);
// scal[4] <- ||C v||^2 from the capply partials (the Rayleigh quotient, v having
// unit norm), scal[5] <- ||w||, and v <- w / ||w|| into (y, xis).
__global__ __launch_bounds__(kBlock) void k_papg_pnorm(PapgArgs a, double* vy, double* vxi, int with_rayleigh) {
    const int64_t N = a.N, Nn = a.N * a.n;
    double q = 0.0, w2 = 0.0;
    if (with_rayleigh) {
        const int64_t parts = papg_step_parts(N);
        for (int64_t e = threadIdx.x; e < parts; e += kBlock) q += a.part[3 * e];
    }
    for (int64_t e = threadIdx.x; e < N; e += kBlock) w2 += a.ybs[e] * a.ybs[e];
    for (int64_t e = threadIdx.x; e < Nn; e += kBlock) w2 += a.shift[e] * a.shift[e];
    block_sum2(q, w2);
    const double nw = sqrt(w2);
    const double inv = nw > 0.0 ? 1.0 / nw : 0.0;
    for (int64_t e = threadIdx.x; e < N; e += kBlock) vy[e] = a.ybs[e] * inv;
    for (int64_t e = threadIdx.x; e < Nn; e += kBlock) vxi[e] = a.shift[e] * inv;
    if (threadIdx.x == 0) {
        if (with_rayleigh) a.scal[4] = q;
        a.scal[5] = nw;
    }
}

// A fixed start for the power iteration: entries in [0.5, 1.5) from a
// counter-based integer hash of the index (no state, same on every call).
__global__ __launch_bounds__(kBlock) void k_papg_pstart(PapgArgs a) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t Nn = a.N * a.n;
    if (e >= a.N + Nn) return;
    uint64_t z = (uint64_t)e + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = 0.5 + (double)(z >> 11) * (1.0 / 9007199254740992.0);
    if (e < a.N) a.ybs[e] = u;
    else a.shift[e - a.N] = u;
}

__global__ __launch_bounds__(kBlock) void k_papg_ball(PapgArgs a) {
    double s = 0.0, g = 0.0, d = 0.0;
    const int64_t parts = papg_step_parts(a.N);
    for (int64_t i = threadIdx.x; i < parts; i += kBlock) {
        s += a.part[3 * i];
        g += a.part[3 * i + 1];
        d += a.part[3 * i + 2];
    }
    block_sum2(s, g);
    d = block_reduce(d, 0);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(s);
        const double sc = (a.B > 0.0 && isfinite(a.B) && nrm > a.B) ? a.B / nrm : 1.0;
        a.scal[0] = sc;
        a.scal[1] = nrm * sc;
        a.scal[2] = sqrt(g);
        a.scal[3] = d;
        a.trace[3 * a.it] = nrm * sc;
        a.trace[3 * a.it + 1] = sqrt(g);
        a.trace[3 * a.it + 2] = d;
    }
}

__global__ __launch_bounds__(kBlock) void k_papg_scale(PapgArgs a) {
    const double sc = a.scal[0];
    if (sc == 1.0) return;
    const int64_t NN = a.N * a.N;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < NN + a.N; e += stride) {
        if (e < NN) a.tp[e] *= sc;
        else a.typ[e - NN] *= sc;
    }
}

__global__ __launch_bounds__(kBlock) void k_papg_out(PapgArgs a, double* y_out, double* xi_out) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t Nn = a.N * a.n;
    if (e < Nn) xi_out[e] = a.xis[e] + a.shift[e];
    if (e < a.N) y_out[e] = a.y[e] - a.yshift;
}

// The per-thread arrays of the tiled kernels hold NM >= n slots.
hipError_t launch_papg_lin(const PapgArgs& a, hipStream_t s) {
    const unsigned cb = (unsigned)((a.N + kBlock - 1) / kBlock);
    const dim3 g(cb, (unsigned)papg_col_chunks(a.N));
    if (a.n <= 8) hipLaunchKernelGGL(k_papg_colsum<8>, g, dim3(kBlock), 0, s, a);
    else if (a.n <= 16) hipLaunchKernelGGL(k_papg_colsum<16>, g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_papg_colsum<kPapgMaxN>, g, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_papg_lin, dim3((unsigned)a.N), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_papg_step2(const PapgArgs& a, hipStream_t s) {
    const unsigned cb = (unsigned)((a.N + kBlock - 1) / kBlock);
    const unsigned rb = (unsigned)((a.N + kPapgStepRows - 1) / kPapgStepRows);
    if (a.n <= 8) hipLaunchKernelGGL(k_papg_step2<8>, dim3(cb, rb), dim3(kBlock), 0, s, a);
    else if (a.n <= 16) hipLaunchKernelGGL(k_papg_step2<16>, dim3(cb, rb), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_papg_step2<kPapgMaxN>, dim3(cb, rb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_papg_ball, dim3(1), dim3(kBlock), 0, s, a);
    const int64_t tot = a.N * a.N + a.N;
    const unsigned grid = (unsigned)std::min<int64_t>((tot + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_papg_scale, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_papg_power(const PapgArgs& a0, double* vy, double* vxi, const double* zero, int iters,
                             hipStream_t s) {
    // v0 from the hash start, normalised
    PapgArgs a = a0;
    const int64_t tot = a.N + a.N * a.n;
    hipLaunchKernelGGL(k_papg_pstart, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_papg_pnorm, dim3(1), dim3(kBlock), 0, s, a, vy, vxi, 0);
    const unsigned cb = (unsigned)((a.N + kBlock - 1) / kBlock);
    const unsigned rb = (unsigned)((a.N + kPapgStepRows - 1) / kPapgStepRows);
    // C^T through the step-1 kernels: theta2 = R (beta 0), theta2_y = y, zero data, gamma 1
    PapgArgs b = a;
    b.y = vy; b.xis = vxi;
    b.tp = b.tc; b.beta = 0.0;
    b.tyc = vy; b.typ = vy;
    b.ybar = zero; b.yshift = 0.0; b.gamma = 1.0;
    for (int it = 0; it < iters; ++it) {
        if (a.n <= 8) hipLaunchKernelGGL(k_papg_capply<8>, dim3(cb, rb), dim3(kBlock), 0, s, b);
        else if (a.n <= 16) hipLaunchKernelGGL(k_papg_capply<16>, dim3(cb, rb), dim3(kBlock), 0, s, b);
        else hipLaunchKernelGGL(k_papg_capply<kPapgMaxN>, dim3(cb, rb), dim3(kBlock), 0, s, b);
        hipError_t e = launch_papg_lin(b, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_papg_pnorm, dim3(1), dim3(kBlock), 0, s, b, vy, vxi, 1);
    }
    return hipGetLastError();
}

hipError_t launch_papg_out(const PapgArgs& a, double* y_out, double* xi_out, hipStream_t s) {
    const int64_t tot = std::max<int64_t>(a.N * a.n, a.N);
    hipLaunchKernelGGL(k_papg_out, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, y_out,
                       xi_out);
    return hipGetLastError();
}

}  // namespace cr
