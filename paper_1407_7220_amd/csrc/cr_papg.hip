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
//  k_papg_lin   data of the block problems of step 1 (eq. "g_gamma" after
//               completing the square): ybar + yshift + u and centres v/gamma,
//               u = A3^T theta2 + theta2_y, v = A4^T theta2.  One workgroup
//               per point l, reading row l and column l of theta2.
//  k_papg_step2 step 2 before the ball: theta^(1)_l = max(theta2 - C eta / L, 0)
//               written over tp, with per-row sums of theta^2, of the squared
//               negative parts of the cross residuals and of theta2 * (C eta).
//               One workgroup per row.
//  k_papg_ball  ||theta||, the scale of the projection onto the ball of Q2.
//  k_papg_scale the scale applied (only when the ball is active).
//
// The projection onto Q2 = {theta >= 0, ||theta|| <= B} is the clip at zero
// followed by a radial scale: the ball is centred at the origin and the
// orthant is a cone.
#include "cr_device.h"
#include "cr_ops.h"

namespace cr {

constexpr int kPapgMaxN = 32;

__device__ __forceinline__ double theta2_at(const PapgArgs& a, int64_t idx) {
    const double c = a.tc[idx];
    return c + a.beta * (c - a.tp[idx]);
}

__global__ __launch_bounds__(kBlock) void k_papg_lin(PapgArgs a) {
    const int64_t l = blockIdx.x;
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t bl = l / a.Nbar;
    double su = 0.0, sv[kPapgMaxN], xl[kPapgMaxN];
#pragma unroll
    for (int k = 0; k < kPapgMaxN; ++k) {
        sv[k] = 0.0;
        xl[k] = k < n ? a.X[l * n + k] : 0.0;
    }
    for (int64_t m = threadIdx.x; m < N; m += kBlock) {
        if (m / a.Nbar == bl) continue;
        const double r = theta2_at(a, l * N + m);    // pair (l, m): +y_l
        const double c = theta2_at(a, m * N + l);    // pair (m, l): -y_l and -xi_l^T (x_m - x_l)
        su += r - c;
#pragma unroll
        for (int k = 0; k < kPapgMaxN; ++k)
            if (k < n) sv[k] -= c * (a.X[m * n + k] - xl[k]);
    }
    __shared__ double red[kBlock / 64][kPapgMaxN + 1];
    su = wave_sum(su);
#pragma unroll
    for (int k = 0; k < kPapgMaxN; ++k)
        if (k < n) sv[k] = wave_sum(sv[k]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][kPapgMaxN] = su;
#pragma unroll
        for (int k = 0; k < kPapgMaxN; ++k)
            if (k < n) red[w][k] = sv[k];
    }
    __syncthreads();
    if (threadIdx.x <= n) {
        const int k = threadIdx.x == n ? kPapgMaxN : (int)threadIdx.x;
        double t = red[0][k];
        for (int q = 1; q < kBlock / 64; ++q) t += red[q][k];
        if (threadIdx.x == n) {
            const double ty = a.tyc[l] + a.beta * (a.tyc[l] - a.typ[l]);
            a.ybs[l] = (a.ybar[l] + a.yshift) + (t + ty);
        } else {
            a.shift[l * n + k] = t / a.gamma;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_papg_step2(PapgArgs a) {
    const int64_t i = blockIdx.x;
    const int64_t N = a.N;
    const int n = a.n;
    const int64_t bi = i / a.Nbar;
    double xi_[kPapgMaxN];
#pragma unroll
    for (int k = 0; k < kPapgMaxN; ++k) xi_[k] = k < n ? a.X[i * n + k] : 0.0;
    const double yi = a.y[i];
    const double L = a.L;
    double s2 = 0.0, neg2 = 0.0, gap = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kBlock) {
        const int64_t idx = i * N + j;
        double tn = 0.0;
        if (j / a.Nbar != bi) {
            // r_ij = y_i - y_j - xi_j^T (x_i - x_j), xi_j = xi'_j + c_j
            double h = 0.0;
#pragma unroll
            for (int k = 0; k < kPapgMaxN; ++k)
                if (k < n) h += (a.xis[j * n + k] + a.shift[j * n + k]) * (xi_[k] - a.X[j * n + k]);
            const double r = (yi - a.y[j]) - h;
            const double t2 = theta2_at(a, idx);
            tn = fmax(t2 - r / L, 0.0);
            if (r < 0.0) neg2 += r * r;
            gap += t2 * r;
        }
        a.tp[idx] = tn;
        s2 += tn * tn;
    }
    if (threadIdx.x == 0) {
        const double ty = a.tyc[i] + a.beta * (a.tyc[i] - a.typ[i]);
        const double tn = fmax(ty - yi / L, 0.0);
        a.typ[i] = tn;
        s2 += tn * tn;
        gap += ty * yi;
    }
    block_sum2(s2, neg2);
    gap = block_reduce(gap, 0);
    if (threadIdx.x == 0) {
        a.part[3 * i] = s2;
        a.part[3 * i + 1] = neg2;
        a.part[3 * i + 2] = gap;
    }
}

__global__ __launch_bounds__(kBlock) void k_papg_ball(PapgArgs a) {
    double s = 0.0, g = 0.0, d = 0.0;
    for (int64_t i = threadIdx.x; i < a.N; i += kBlock) {
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

hipError_t launch_papg_lin(const PapgArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_papg_lin, dim3((unsigned)a.N), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_papg_step2(const PapgArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_papg_step2, dim3((unsigned)a.N), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_papg_ball, dim3(1), dim3(kBlock), 0, s, a);
    const int64_t tot = a.N * a.N + a.N;
    const unsigned grid = (unsigned)std::min<int64_t>((tot + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_papg_scale, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_papg_out(const PapgArgs& a, double* y_out, double* xi_out, hipStream_t s) {
    const int64_t tot = std::max<int64_t>(a.N * a.n, a.N);
    hipLaunchKernelGGL(k_papg_out, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, y_out,
                       xi_out);
    return hipGetLastError();
}

}  // namespace cr
