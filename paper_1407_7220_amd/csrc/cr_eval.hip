// Evaluation of the fitted estimator at new points (gfx950).
//
// The least-squares estimator of Sec. I (Aybat & Wang) is the piecewise-linear
// convex function with value y_l at x_l and subgradient xi_l there; at a query
// point q it is the largest supporting hyperplane,
//   f(q) = max_l ( y_l + xi_l^T (q - x_l) ) = max_l ( [q 1] . [xi_l  d_l] ),
//   d_l = y_l - x_l^T xi_l,
// and the maximising l names a subgradient xi_l of f at q.  For M queries and N
// planes the values form the M x N product [Q 1] [Xi d]^T, a dense contraction
// with K = n + 1: FP64 MFMA (16x16x4) tiles, with a running maximum and argmax
// per query instead of a stored product.
//
// Launch: one workgroup per 32 queries (two 16-row blocks); its 8 waves take
// interleaved 32-plane tiles (two 16-column MFMA tiles) of all N planes, each
// wave keeping (max, argmax) per query, and the 8 waves' results are combined
// in LDS.  Ties go to the smaller plane index, so the result does not depend
// on the traversal order.
#include "cr_device.h"
#include "cr_ops.h"
#include "../../include/cr.h"

#include <cmath>
#include <mutex>
#include <string>

namespace cr {

constexpr int kEvalRows = 32;     // queries per workgroup
constexpr int kEvalCols = 32;     // planes per wave step
constexpr int kEvalWaves = 8;     // waves per workgroup (interleaved plane tiles)

// Packed plane operands: row l holds [xi_l (n), d_l, 0 ...] (4 KS doubles).
// Padding rows l >= N hold d = -Inf and zeros: their value -Inf at every valid
// query never exceeds a running maximum, so the loop needs no index mask.
__global__ __launch_bounds__(kBlock) void k_eval_prep(const double* __restrict__ X, const double* __restrict__ y,
                                                      const double* __restrict__ xi, int64_t N, int n, int kp,
                                                      int64_t Npad, double* __restrict__ B) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= Npad * kp) return;
    const int64_t l = e / kp;
    const int k = (int)(e % kp);
    double v = 0.0;
    if (l < N) {
        if (k < n) {
            v = xi[l * n + k];
        } else if (k == n) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += X[l * n + q] * xi[l * n + q];
            v = y[l] - s;
        }
    } else if (k == n) {
        v = -INFINITY;
    }
    B[e] = v;
}

struct EvalArgs {
    int64_t N, M;
    int32_t n, kp;
    int64_t ntiles;           // 32-plane tiles
    const double* Q;          // M x n
    const double* B;          // packed planes, ntiles * 32 rows of kp
    double* f;                // M
    int64_t* arg;             // M or null
};

__device__ __forceinline__ void better(double& bv, int32_t& bl, double v, int32_t l) {
    if (v > bv || (v == bv && l < bl)) { bv = v; bl = l; }
}

template <int KS>
__global__ __launch_bounds__(64 * kEvalWaves) void k_eval(EvalArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t m0 = (int64_t)blockIdx.x * kEvalRows;
    const int n = a.n, kp = a.kp;

    // A operands of the two query blocks: lane (g, c) holds [q_m 1][4 s + g], m = block + c
    double A[2][KS];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        const int64_t m = m0 + 16 * rb + c;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + g;
            double v = 0.0;
            if (m < a.M) v = k < n ? a.Q[m * n + k] : (k == n ? 1.0 : 0.0);
            A[rb][s] = v;
        }
    }

    // Running (max, argmax) of this lane's 4 accumulator rows (g + 4 v) per
    // block; plane indices fit 32 bits (N < 2^31 is checked by the host).
    double bv[2][4];
    int32_t bl[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) { bv[rb][v] = -INFINITY; bl[rb][v] = INT32_MAX; }

    // B operands of one 32-plane tile: lane (g, c) holds plane (tile + 16 h + c), slot 4 s + g
    auto load_b = [&](int64_t t, double (&b)[2][KS]) {
        const int64_t tt = t < a.ntiles ? t : a.ntiles - 1;     // past the end: any valid tile, masked below
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* row = a.B + (tt * kEvalCols + 16 * h + c) * kp + g;
#pragma unroll
            for (int s = 0; s < KS; ++s) b[h][s] = row[4 * s];
        }
    };
    double bcur[2][KS], bnext[2][KS];
    int64_t t = wave;
    load_b(t, bcur);
    for (; t < a.ntiles; t += kEvalWaves) {
        load_b(t + kEvalWaves, bnext);                              // next tile in flight during this one
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t l = (int32_t)t * kEvalCols + 16 * h + c;   // this lane's plane
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KS; ++s) acc = mfma4(A[rb][s], bcur[h][s], acc);
                // l increases along a lane: a strict test keeps the first of equal
                // values; fmax keeps the running value when acc is NaN
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    bl[rb][v] = acc[v] > bv[rb][v] ? l : bl[rb][v];
                    bv[rb][v] = fmax(bv[rb][v], acc[v]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < KS; ++s) bcur[h][s] = bnext[h][s];
    }

    // Combine over the 16 lanes of each row group (different planes), then over the waves.
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const double ov = __shfl_xor(bv[rb][v], o);
                const int32_t ol = __shfl_xor(bl[rb][v], o);
                better(bv[rb][v], bl[rb][v], ov, ol);
            }
    __shared__ double sv[kEvalWaves][kEvalRows];
    __shared__ int32_t sl[kEvalWaves][kEvalRows];
    if (c == 0) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * rb + g + 4 * v;              // FP64 accumulator row map
                sv[wave][r] = bv[rb][v];
                sl[wave][r] = bl[rb][v];
            }
    }
    __syncthreads();
    if (threadIdx.x < kEvalRows) {
        const int r = threadIdx.x;
        double best = sv[0][r];
        int32_t bi = sl[0][r];
        for (int w = 1; w < kEvalWaves; ++w) better(best, bi, sv[w][r], sl[w][r]);
        const int64_t m = m0 + r;
        if (m < a.M) {
            a.f[m] = best;
            if (a.arg) a.arg[m] = bi == INT32_MAX ? INT64_MAX : (int64_t)bi;
        }
    }
}

static int eval_ks(int n) { return (n + 1 + 3) / 4; }
static int64_t eval_tiles(int64_t N) { return (N + kEvalCols - 1) / kEvalCols; }

static hipError_t launch_eval(const EvalArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.M + kEvalRows - 1) / kEvalRows));
    switch (eval_ks(a.n)) {
        case 1: hipLaunchKernelGGL(k_eval<1>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_eval<2>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_eval<3>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_eval<4>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 5: hipLaunchKernelGGL(k_eval<5>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 6: hipLaunchKernelGGL(k_eval<6>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 7: hipLaunchKernelGGL(k_eval<7>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_eval<8>, grid, dim3(64 * kEvalWaves), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cr

// Static scratch of cr_eval_noalloc: the packed planes live in a file-scope
// device array (one copy per GPU, held until the process ends) instead of a
// workspace, for callers that cannot allocate.  32 MiB hold N * 4 ceil((n+1)/4)
// doubles, e.g. 174752 planes at n = 20 or 1048576 at n = 3.
constexpr size_t kEvalScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double eval_scratch_mem[kEvalScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

size_t eval_ws_bytes(int64_t N, int n) {
    return (size_t)(cr::eval_tiles(N) * cr::kEvalCols) * (size_t)(4 * cr::eval_ks(n)) * 8 + 256;
}

cr_status eval_fail(cr_status s, const std::string& msg) {
    cr::set_last_error(msg);
    return s;
}

// Host-side argument checks shared by both entry points (before any HIP call).
cr_status eval_check(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n,
                     const void* Q_dev, int64_t M, const void* fhat_dev) {
    if (N < 1 || n < 1 || M < 0) return eval_fail(CR_ERR_ARG, "N and n must be >= 1 and M >= 0");
    if (N >= ((int64_t)1 << 31) - 64) return eval_fail(CR_ERR_UNSUPPORTED, "N must be below 2^31 - 64");
    if (n > CR_MAX_DIM) return eval_fail(CR_ERR_UNSUPPORTED, "n above CR_MAX_DIM is not supported");
    if (!X_dev || !y_dev || !xi_dev || (M > 0 && (!Q_dev || !fhat_dev)))
        return eval_fail(CR_ERR_ARG, "X, y, xi, Q and fhat must be non-NULL");
    return CR_OK;
}

// Packing kernel and evaluation kernel on the packed-plane buffer B (256-byte aligned).
cr_status eval_launch(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n,
                      const void* Q_dev, int64_t M, void* fhat_dev, int64_t* arg_dev, double* B, hipStream_t s) {
    const int kp = 4 * cr::eval_ks(n);
    const int64_t ntiles = cr::eval_tiles(N);
    const int64_t Npad = ntiles * cr::kEvalCols;
    const int64_t elems = Npad * kp;
    hipLaunchKernelGGL(cr::k_eval_prep, dim3((unsigned)((elems + cr::kBlock - 1) / cr::kBlock)), dim3(cr::kBlock), 0, s,
                       (const double*)X_dev, (const double*)y_dev, (const double*)xi_dev, N, (int)n, kp, Npad, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return eval_fail(CR_ERR_HIP, std::string("eval prep: ") + hipGetErrorString(e));
    cr::EvalArgs a{};
    a.N = N; a.M = M; a.n = n; a.kp = kp; a.ntiles = ntiles;
    a.Q = (const double*)Q_dev; a.B = B; a.f = (double*)fhat_dev; a.arg = arg_dev;
    e = cr::launch_eval(a, s);
    if (e != hipSuccess) return eval_fail(CR_ERR_HIP, std::string("eval: ") + hipGetErrorString(e));
    return CR_OK;
}

// Device address of this GPU's copy of eval_scratch_mem, looked up once per device
// (with that device current) and kept; never the host-side name of the array.
cr_status eval_scratch(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return eval_fail(CR_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return eval_fail(CR_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(eval_scratch_mem));
        if (e != hipSuccess || !ptr)
            return eval_fail(CR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return CR_OK;
}

}  // namespace

extern "C" {

cr_status cr_eval_workspace_bytes(int64_t N, int32_t n, size_t* bytes) {
    if (!bytes) return eval_fail(CR_ERR_ARG, "bytes is NULL");
    if (N < 1 || n < 1) return eval_fail(CR_ERR_ARG, "N and n must be >= 1");
    if (n > CR_MAX_DIM) return eval_fail(CR_ERR_UNSUPPORTED, "n above CR_MAX_DIM is not supported");
    if (N >= ((int64_t)1 << 31) - 64) return eval_fail(CR_ERR_UNSUPPORTED, "N must be below 2^31 - 64");
    *bytes = eval_ws_bytes(N, n);
    return CR_OK;
}

cr_status cr_eval(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n, const void* Q_dev,
                  int64_t M, void* fhat_dev, int64_t* arg_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
    cr_status st = eval_check(X_dev, y_dev, xi_dev, N, n, Q_dev, M, fhat_dev);
    if (st != CR_OK) return st;
    if (!workspace_dev) return eval_fail(CR_ERR_ARG, "the workspace must be non-NULL");
    if (ws_bytes < eval_ws_bytes(N, n)) return eval_fail(CR_ERR_NOMEM, "workspace smaller than cr_eval_workspace_bytes()");
    if (M == 0) return CR_OK;
    double* B = reinterpret_cast<double*>(((uintptr_t)workspace_dev + 255) & ~(uintptr_t)255);
    return eval_launch(X_dev, y_dev, xi_dev, N, n, Q_dev, M, fhat_dev, arg_dev, B, (hipStream_t)stream);
}

cr_status cr_eval_noalloc(const void* X_dev, const void* y_dev, const void* xi_dev, int64_t N, int32_t n,
                          const void* Q_dev, int64_t M, void* fhat_dev, int64_t* arg_dev, void* stream) {
    cr_status st = eval_check(X_dev, y_dev, xi_dev, N, n, Q_dev, M, fhat_dev);
    if (st != CR_OK) return st;
    if (eval_ws_bytes(N, n) - 256 > kEvalScratchBytes)
        return eval_fail(CR_ERR_NOMEM, "the packed planes (" + std::to_string(eval_ws_bytes(N, n) - 256) +
                                           " bytes) exceed the static scratch of cr_eval_noalloc (" +
                                           std::to_string(kEvalScratchBytes) + " bytes)");
    if (M == 0) return CR_OK;
    double* B = nullptr;
    st = eval_scratch(&B);
    if (st != CR_OK) return st;
    return eval_launch(X_dev, y_dev, xi_dev, N, n, Q_dev, M, fhat_dev, arg_dev, B, (hipStream_t)stream);
}

}  // extern "C"
