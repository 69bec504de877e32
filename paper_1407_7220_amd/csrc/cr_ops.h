// Device helpers shared by the pair-pass kernels (cr_kernels.hip) and the
// adjoint kernels (cr_adjoint.hip): MFMA wrappers and their lane layouts,
// DPP row sums, block reductions, and the operand policies of the pass.
#pragma once
#include "cr_device.h"

namespace cr {


typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Tr;
template <> struct Tr<float> {
    static constexpr int TW = 4;   // j-tiles per wave: 16 lanes x 4 floats = 256 B per row
    typedef f32x4 acc;
};
template <> struct Tr<double> {
    static constexpr int TW = 2;   // 16 lanes x 2 doubles = 256 B per row
    typedef f64x4 acc;
};

// 16x16x4 MFMA.  Operand layout for lane l = 16 g + c (g = l / 16, c = l % 16):
//   A element (row c, k g), B element (k g, col c); accumulator element v is
//   (row rmap(g, v), col c) with rmap = 4 g + v for FP32 and g + 4 v for FP64
//   (measured on gfx950 with a one-wave layout probe).
static __device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
static __device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

template <typename T> __host__ __device__ constexpr int rmap(int g, int v) {
    return sizeof(T) == 4 ? 4 * g + v : g + 4 * v;
}

template <typename T> struct alignas(16) V16 { T v[16 / sizeof(T)]; };

// Sum over each 16-lane row of the wave with DPP moves (every lane of the row
// receives the total): pairs (quad_perm 1,0,3,2), quads (quad_perm 2,3,0,1),
// half rows (row_half_mirror), full row (row_mirror).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return v;
}

// Sum over each aligned group of P consecutive lanes (P = 1, 2, 4, 8 or 16),
// by the first log2(P) steps of row16_sum.
template <int P, typename T>
__device__ __forceinline__ T lane_group_sum(T v) {
    if constexpr (P >= 2) v += dpp_f<0xB1>(v);
    if constexpr (P >= 4) v += dpp_f<0x4E>(v);
    if constexpr (P >= 8) v += dpp_f<0x141>(v);
    if constexpr (P >= 16) v += dpp_f<0x140>(v);
    return v;
}

// Rows of a wave pairwise (gfx950 lane swaps, no LDS): with the same value in
// both operands, v_permlane16_swap returns in every lane the value of the even
// row and of the odd row of its row pair (SW = 16), v_permlane32_swap those of
// the lower and upper half (SW = 32); ev and od are the same in both lanes of a
// pair, so an operation on them gives bit-identical results there.
template <int SW>
__device__ __forceinline__ void row_pair(double v, double& ev, double& od) {
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = (int)(u & 0xffffffffLL), hi = (int)(u >> 32);
    if constexpr (SW == 16) {
        const auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        ev = __builtin_bit_cast(double, ((long long)H[0] << 32) | (unsigned int)L[0]);
        od = __builtin_bit_cast(double, ((long long)H[1] << 32) | (unsigned int)L[1]);
    } else {
        const auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        ev = __builtin_bit_cast(double, ((long long)H[0] << 32) | (unsigned int)L[0]);
        od = __builtin_bit_cast(double, ((long long)H[1] << 32) | (unsigned int)L[1]);
    }
}

// Sum over each aligned group of G = 16, 32 or 64 lanes (every lane of the
// group receives it): DPP within a row, lane swaps across rows.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    v = row16_sum(v);
    double e, o;
    if constexpr (G >= 32) { row_pair<16>(v, e, o); v = e + o; }
    if constexpr (G >= 64) { row_pair<32>(v, e, o); v = e + o; }
    return v;
}

// Sums over each 16-lane row of the wave of four values at once, by exchange:
// at each step a lane keeps half of its values and adds its partner's
// copies of them (partners 15 - c, then the mirror within 8 lanes, then the
// quad pairs), so after four steps lane c of the row holds the total of value
// s[c >> 2] (lanes 0, 4, 8, 12 hold values 0, 1, 2, 3).  27 instructions in
// FP64 and 11 in FP32 instead of 48 and 16 for four separate sums.
template <typename T>
__device__ __forceinline__ T row16_sum4(const T s[4], int c) {
    const bool hi8 = c >= 8, hi4 = (c & 4) != 0;
    T k0 = hi8 ? s[2] : s[0], k1 = hi8 ? s[3] : s[1];
    const T p0 = hi8 ? s[0] : s[2], p1 = hi8 ? s[1] : s[3];
    k0 += dpp_f<0x140>(p0);
    k1 += dpp_f<0x140>(p1);
    T k = hi4 ? k1 : k0;
    const T p = hi4 ? k0 : k1;
    k += dpp_f<0x141>(p);
    k += dpp_f<0xB1>(k);
    k += dpp_f<0x4E>(k);
    return k;
}

// Global-memory view of a pointer.  Pointers read from device memory (the
// batched kernels' argument tables) are otherwise generic, accessed with flat
// instructions whose completion the compiler cannot order against other
// loads (so every wait on one drains all of them).
template <typename T> using gp = T __attribute__((address_space(1)))*;
template <typename T> __device__ __forceinline__ gp<T> glob(T* p) { return (gp<T>)p; }

template <typename T>
__device__ __forceinline__ V16<T> ld16(const T* p) { return *reinterpret_cast<const V16<T>*>(p); }
template <typename T>
__device__ __forceinline__ void st16(T* p, const V16<T>& x) { *reinterpret_cast<V16<T>*>(p) = x; }

// Buffer views (gfx9 raw buffer resources, third descriptor word 0x00020000):
// a load at byte offset voffset + soffset at or past `bytes` returns zeros and
// touches no memory, so a prefetch that runs past a workgroup's rows needs no
// clamp; the per-tile step goes into the scalar soffset.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ V16<T> bld16(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(V16<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double bld8(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// A value that is the same for every lane, read with a vector load (vld_*)
// and made uniform at its first use (uniform()): vector loads complete in issue
// order, so waiting for this one does not drain the loads issued after it (a
// scalar load's wait would take every outstanding scalar load with it, the
// kernel arguments of those later loads among them).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
// With ok false the view is empty: the load reads 0 and touches no memory (p
// may then be anything), so the load needs no branch around it.
__device__ __forceinline__ int vld_i32(const int32_t* p, bool ok = true) {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(make_rsrc(p, ok ? 4u : 0u), 0, 0, 0);
}
__device__ __forceinline__ u32x2 vld_i64(const int64_t* p, bool ok = true) {
    return __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(make_rsrc(p, ok ? 8u : 0u), 0, 0, 0));
}
__device__ __forceinline__ int32_t uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform(u32x2 v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.y);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T bld_t(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bld_t<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bld_t<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return bld8(r, voff, soff);
}

// ---------------------------------------------------------------------------
// Block reductions (256 threads) and the last-arriving-block handshake.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }
static __device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f<0xB1>(v));
    v = fmax(v, dpp_f<0x4E>(v));
    v = fmax(v, dpp_f<0x141>(v));
    v = fmax(v, dpp_f<0x140>(v));
    double e, o;
    row_pair<16>(v, e, o);
    v = fmax(e, o);
    row_pair<32>(v, e, o);
    return fmax(e, o);
}

// Sum (op 0) or max (op 1) of one double per thread; result valid in every thread.
static __device__ double block_reduce(double v, int op) {
    __shared__ double red[kBlock / 64];
    v = op == 0 ? wave_sum(v) : wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < kBlock / 64; ++w) r = op == 0 ? r + red[w] : fmax(r, red[w]);
    return r;
}

// Sums of two doubles per thread over the block, one barrier pair for both;
// results valid in every thread.
static __device__ void block_sum2(double& a, double& b) {
    __shared__ double red2[kBlock / 64][2];
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red2[threadIdx.x >> 6][0] = a; red2[threadIdx.x >> 6][1] = b; }
    __syncthreads();
    a = red2[0][0];
    b = red2[0][1];
    for (int w = 1; w < kBlock / 64; ++w) { a += red2[w][0]; b += red2[w][1]; }
}

// Sums of fields q0 and q1 of the first `count` 4-double records that an
// earlier kernel wrote (plain loads: the kernel boundary orders them), by all
// threads of the block in a fixed order.
static __device__ void gather_sum2(const double* part, int count, int q0, int q1, double& s0, double& s1) {
    s0 = 0.0;
    s1 = 0.0;
    // four records per thread in flight, summed in index order
    for (int b = threadIdx.x; b < count; b += 4 * kBlock) {
        double u0[4], u1[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // clamped address and a select (no branch, so the loads stay in flight together)
            const int r = b + e * kBlock;
            const int64_t rc = min(r, count - 1);
            const double x0 = part[rc * 4 + q0], x1 = part[rc * 4 + q1];
            u0[e] = r < count ? x0 : 0.0;
            u1[e] = r < count ? x1 : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) { s0 += u0[e]; s1 += u1[e]; }
    }
    block_sum2(s0, s1);
}

// Workgroup b of a launch runs on XCD b mod 8 (round-robin dispatch, each
// XCD with its own L2).  xcd_remap maps b to a logical index such that every
// XCD takes one contiguous range of logical indices, so workgroups that share
// cache lines (neighbouring points of the partial-sum arrays) share an L2.
// A bijection on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int X = 8;
    const int q = (n + X - 1) / X, tall = n % X == 0 ? X : n % X;
    const int x = b % X, i = b / X;
    return x < tall ? x * q + i : tall * q + (x - tall) * (q - 1) + i;
}

// gather_sum2 in two steps, with the same sums in the same order: the loads of
// the first NB x 4 kBlock records (issue), then the rest and the block sum
// (finish).  Records past `count` read as 0.0, which leaves the sums unchanged.
template <int NB>
static __device__ __forceinline__ void gather_issue(const double* part_, int count, int q0, int q1,
                                                    double u0[4 * NB], double u1[4 * NB]) {
    const gp<const double> part = glob(part_);
#pragma unroll
    for (int e = 0; e < 4 * NB; ++e) {
        const int r = threadIdx.x + e * kBlock;
        const int64_t rc = max(min(r, count - 1), 0);
        const double x0 = part[rc * 4 + q0], x1 = part[rc * 4 + q1];
        u0[e] = r < count ? x0 : 0.0;
        u1[e] = r < count ? x1 : 0.0;
    }
}
template <int NB>
static __device__ void gather_finish(const double* part_, int count, int q0, int q1, const double u0[4 * NB],
                                     const double u1[4 * NB], double& s0, double& s1) {
    const gp<const double> part = glob(part_);
    s0 = 0.0;
    s1 = 0.0;
#pragma unroll
    for (int e = 0; e < 4 * NB; ++e) { s0 += u0[e]; s1 += u1[e]; }
    for (int b = threadIdx.x + 4 * NB * kBlock; b < count; b += 4 * kBlock) {
        double w0[4], w1[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = b + e * kBlock;
            const int64_t rc = min(r, count - 1);
            const double x0 = part[rc * 4 + q0], x1 = part[rc * 4 + q1];
            w0[e] = r < count ? x0 : 0.0;
            w1[e] = r < count ? x1 : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) { s0 += w0[e]; s1 += w1[e]; }
    }
    block_sum2(s0, s1);
}

// Each of `total` blocks calls this once after writing its partial results; it
// returns true in every thread of the one block that arrives last (that block
// then sees every other block's partials) and re-arms the counter.
static __device__ bool last_block(unsigned int* counter, unsigned int total) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int prev = atomicAdd(counter, 1u);
        is_last = (prev == total - 1) ? 1 : 0;
        if (is_last) atomicExch(counter, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

static __device__ __forceinline__ double ld_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Operand policies of the pair pass.  A policy says what one lane holds for
// the two contractions and how they run:
//   R = [X 1] [-Xi c]^T + y 1^T      (residuals, one 16 x 16 tile per j-tile)
//   C += W^T [X 1]                   (sum_i w_ij x_i and colsum_j)
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

static __device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// FP64 / FP32: 16x16x4 MFMA in the pass precision; c_j and y_i enter R exactly.
// Row stride (elements) of the column operands a lazy pass stages in LDS.
constexpr int kBsStride = 33;

template <typename T, int KS, int NSET_ = 0> struct PlainOps {
    typedef T elem;
    typedef typename Tr<T>::acc acc_t;
    static constexpr int TW = Tr<T>::TW;
    static constexpr int NKB = nkb_of_ks(KS);
    static constexpr int QP = qp_of_ks(KS, (int)sizeof(T));
    static constexpr int EV = 16 / (int)sizeof(T);
    // two staging sets: with them the FP32 pass fits 4 waves per SIMD, which hides
    // the per-tile chain better than a third set at 3 waves (measured)
    static constexpr int NSET = NSET_ > 0 ? NSET_ : 2;
    static constexpr int RM4 = sizeof(T) == 4;   // accumulator row map 4 g + v (else g + 4 v)
    struct Breg { T b[KS][TW]; };
    struct Xop { T q[QP]; };
    // B operand of R for every j-tile: [-xi_j, c_j, 0...] (k = 4 s + g)
    static __device__ void load_breg(Breg& B, const PassArgs& a, int64_t jl, int g) {
        const gp<const T> xiaug = glob((const T*)a.xiaug);
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const gp<const T> row = xiaug + (jl + t) * (4 * KS);
#pragma unroll
            for (int s = 0; s < KS; ++s) B.b[s][t] = row[4 * s + g];
        }
    }
    // slots of one column's operand row: [-xi_j (n), c_j, 0 ...]
    static constexpr int KCAP = 4 * KS;
    // the same from a staged LDS copy (column c0 + t at row c0 + t, stride kBsStride)
    static __device__ void load_breg_lds(Breg& B, const T* Bs, int c0, int g, int) {
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int s = 0; s < KS; ++s) B.b[s][t] = Bs[(c0 + t) * kBsStride + 4 * s + g];
    }
    static __device__ void load_xop(Xop& X, const PassArgs& a, int64_t i0, int lane) {
        const T* xp = (const T*)a.xp;
#pragma unroll
        for (int q = 0; q < QP / EV; ++q) {
            V16<T> tv = ld16(xp + ((i0 >> 4) * 64 + lane) * QP + q * EV);
#pragma unroll
            for (int e = 0; e < EV; ++e) X.q[q * EV + e] = tv.v[e];
        }
    }
    // bytes of one (16-row tile, lane) entry of the packed operands
    static constexpr int XPB = QP * (int)sizeof(T);
    static __device__ void load_xop_b(Xop& X, rsrc_t r, uint32_t voff, uint32_t soff) {
#pragma unroll
        for (int q = 0; q < QP / EV; ++q) {
            V16<T> tv = bld16<T>(r, voff + 16 * q, soff);
#pragma unroll
            for (int e = 0; e < EV; ++e) X.q[q * EV + e] = tv.v[e];
        }
    }
    static __device__ void residual(acc_t R[TW], const Xop& X, const Breg& B, const T yv[4]) {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            R[t] = acc_t{yv[0], yv[1], yv[2], yv[3]};
#pragma unroll
            for (int s = 0; s < KS; ++s) R[t] = mfma4(X.q[s], B.b[s][t], R[t]);
        }
    }
    // i-slot g of step s is row i0 + rmap(g, s): W comes straight from R's registers
    static __device__ void colsums(acc_t C[TW][NKB], const T W[TW][4], const Xop& X) {
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int s = 0; s < 4; ++s) C[t][kb] = mfma4(W[t][s], X.q[KS + 4 * kb + s], C[t][kb]);
    }
};

// Mixed: BF16 16x16x32 MFMA on hi/lo splits with FP32 accumulation; theta,
// W and the accumulators are FP32.  R: K-slots [x_hi | x_lo | x_hi] against
// [-xi_hi | -xi_hi | -xi_lo] (K = 3n, KB blocks of 32), accumulator started
// at y_i + c_j in FP32.  C: [W_hi, W_hi] . [X_hi, X_lo] plus
// [W_lo, W_lo] . [X_hi, X_lo] over the lane's 4 rows (all four products of
// the splits), so one 16-byte X operand per column block serves both.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <int KB, int NKB_> struct MixedOps {
    typedef float elem;
    typedef f32x4 acc_t;
    static constexpr int TW = 4;
    static constexpr int NKB = NKB_;
    static constexpr int NSET = KB + NKB <= 2 ? 3 : 2;
    static constexpr int RM4 = 1;
    struct Breg { bf16x8 b[KB][TW]; float cc[TW]; };
    struct Xop { bf16x8 r[KB]; bf16x8 cx[NKB]; };
    static __device__ void load_breg(Breg& B, const PassArgs& a, int64_t jl, int g) {
        const __bf16* xb = (const __bf16*)a.xiaug;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                B.b[kb][t] = *glob(reinterpret_cast<const bf16x8*>(xb + ((jl + t) * KB + kb) * 32 + 8 * g));
            B.cc[t] = glob(a.cvec)[jl + t];
        }
    }
    // -xi_j entries of one column (3n <= 32 KB)
    static constexpr int KCAP = (32 * KB) / 3 + 1 < 32 ? (32 * KB) / 3 + 1 : 32;
    // from a staged LDS copy of [-xi_j (n), c_j] in FP32: the hi/lo slots as k_set_point lays them out
    static __device__ void load_breg_lds(Breg& B, const float* Bs, int c0, int g, int n) {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const float* row = Bs + (c0 + t) * kBsStride;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                bf16x8 v;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = 32 * kb + 8 * g + e;
                    __bf16 val = (__bf16)0.0f;
                    if (q < 3 * n) {
                        const float x = row[q % n];
                        const __bf16 hi = (__bf16)x;
                        val = q < 2 * n ? hi : (__bf16)(x - (float)hi);
                    }
                    v[e] = val;
                }
                B.b[kb][t] = v;
            }
            B.cc[t] = row[n];
        }
    }
    static __device__ void load_xop(Xop& X, const PassArgs& a, int64_t i0, int lane) {
        const bf16x8* xp = (const bf16x8*)a.xp + ((i0 >> 4) * 64 + lane) * (KB + NKB);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) X.r[kb] = xp[kb];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) X.cx[kb] = xp[KB + kb];
    }
    static constexpr int XPB = (KB + NKB) * 16;
    static __device__ void load_xop_b(Xop& X, rsrc_t r, uint32_t voff, uint32_t soff) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) X.r[kb] = __builtin_bit_cast(bf16x8, bld16<float>(r, voff + 16 * kb, soff));
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
            X.cx[kb] = __builtin_bit_cast(bf16x8, bld16<float>(r, voff + 16 * (KB + kb), soff));
    }
    static __device__ void residual(acc_t R[TW], const Xop& X, const Breg& B, const float yv[4]) {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            R[t] = acc_t{yv[0] + B.cc[t], yv[1] + B.cc[t], yv[2] + B.cc[t], yv[3] + B.cc[t]};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) R[t] = mfma_bf16(X.r[kb], B.b[kb][t], R[t]);
        }
    }
    // Split of four FP32 values into packed BF16 pairs: hi = RNE(w), lo =
    // RNE(w - hi) (w - hi is exact in FP32; hi read back from its bits).
    static __device__ __forceinline__ void split4(const float w[4], unsigned int h[2], unsigned int l[2]) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const bf16x2 hb = {(__bf16)w[2 * p], (__bf16)w[2 * p + 1]};
            const unsigned int u = __builtin_bit_cast(unsigned int, hb);
            const float h0 = __builtin_bit_cast(float, u << 16), h1 = __builtin_bit_cast(float, u & 0xffff0000u);
            const bf16x2 lb = {(__bf16)(w[2 * p] - h0), (__bf16)(w[2 * p + 1] - h1)};
            h[p] = u;
            l[p] = __builtin_bit_cast(unsigned int, lb);
        }
    }
    static __device__ void colsums(acc_t C[TW][NKB], const float W[TW][4], const Xop& X) {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            unsigned int h[2], l[2];
            split4(W[t], h, l);
            const bf16x8 wh = __builtin_bit_cast(bf16x8, u32x4{h[0], h[1], h[0], h[1]});
            const bf16x8 wl = __builtin_bit_cast(bf16x8, u32x4{l[0], l[1], l[0], l[1]});
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                C[t][kb] = mfma_bf16(wh, X.cx[kb], C[t][kb]);
                C[t][kb] = mfma_bf16(wl, X.cx[kb], C[t][kb]);
            }
        }
    }
};

template <typename Ops> __device__ __forceinline__ int orow(int g, int v) {
    return Ops::RM4 ? 4 * g + v : g + 4 * v;
}

}  // namespace cr
