// MFMA block-GEMM cores for gfx950: acc(BM x BN) += A(BM x K) * B(BN x K)^T.
//
// Two operand layouts:
//   * "cm" (FP64, FP32): A(r, k) = A[r + k*lda]  (a column-major tile: rows
//     contiguous for each k), MFMA 16x16x4 (one element per lane);
//   * "rm" (FP16, BF16, FP8): A(r, k) = A[r*lda + k]  (k contiguous), MFMA
//     16x16x32 for FP16/BF16 (eight elements per lane) and 16x16x128 for FP8
//     (32 elements per lane), FP32 accumulation.
// WM x WN waves per block; each wave owns (BM/WM) x (BN/WN) of the block as
// 16 x 16 MFMA tiles.  Operands are staged through double-buffered LDS, the
// next K slice is fetched into registers while the current one is multiplied.
//
// MFMA lane layout used (lane l = 0..63, g = l / 16, i = l % 16):
//   16x16x4 :  a = A[i][g],          b = B[g][i]
//   16x16x32:  a[j] = A[i][8g + j],  b[j] = B[8g + j][i]   (j = 0..7)
//   16x16x128 (8-bit): 32 K elements of row i / column i per lane, the same
//              K assignment for a and b
//   result  :  d[v] = D[4g + v][i]   (v = 0..3) for the FP32-accumulating forms,
//              d[v] = D[g + 4v][i]   for 16x16x4 FP64 (64-bit accumulator registers)
#pragma once
#include "common.h"

namespace mpc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Row (within a 16 x 16 MFMA tile) of accumulator element v of a lane in lane group g.
template <typename T> __device__ inline int acc_row(int g, int v) { return sizeof(T) == 8 ? g + 4 * v : 4 * g + v; }
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- cm (FP64 / FP32)
template <typename T> struct CM;
template <> struct CM<double> {
    typedef double4_t acc_t;
    static constexpr int PAD = 16;
    __device__ static inline acc_t mfma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct CM<float> {
    typedef float4_t acc_t;
    static constexpr int PAD = 16;
    __device__ static inline acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// WM x WN waves (64 * WM * WN threads); each wave owns (BM/WM) x (BN/WN) of
// the block as MB x NB MFMA tiles of 16 x 16.
template <typename T, int BM, int BN, int BK, int WM = 2, int WN = 2>
struct CMShape {
    static constexpr int NTH = 64 * WM * WN;
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int LDM = BM + CM<T>::PAD, LDN = BN + CM<T>::PAD;
    static constexpr int CHA = BK * BM / VEC, CHB = BK * BN / VEC;  // 16-byte chunks of A and B
    static constexpr int CA = (CHA + NTH - 1) / NTH, CB = (CHB + NTH - 1) / NTH;  // per thread
    static constexpr int MB = BM / WM / 16, NB = BN / WN / 16;
    static constexpr size_t SMEM = sizeof(T) * (size_t)2 * BK * (LDM + LDN);
    static_assert((CHA % NTH == 0 || CHA < NTH) && (CHB % NTH == 0 || CHB < NTH), "load split");
    static_assert(BK % 4 == 0 && MB >= 1 && NB >= 1, "shape");
};

// acc += A * B^T over K (K a multiple of BK); with A2/B2 given, the product
// continues over a second K range, acc += A2 * B2^T (same leading dimensions),
// in the same pipelined loop.  With SWAP the MFMA operands are
// exchanged, so each 16 x 16 accumulator holds the transposed tile: lane i
// owns row i of the block's sub-tile and element v its column acc_row(g, v)
// (rows contiguous in memory, so column-major stores coalesce).
// PRIO raises the wave's issue priority while it multiplies, so that a wave
// with operands ready in LDS is not held back by waves still loading.
template <typename T, int BM, int BN, int BK, int WM = 2, int WN = 2, bool SWAP = false, bool PRIO = false>
__device__ inline void cm_block(const T *__restrict__ A, int64_t lda, const T *__restrict__ B, int64_t ldb, int K,
                                typename CM<T>::acc_t (&acc)[CMShape<T, BM, BN, BK, WM, WN>::MB]
                                                              [CMShape<T, BM, BN, BK, WM, WN>::NB],
                                T *smem, const T *__restrict__ A2 = nullptr, const T *__restrict__ B2 = nullptr)
{
    typedef CMShape<T, BM, BN, BK, WM, WN> S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int gi = lane & 15, gg = lane >> 4;
    T *As = smem;                       // [2][BK][LDM]
    T *Bs = smem + 2 * BK * S::LDM;     // [2][BK][LDN]
    u32x4 ra[S::CA], rb[S::CB];
    const int nk1 = K / BK, nk = A2 ? 2 * nk1 : nk1;

    auto gload = [&](int kt) {
        const T *a = A, *bp = B;
        if (kt >= nk1) {
            a = A2;
            bp = B2;
            kt -= nk1;
        }
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BM / S::VEC), r = (ch % (BM / S::VEC)) * S::VEC;
            if (ch < S::CHA) ra[c] = *(const u32x4 *)(a + r + (int64_t)(kt * BK + col) * lda);
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BN / S::VEC), r = (ch % (BN / S::VEC)) * S::VEC;
            if (ch < S::CHB) rb[c] = *(const u32x4 *)(bp + r + (int64_t)(kt * BK + col) * ldb);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BM / S::VEC), r = (ch % (BM / S::VEC)) * S::VEC;
            if (ch < S::CHA) *(u32x4 *)(As + (buf * BK + col) * S::LDM + r) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BN / S::VEC), r = (ch % (BN / S::VEC)) * S::VEC;
            if (ch < S::CHB) *(u32x4 *)(Bs + (buf * BK + col) * S::LDN + r) = rb[c];
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        const T *as = As + cur * BK * S::LDM + wm * (BM / WM) + gi;
        const T *bs = Bs + cur * BK * S::LDN + wn * (BN / WN) + gi;
        if (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            T fa[S::MB], fb[S::NB];
#pragma unroll
            for (int m = 0; m < S::MB; ++m) fa[m] = as[(s * 4 + gg) * S::LDM + m * 16];
#pragma unroll
            for (int n = 0; n < S::NB; ++n) fb[n] = bs[(s * 4 + gg) * S::LDN + n * 16];
#pragma unroll
            for (int m = 0; m < S::MB; ++m)
#pragma unroll
                for (int n = 0; n < S::NB; ++n)
                    acc[m][n] = SWAP ? CM<T>::mfma(fb[n], fa[m], acc[m][n]) : CM<T>::mfma(fa[m], fb[n], acc[m][n]);
        }
        if (PRIO) __builtin_amdgcn_s_setprio(0);
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
}

// cm_block with the global loads issued two K slices ahead (two register
// sets, slice kt + 2 in flight while slice kt is multiplied and slice kt + 1
// waits in registers), the same LDS stages and the same products in the same
// order, so the results are bit-identical.  The number of slices (K / BK, or
// twice that with A2/B2) must be even.
template <typename T, int BM, int BN, int BK, int WM = 2, int WN = 2, bool SWAP = false>
__device__ inline void cm_block_deep(const T *__restrict__ A, int64_t lda, const T *__restrict__ B, int64_t ldb, int K,
                                     typename CM<T>::acc_t (&acc)[CMShape<T, BM, BN, BK, WM, WN>::MB]
                                                                   [CMShape<T, BM, BN, BK, WM, WN>::NB],
                                     T *smem, const T *__restrict__ A2 = nullptr, const T *__restrict__ B2 = nullptr)
{
    typedef CMShape<T, BM, BN, BK, WM, WN> S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int gi = lane & 15, gg = lane >> 4;
    T *As = smem;                       // [2][BK][LDM]
    T *Bs = smem + 2 * BK * S::LDM;     // [2][BK][LDN]
    u32x4 ra0[S::CA], rb0[S::CB], ra1[S::CA], rb1[S::CB];
    const int nk1 = K / BK, nk = A2 ? 2 * nk1 : nk1;

    auto gload = [&](int kt, u32x4(&ra)[S::CA], u32x4(&rb)[S::CB]) {
        const T *a = A, *bp = B;
        if (kt >= nk1) {
            a = A2;
            bp = B2;
            kt -= nk1;
        }
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BM / S::VEC), r = (ch % (BM / S::VEC)) * S::VEC;
            if (ch < S::CHA) ra[c] = *(const u32x4 *)(a + (r + (kt * BK + col) * (int)lda));
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BN / S::VEC), r = (ch % (BN / S::VEC)) * S::VEC;
            if (ch < S::CHB) rb[c] = *(const u32x4 *)(bp + (r + (kt * BK + col) * (int)ldb));
        }
    };
    auto sstore = [&](int buf, const u32x4(&ra)[S::CA], const u32x4(&rb)[S::CB]) {
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BM / S::VEC), r = (ch % (BM / S::VEC)) * S::VEC;
            if (ch < S::CHA) *(u32x4 *)(As + (buf * BK + col) * S::LDM + r) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int col = ch / (BN / S::VEC), r = (ch % (BN / S::VEC)) * S::VEC;
            if (ch < S::CHB) *(u32x4 *)(Bs + (buf * BK + col) * S::LDN + r) = rb[c];
        }
    };
    auto compute = [&](int cur) {
        const T *as = As + cur * BK * S::LDM + wm * (BM / WM) + gi;
        const T *bs = Bs + cur * BK * S::LDN + wn * (BN / WN) + gi;
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            T fa[S::MB], fb[S::NB];
#pragma unroll
            for (int m = 0; m < S::MB; ++m) fa[m] = as[(s * 4 + gg) * S::LDM + m * 16];
#pragma unroll
            for (int n = 0; n < S::NB; ++n) fb[n] = bs[(s * 4 + gg) * S::LDN + n * 16];
#pragma unroll
            for (int m = 0; m < S::MB; ++m)
#pragma unroll
                for (int n = 0; n < S::NB; ++n)
                    acc[m][n] = SWAP ? CM<T>::mfma(fb[n], fa[m], acc[m][n]) : CM<T>::mfma(fa[m], fb[n], acc[m][n]);
        }
    };

    gload(0, ra0, rb0);
    gload(1, ra1, rb1);
    sstore(0, ra0, rb0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
        // slice kt staged in LDS buffer 0, slice kt + 1 in the second register set
        if (kt + 2 < nk) gload(kt + 2, ra0, rb0);
        compute(0);
        sstore(1, ra1, rb1);
        __syncthreads();
        // slice kt + 1 staged in buffer 1, slice kt + 2 in the first set
        if (kt + 3 < nk) gload(kt + 3, ra1, rb1);
        compute(1);
        if (kt + 2 < nk) sstore(0, ra0, rb0);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- rm (FP16 / BF16 / FP8)
enum { RM_F16 = 0, RM_BF16 = 1, RM_FP8 = 2 };

template <int KIND> struct RM;
template <> struct RM<RM_F16> {
    typedef uint16_t T;
    typedef u32x4 frag_t;  // 8 halves
    static constexpr int KSTEP = 32;
    __device__ static inline float4_t mfma(frag_t a, frag_t b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a), __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
    }
};
template <> struct RM<RM_BF16> {
    typedef uint16_t T;
    typedef u32x4 frag_t;
    static constexpr int KSTEP = 32;
    __device__ static inline float4_t mfma(frag_t a, frag_t b, float4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    }
};
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
// FP8 E4M3 operands, 16 x 16 x 128 per instruction (format code 0 for both
// operands, no block scaling: the per-tile power-of-two scales are applied in
// the epilogue).  Each lane holds 32 consecutive K elements of its row; A and
// B use the same lane -> K assignment, so the K order inside the instruction
// does not affect the sum.
template <> struct RM<RM_FP8> {
    typedef uint8_t T;
    typedef i32x8 frag_t;  // 32 bytes
    static constexpr int KSTEP = 128;
    __device__ static inline float4_t mfma(frag_t a, frag_t b, float4_t c)
    {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
    // block-scaled form: sa, sb are the E8M0 scales (value 2^(s - 127), in the
    // low byte) of the 32 K elements this lane holds of its A row and B column
    __device__ static inline float4_t mfma_mx(frag_t a, frag_t b, float4_t c, int sa, int sb)
    {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
    }
};

// The operand of one lane of the block-scaled FP8 instruction: bytes
// 0 .. 15 and 64 .. 79 from p (a row of a 128-element K slice, offset 16 gg).
__device__ inline i32x8 mx_frag(const uint8_t *p)
{
    const u32x4 lo = *(const u32x4 *)p, hi = *(const u32x4 *)(p + 64);
    return (i32x8){(int32_t)lo[0], (int32_t)lo[1], (int32_t)lo[2], (int32_t)lo[3],
                   (int32_t)hi[0], (int32_t)hi[1], (int32_t)hi[2], (int32_t)hi[3]};
}

template <int KIND, int BM, int BN, int BK, int WM = 2, int WN = 2>
struct RMShape {
    typedef typename RM<KIND>::T T;
    static constexpr int NTH = 64 * WM * WN;
    static constexpr int ROWB = BK * (int)sizeof(T);       // bytes per staged row
    static constexpr int LDB = ROWB + 16;                   // padded row stride in bytes
    static constexpr int CPR = ROWB / 16;                   // 16-byte chunks per row
    static constexpr int CHA = BM * CPR, CHB = BN * CPR;
    static constexpr int CA = (CHA + NTH - 1) / NTH, CB = (CHB + NTH - 1) / NTH;
    static constexpr int MB = BM / WM / 16, NB = BN / WN / 16;
    static constexpr size_t SMEM = (size_t)2 * (BM + BN) * LDB;
    static constexpr size_t SMEM_MX = SMEM + (size_t)2 * (BM + BN) * 4;  // + one scale word per row and buffer
    static_assert((CHA % NTH == 0 || CHA < NTH) && (CHB % NTH == 0 || CHB < NTH), "load split");
    static_assert(BK % RM<KIND>::KSTEP == 0 && MB >= 1 && NB >= 1, "shape");
};

// MX (FP8 only): SA and SB hold E8M0 block scales, K / 32 bytes per row of
// A and of B (row-major, 4-byte aligned rows); a slice of BK = 128 spans four
// blocks, one 32-bit word per row, staged through LDS beside the codes.  The
// lane that holds K elements 32 gg .. 32 gg + 31 of a row passes byte gg.
template <int KIND, int BM, int BN, int BK, int WM = 2, int WN = 2, bool MX = false>
__device__ inline void rm_block(const typename RM<KIND>::T *__restrict__ A, int64_t lda,
                                const typename RM<KIND>::T *__restrict__ B, int64_t ldb, int K,
                                float4_t (&acc)[RMShape<KIND, BM, BN, BK, WM, WN>::MB][RMShape<KIND, BM, BN, BK, WM, WN>::NB],
                                uint8_t *smem, const uint8_t *__restrict__ SA = nullptr,
                                const uint8_t *__restrict__ SB = nullptr)
{
    static_assert(!MX || (KIND == RM_FP8 && BK == 128 && BM + BN <= 64 * WM * WN), "MX: one scale word per row and slice");
    typedef RMShape<KIND, BM, BN, BK, WM, WN> S;
    typedef typename RM<KIND>::T T;
    typedef typename RM<KIND>::frag_t F;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int gi = lane & 15, gg = lane >> 4;
    uint8_t *As = smem;                         // [2][BM][LDB]
    uint8_t *Bs = smem + 2 * BM * S::LDB;       // [2][BN][LDB]
    uint32_t *Ss = (uint32_t *)(smem + 2 * (BM + BN) * S::LDB);  // MX: [2][BM + BN] scale words
    u32x4 ra[S::CA], rb[S::CB];
    uint32_t rs = 0;
    const int nk = K / BK;
    // every thread stages whole chunks (no partial rounds): the MX variant
    // drops the always-true bounds tests so that its products and the next
    // slice's stores stay in one block, in that order
    constexpr bool FULL = MX && S::CHA % S::NTH == 0 && S::CHB % S::NTH == 0 && BM + BN == S::NTH;

    auto gload = [&](int kt) {
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int row = ch / S::CPR, cb = (ch % S::CPR) * 16;
            if (FULL || ch < S::CHA) ra[c] = *(const u32x4 *)((const uint8_t *)(A + (int64_t)row * lda + kt * BK) + cb);
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int row = ch / S::CPR, cb = (ch % S::CPR) * 16;
            if (FULL || ch < S::CHB) rb[c] = *(const u32x4 *)((const uint8_t *)(B + (int64_t)row * ldb + kt * BK) + cb);
        }
        if constexpr (MX) {
            const uint32_t *src = tid < BM ? (const uint32_t *)SA + (int64_t)tid * nk
                                           : (const uint32_t *)SB + (int64_t)(tid - BM) * nk;
            if (FULL || tid < BM + BN) rs = src[kt];
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < S::CA; ++c) {
            int ch = tid + S::NTH * c;
            int row = ch / S::CPR, cb = (ch % S::CPR) * 16;
            if (FULL || ch < S::CHA) *(u32x4 *)(As + (buf * BM + row) * S::LDB + cb) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            int ch = tid + S::NTH * c;
            int row = ch / S::CPR, cb = (ch % S::CPR) * 16;
            if (FULL || ch < S::CHB) *(u32x4 *)(Bs + (buf * BN + row) * S::LDB + cb) = rb[c];
        }
        if constexpr (MX) {
            if (FULL || tid < BM + BN) Ss[buf * (BM + BN) + tid] = rs;
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        const uint8_t *as = As + (cur * BM + wm * (BM / WM) + gi) * S::LDB;
        const uint8_t *bs = Bs + (cur * BN + wn * (BN / WN) + gi) * S::LDB;
        // raised issue priority while multiplying, so that a wave whose
        // operands are in LDS goes ahead of waves still loading (measured
        // +0.4% on the mixed factorization)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int s = 0; s < BK / RM<KIND>::KSTEP; ++s) {
            constexpr int KS = RM<KIND>::KSTEP;  // K per instruction; KS / 4 per lane
            const int kb = (s * KS + (KS / 4) * gg) * (int)sizeof(T);
            F fa[S::MB], fb[S::NB];
            if constexpr (MX) {
                // the block-scaled instruction splits K into two halves of 64:
                // lane group gg passes K elements 16 gg .. 16 gg + 15 of each
                // half, and block b (K 32 b .. 32 b + 31) takes lane group b's
                // scale; so each lane reads those two 16-byte pieces of its row
                // and passes the scale of block gg
#pragma unroll
                for (int m = 0; m < S::MB; ++m) fa[m] = mx_frag(as + m * 16 * S::LDB + 16 * gg);
#pragma unroll
                for (int n = 0; n < S::NB; ++n) fb[n] = mx_frag(bs + n * 16 * S::LDB + 16 * gg);
            } else {
#pragma unroll
                for (int m = 0; m < S::MB; ++m) fa[m] = *(const F *)(as + m * 16 * S::LDB + kb);
#pragma unroll
                for (int n = 0; n < S::NB; ++n) fb[n] = *(const F *)(bs + n * 16 * S::LDB + kb);
            }
            if constexpr (MX) {
                const uint32_t *ss = Ss + cur * (BM + BN);
                int sa[S::MB], sb[S::NB];
#pragma unroll
                for (int m = 0; m < S::MB; ++m) sa[m] = (ss[wm * (BM / WM) + m * 16 + gi] >> (8 * gg)) & 0xff;
#pragma unroll
                for (int n = 0; n < S::NB; ++n) sb[n] = (ss[BM + wn * (BN / WN) + n * 16 + gi] >> (8 * gg)) & 0xff;
#pragma unroll
                for (int m = 0; m < S::MB; ++m)
#pragma unroll
                    for (int n = 0; n < S::NB; ++n) acc[m][n] = RM<KIND>::mfma_mx(fa[m], fb[n], acc[m][n], sa[m], sb[n]);
                // keep the products ahead of the next slice's LDS stores: left to
                // itself the compiler sinks them below those stores' wait for the
                // global loads and the barrier, and nothing overlaps the loads
                __builtin_amdgcn_sched_barrier(0);
            } else {
#pragma unroll
                for (int m = 0; m < S::MB; ++m)
#pragma unroll
                    for (int n = 0; n < S::NB; ++n) acc[m][n] = RM<KIND>::mfma(fa[m], fb[n], acc[m][n]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // (FULL: on the last slice this rewrites the other buffer, which no
        // wave reads any more, with registers already staged -- harmless, and
        // it leaves no branch for the products to sink past)
        if (FULL || kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
}

}  // namespace mpc
