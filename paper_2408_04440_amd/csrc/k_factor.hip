// The factorization's tasks (Sec. V.A): POTRF of a diagonal tile, TRSM of the
// panel below it, and the SYRK/GEMM trailing update grouped per precision
// class, all for gfx950.
#include "common.h"
#include "gemm_core.h"
#include "launch.h"

namespace mpc {

// ---------------------------------------------------------------- POTRF
// Cholesky of the 64 x 64 block at (j0, j0) of an FP64 tile (column-major,
// leading dimension b) by one wavefront, in four quarters of 16 columns: lane
// r holds its row of the quarter in registers, first less the earlier
// quarters' contribution, then right-looking over the quarter's columns with
// each finished column broadcast through LDS (a[c][r] = L(j0 + r, j0 + c)).
// A pivot that is not positive (or NaN) records its 1-based global column in
// *info (minimum over failures); the computation then continues on NaNs and
// still terminates.  Zeros are written above the diagonal.
__device__ inline void wave_sync()
{
    // orders one wavefront's LDS accesses across lanes (the hardware executes a
    // wave's LDS instructions in order; this keeps the compiler from moving them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64) void potrf_block_kernel(double *tile, int b, int j0, int64_t col0, int64_t n,
                                                         unsigned long long *info)
{
    __builtin_amdgcn_s_setprio(3);  // the panel chain: issue ahead of update waves sharing the SIMD
    __shared__ double a[64][65];
    const int r = threadIdx.x;
    double *base = tile + j0 + (int64_t)j0 * b;
#pragma nounroll
    for (int h = 0; h < 64; h += 16) {
        double x[16];  // x[j] = A(j0 + r, j0 + h + j)
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = base[r + (int64_t)(h + j) * b];
        for (int c = 0; c < h; ++c) {  // less L(r, 0:h) L(h+j, 0:h)^T
            const double lrc = a[c][r];
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] -= lrc * a[c][h + j];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            a[h + c][r] = x[c];
            wave_sync();
            const double d = a[h + c][h + c];
            if (r == 0 && !(d > 0.0) && col0 + j0 + h + c < n)
                atomicMin(info, (unsigned long long)(col0 + j0 + h + c + 1));
            const double piv = sqrt(d);
            x[c] = (r == h + c) ? piv : x[c] / piv;
            wave_sync();
            a[h + c][r] = x[c];
            wave_sync();
#pragma unroll
            for (int j = c + 1; j < 16; ++j) x[j] -= x[c] * a[h + c][h + j];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) base[r + (int64_t)(h + j) * b] = (r >= h + j) ? x[j] : 0.0;
        wave_sync();
    }
}

// ---------------------------------------------------------------- TRSM
// X = W L^-T for strips of 64 rows (X L^T = W, L lower nL x nL, FP64), four
// waves per strip, each owning 16 rows.  Column blocks of 32: the block's
// right-hand side W - X_left L_row^T is formed with FP64 MFMA from the
// already solved columns -- each wave reads its own rows of X and the L rows
// straight into registers, the next 48 columns of K in flight while the
// current ones are multiplied, with no barrier inside the K loop -- then
// solved by forward substitution against the 32 x 32 diagonal block, one row
// per lane in registers.
// mode 0: the panel of step k -- item I = k+1+blockIdx.y, W = tile (I,k) in
//         its work precision (FP64, or FP32 for lower classes), X = p64[I];
//         the strip's largest |X| is folded into pmax[I] (atomic max of the
//         FP64 bits, which order like the values; the caller zeroes pmax),
//         and the first column holding an Inf or NaN into P.info (every
//         off-diagonal factor tile passes here, so a non-finite value is
//         reported even where a low-precision code would saturate it);
// mode 1: one FP64 strip set in place (W = X = xin, leading dimension ldin).
// nL is a multiple of 32.
__global__ __launch_bounds__(256) void trsm_kernel(Tiles T, Panel P, int k, const double *__restrict__ L, int64_t ldl,
                                                   int nL, double *xin, int64_t ldin, int mode)
{
    __builtin_amdgcn_s_setprio(3);  // the panel chain: issue ahead of update waves sharing the SIMD
    __shared__ double ts[32][64 + 1];  // right-hand side / solution: ts[c][row]
    __shared__ double lb[32][33];      // diagonal block: lb[cc][c] = L(cb + c, cb + cc)
    const void *W;
    bool wf32 = false;
    int64_t ldw, ldx;
    double *X;
    if (mode == 0) {
        const int I = k + 1 + blockIdx.y;
        wf32 = T.map[I + (int64_t)k * T.nt] != P64;
        W = T.slots + tile_index(I, k) * T.slot_bytes;
        ldw = T.b;
        X = P.p64 + (int64_t)I * T.b * T.b;
        ldx = T.b;
    } else {
        W = xin;
        ldw = ldin;
        X = xin;
        ldx = ldin;
    }
    const int row0 = blockIdx.x * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gi = lane & 15, gg = lane >> 4;
    double *Xs = X + row0;
    double xmax = 0.0;     // wave 0: largest |X| written
    int bad = 0x7FFFFFFF;  // wave 0: first column (in the tile) of a non-finite X written

    for (int cb = 0; cb < nL; cb += 32) {
        // this column block's right-hand side and diagonal block, read before
        // the K loop so that their latency overlaps its first loads
        double wv[4][2], lv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = wave * 16 + acc_row<double>(gg, v);
            const int64_t o0 = (int64_t)(row0 + r) + (int64_t)(cb + gi) * ldw;
            const int64_t o1 = o0 + 16 * ldw;
            wv[v][0] = wf32 ? (double)((const float *)W)[o0] : ((const double *)W)[o0];
            wv[v][1] = wf32 ? (double)((const float *)W)[o1] : ((const double *)W)[o1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, c = e & 31, cc = e >> 5;
            lv[q] = L[(cb + c) + (int64_t)(cb + cc) * ldl];
        }
        double4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        // MFMA k-step kk (4 columns of K): a = X(row0 + 16 wave + gi, kk + gg),
        // b_n = L(cb + 16 n + gi, kk + gg); chunks of four k-steps
        const double *xa = Xs + wave * 16 + gi + (int64_t)gg * ldx;
        const double *lp = L + (cb + gi) + (int64_t)gg * ldl;
        double a0[4], b0[4][2], a1[4], b1[4][2], a2[4], b2[4][2], a3[4], b3[4][2];
        // offsets within one tile (below b * b), kept in 32 bits
        const int ldx32 = (int)ldx, ldl32 = (int)ldl;
        auto load = [&](int kc, double(&a)[4], double(&bv)[4][2]) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int kk = kc * 16 + 4 * s;
                a[s] = xa[kk * ldx32];
                bv[s][0] = lp[kk * ldl32];
                bv[s][1] = lp[16 + kk * ldl32];
            }
        };
        auto mma = [&](const double(&a)[4], const double(&bv)[4][2]) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bv[s][0], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bv[s][1], acc1, 0, 0, 0);
            }
        };
        // three chunks in flight (a chunk is 512 cycles of MFMA work, well
        // short of a load's latency); nc is even
        const int nc = cb / 16;
        if (nc > 0) {
            load(0, a0, b0);
            load(1, a1, b1);
            if (nc > 2) load(2, a2, b2);
            for (int kc = 0; kc < nc; kc += 4) {
                if (kc + 3 < nc) load(kc + 3, a3, b3);
                mma(a0, b0);
                if (kc + 4 < nc) load(kc + 4, a0, b0);
                mma(a1, b1);
                if (kc + 2 >= nc) break;
                if (kc + 5 < nc) load(kc + 5, a1, b1);
                mma(a2, b2);
                if (kc + 6 < nc) load(kc + 6, a2, b2);
                mma(a3, b3);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = wave * 16 + acc_row<double>(gg, v);
            ts[gi][r] = wv[v][0] - acc0[v];
            ts[16 + gi][r] = wv[v][1] - acc1[v];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q, c = e & 31, cc = e >> 5;
            lb[cc][c] = lv[q];
        }
        __syncthreads();
        if (wave == 0) {
            double t[32];
#pragma unroll
            for (int c = 0; c < 32; ++c) t[c] = ts[c][lane];
            // column by column: once x_c is final it is divided out and
            // subtracted from every later column of the row -- each x_j still
            // receives its terms in increasing c, then its division, but the
            // updates of different j are independent of each other
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                t[c] = t[c] / lb[c][c];
#pragma unroll
                for (int j = c + 1; j < 32; ++j) t[j] -= t[c] * lb[c][j];
            }
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                Xs[lane + (int64_t)(cb + c) * ldx] = t[c];
                xmax = fmax(xmax, fabs(t[c]));
                if (!(fabs(t[c]) <= 1.7976931348623157e308)) bad = min(bad, cb + c);
            }
        }
        __syncthreads();  // the solved columns are read back by the next column block
    }
    if (mode == 0 && wave == 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) xmax = fmax(xmax, __shfl_xor(xmax, off));
        if (lane == 0) atomicMax(P.pmax + k + 1 + blockIdx.y, (unsigned long long)__double_as_longlong(xmax));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) bad = min(bad, __shfl_xor(bad, off));
        if (lane == 0 && bad != 0x7FFFFFFF && P.info)
            atomicMin(P.info, (unsigned long long)((int64_t)k * T.b + bad + 1));
    }
}

// ---------------------------------------------------------------- SYRK inside a diagonal tile
// C -= X X^T on the lower 64 x 64 blocks of an M x M FP64 block (K = 64).
__global__ __launch_bounds__(256) void syrk_tile_kernel(const double *X, double *Cm, int b, int nblk)
{
    __builtin_amdgcn_s_setprio(3);  // the panel chain: issue ahead of update waves sharing the SIMD
    extern __shared__ __align__(16) char smem_raw[];
    // block (bi, bj), bi >= bj, from the linear index
    int t = blockIdx.x;
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    int bj = t - bi * (bi + 1) / 2;
    double4_t acc[2][2];
    for (int m = 0; m < 2; ++m)
        for (int nn = 0; nn < 2; ++nn) acc[m][nn] = (double4_t){0.0, 0.0, 0.0, 0.0};
    cm_block<double, 64, 64, 16>(X + bi * 64, b, X + bj * 64, b, 64, acc, (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1, gi = lane & 15, gg = lane >> 4;
    double *C = Cm + bi * 64 + (int64_t)bj * 64 * b;
    for (int m = 0; m < 2; ++m)
        for (int nn = 0; nn < 2; ++nn)
            for (int v = 0; v < 4; ++v) {
                int r = wm * 32 + m * 16 + acc_row<double>(gg, v), c = wn * 32 + nn * 16 + gi;
                C[r + (int64_t)c * b] -= acc[m][nn][v];
            }
}

void launch_potrf_tile(const Tiles &T, int k, unsigned long long *info, hipStream_t st)
{
    const int b = T.b;
    double *tile = (double *)(T.slots + tile_index(k, k) * T.slot_bytes);
    Panel none{};
    for (int j0 = 0; j0 < b; j0 += 64) {
        potrf_block_kernel<<<1, 64, 0, st>>>(tile, b, j0, (int64_t)k * b, T.n, info);
        const int M = b - j0 - 64;
        if (M <= 0) break;
        double *xin = tile + (j0 + 64) + (int64_t)j0 * b;
        trsm_kernel<<<dim3(M / 64, 1), 256, 0, st>>>(T, none, k, tile + j0 + (int64_t)j0 * b, b, 64, xin, b, 1);
        const int nblk = M / 64;
        syrk_tile_kernel<<<nblk * (nblk + 1) / 2, 256, CMShape<double, 64, 64, 16>::SMEM, st>>>(
            xin, tile + (j0 + 64) + (int64_t)(j0 + 64) * b, b, nblk);
    }
    launch_zero_upper_diag(T, k, st);
}

void launch_trsm_panel(const Tiles &T, const Panel &P, int k, hipStream_t st)
{
    const int np = T.nt - k - 1;
    if (np <= 0) return;
    const double *L = (const double *)(T.slots + tile_index(k, k) * T.slot_bytes);
    trsm_kernel<<<dim3(T.b / 64, np), 256, 0, st>>>(T, P, k, L, T.b, T.b, nullptr, 0, 0);
}

// ---------------------------------------------------------------- grouped trailing update
// One launch per class: every work item (I, J) is a b x b tile update
// A_IJ -= L_Ik L_Jk^T from the class's panel copies, or, for a pair of steps,
// A_IJ -= L_Ik L_Jk^T + L_I,k+1 L_J,k+1^T with K = 2b in one accumulation.  Blocks are
// renumbered XCD-aware so the blocks of one item share an L2; an item with
// I == J (SYRK, always FP64) computes its lower blocks only.
// The FP64 block keeps to 64 registers so that two blocks share a compute
// unit (eight waves per SIMD).
template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 8 : 1)))
void update_cm_kernel(Tiles Tt, const T *panel0, const T *panel1, const int32_t *items)
{
    typedef CMShape<T, BM, BN, BK, WM, WN> S;
    extern __shared__ __align__(16) char smem_raw[];
    const int b = Tt.b;
    const int tmn = b / BM, tnn = b / BN;
    const int64_t lg = xcd_remap(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (tmn * tnn));
    const int rem = (int)(lg % (tmn * tnn));
    const int tm = rem % tmn, tn = rem / tmn;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    if (I == J && tn * BN > tm * BM + BM - 1) return;
    const int64_t bb = (int64_t)b * b;
    typename CM<T>::acc_t acc[S::MB][S::NB];
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[m][n][v] = 0;
    // FP64 accumulators hold four rows 4 apart per lane; with the operands
    // swapped each lane owns one row instead, so the stores below cover
    // 16 contiguous doubles per column.  FP32 rows are already contiguous.
    constexpr bool SWAP = sizeof(T) == 8;
    constexpr bool PRIO = sizeof(T) == 4;  // measured: helps FP32, neutral for FP64
    // a pair of steps: K continues over the next panel column; FP64 fetches
    // two K slices ahead (measured +2.3% for the FP64 update alone)
    if constexpr (sizeof(T) == 8)
        cm_block_deep<T, BM, BN, BK, WM, WN, SWAP>(panel0 + I * bb + tm * BM, b, panel0 + J * bb + tn * BN, b, b, acc,
                                                   (T *)smem_raw, panel1 ? panel1 + I * bb + tm * BM : nullptr,
                                                   panel1 ? panel1 + J * bb + tn * BN : nullptr);
    else
        cm_block<T, BM, BN, BK, WM, WN, SWAP, PRIO>(panel0 + I * bb + tm * BM, b, panel0 + J * bb + tn * BN, b, b, acc,
                                                    (T *)smem_raw, panel1 ? panel1 + I * bb + tm * BM : nullptr,
                                                    panel1 ? panel1 + J * bb + tn * BN : nullptr);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM, gi = lane & 15, gg = lane >> 4;
    T *C = (T *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes) + tm * BM + (int64_t)tn * BN * b;
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n) {
            if (SWAP) {
                int r = wm * (BM / WM) + m * 16 + gi, c = wn * (BN / WN) + n * 16;
                T *p = C + r + (int64_t)c * b;
#pragma unroll
                for (int v = 0; v < 4; ++v) p[(int64_t)acc_row<T>(gg, v) * b] -= acc[m][n][v];
            } else {
                int r = wm * (BM / WM) + m * 16, c = wn * (BN / WN) + n * 16 + gi;
                T *p = C + r + (int64_t)c * b;
#pragma unroll
                for (int v = 0; v < 4; ++v) p[acc_row<T>(gg, v)] -= acc[m][n][v];
            }
        }
}

// Up to four panel columns applied in one accumulation (the steps of one or
// two pairs): their copies and scale exponents.
template <typename T> struct PanelSet {
    const T *p[4];
    const int32_t *s[4];  // scale exponents (class q copy of tile I at s[h][I * 4 + q]); unused for the split copies
    const uint8_t *x[4];  // block-scaled FP8: E8M0 block scales of the copies (Panel::p8x)
    int n;
};

template <int KIND, int BM, int BN, int BK, int WM, int WN, bool MX = false>
__global__ __launch_bounds__(64 * WM * WN) void update_rm_kernel(Tiles Tt, PanelSet<typename RM<KIND>::T> ps, int q,
                                                                 const int32_t *items)
{
    typedef RMShape<KIND, BM, BN, BK, WM, WN> S;
    typedef typename RM<KIND>::T T;
    extern __shared__ __align__(16) char smem_raw[];
    const int b = Tt.b;
    const int tmn = b / BM, tnn = b / BN;
    const int64_t lg = xcd_remap(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (tmn * tnn));
    const int rem = (int)(lg % (tmn * tnn));
    const int tm = rem % tmn, tn = rem / tmn;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    const int64_t bb = (int64_t)b * b;
    float4_t acc[S::MB][S::NB];
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n) acc[m][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
    int tsum = 0;
    if constexpr (MX) {
        // block-scaled copies: the MFMA applies every block's scales, so the
        // steps' products add at their own values
        const int64_t xb = bb / 32, xrow = b / 32;
#pragma nounroll
        for (int h = 0; h < ps.n; ++h)
            rm_block<KIND, BM, BN, BK, WM, WN, true>(ps.p[h] + I * bb + (int64_t)tm * BM * b, b,
                                                     ps.p[h] + J * bb + (int64_t)tn * BN * b, b, b, acc,
                                                     (uint8_t *)smem_raw, ps.x[h] + I * xb + (int64_t)tm * BM * xrow,
                                                     ps.x[h] + J * xb + (int64_t)tn * BN * xrow);
    } else {
        // Scaled copies: the product of step h is acc * 2^-(t_I + t_J) with its own
        // exponent sum.  The steps are taken in decreasing exponent sum (smallest
        // values first); before each later step the accumulator is rescaled down
        // to that step's exponent sum, which is exact and cannot overflow, and
        // the step's product then adds at that scale.
        int ord[4], ts[4];
        for (int h = 0; h < ps.n; ++h) {
            const int t = ps.s[h][I * 4 + q] + ps.s[h][J * 4 + q];
            int pos = h;
            while (pos > 0 && ts[pos - 1] < t) {  // insertion by decreasing t (stable)
                ts[pos] = ts[pos - 1];
                ord[pos] = ord[pos - 1];
                --pos;
            }
            ts[pos] = t;
            ord[pos] = h;
        }
        tsum = ts[0];
#pragma nounroll
        for (int h = 0; h < ps.n; ++h) {
            const T *pn = ps.p[ord[h]];
            if (h) {
                const int t2 = ts[h];
#pragma unroll
                for (int m = 0; m < S::MB; ++m)
#pragma unroll
                    for (int n = 0; n < S::NB; ++n)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[m][n][v] = ldexpf(acc[m][n][v], t2 - tsum);
                tsum = t2;
            }
            rm_block<KIND, BM, BN, BK, WM, WN>(pn + I * bb + (int64_t)tm * BM * b, b,
                                               pn + J * bb + (int64_t)tn * BN * b, b, b, acc, (uint8_t *)smem_raw);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM, gi = lane & 15, gg = lane >> 4;
    float *C = (float *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes) + tm * BM + (int64_t)tn * BN * b;
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n) {
            int r = wm * (BM / WM) + m * 16 + 4 * gg, c = wn * (BN / WN) + n * 16 + gi;
            float *p = C + r + (int64_t)c * b;
#pragma unroll
            for (int v = 0; v < 4; ++v) p[v] -= ldexpf(acc[m][n][v], -tsum);
        }
}

// FP32-class update from three-way BF16 splits of the operands (v = hi + mid
// + lo, the FP32 copy exactly): the six significant part products (mid,mid),
// (hi,lo), (lo,hi), (hi,mid), (mid,hi), (hi,hi), smallest first, each over
// the full K on the BF16 MFMA with FP32 accumulation; the three products
// below a float rounding of the result -- (mid,lo), (lo,mid), (lo,lo) -- are
// dropped.  For several steps (a pair, or two pairs) the panels' products of
// one kind follow each other.  Operands: panel + I*3*b*b + part*b*b,
// row-major b x b.
template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void update_split_kernel(Tiles Tt, PanelSet<uint16_t> ps,
                                                                    const int32_t *items)
{
    typedef RMShape<RM_BF16, BM, BN, BK, WM, WN> S;
    extern __shared__ __align__(16) char smem_raw[];
    const int b = Tt.b;
    const int tmn = b / BM, tnn = b / BN;
    const int64_t lg = xcd_remap(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (tmn * tnn));
    const int rem = (int)(lg % (tmn * tnn));
    const int tm = rem % tmn, tn = rem / tmn;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    const int64_t bb = (int64_t)b * b, bb3 = 3 * bb;
    float4_t acc[S::MB][S::NB];
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n) acc[m][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
    const int npan = ps.n;
#pragma nounroll
    for (int s = 0; s < 6 * npan; ++s) {
        const int t = s / npan;                      // kind of product, smallest first
        const int pa = (0x010201 >> (4 * t)) & 0xF;  // part of the I operand: 1 0 2 0 1 0
        const int pb = (0x001021 >> (4 * t)) & 0xF;  // part of the J operand: 1 2 0 1 0 0
        const uint16_t *pn = ps.p[s % npan];
        rm_block<RM_BF16, BM, BN, BK, WM, WN>(pn + I * bb3 + pa * bb + (int64_t)tm * BM * b, b,
                                              pn + J * bb3 + pb * bb + (int64_t)tn * BN * b, b, b, acc,
                                              (uint8_t *)smem_raw);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM, gi = lane & 15, gg = lane >> 4;
    float *C = (float *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes) + tm * BM + (int64_t)tn * BN * b;
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
        for (int n = 0; n < S::NB; ++n) {
            int r = wm * (BM / WM) + m * 16 + 4 * gg, c = wn * (BN / WN) + n * 16 + gi;
            float *p = C + r + (int64_t)c * b;
#pragma unroll
            for (int v = 0; v < 4; ++v) p[v] -= acc[m][n][v];
        }
}

template <int BM, int BN, int BK, int WM, int WN>
static void launch_split(const Tiles &T_, const PanelSet<uint16_t> &ps, const int32_t *items, int nitems,
                         hipStream_t st)
{
    typedef RMShape<RM_BF16, BM, BN, BK, WM, WN> S;
    auto k = update_split_kernel<BM, BN, BK, WM, WN>;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::SMEM);
        attr = true;
    }
    const int64_t grid = (int64_t)nitems * (T_.b / BM) * (T_.b / BN);
    k<<<(unsigned)grid, S::NTH, S::SMEM, st>>>(T_, ps, items);
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
static void launch_cm(const Tiles &T_, const T *panel0, const T *panel1, const int32_t *items, int nitems,
                      hipStream_t st)
{
    typedef CMShape<T, BM, BN, BK, WM, WN> S;
    auto k = update_cm_kernel<T, BM, BN, BK, WM, WN>;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::SMEM);
        attr = true;
    }
    const int64_t grid = (int64_t)nitems * (T_.b / BM) * (T_.b / BN);
    k<<<(unsigned)grid, S::NTH, S::SMEM, st>>>(T_, panel0, panel1, items);
}

template <int KIND, int BM, int BN, int BK, int WM, int WN, bool MX = false>
static void launch_rm(const Tiles &T_, const PanelSet<typename RM<KIND>::T> &ps, int q, const int32_t *items,
                      int nitems, hipStream_t st)
{
    typedef RMShape<KIND, BM, BN, BK, WM, WN> S;
    constexpr size_t smem = MX ? S::SMEM_MX : S::SMEM;
    auto k = update_rm_kernel<KIND, BM, BN, BK, WM, WN, MX>;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        attr = true;
    }
    const int64_t grid = (int64_t)nitems * (T_.b / BM) * (T_.b / BN);
    k<<<(unsigned)grid, S::NTH, smem, st>>>(T_, ps, q, items);
}

// Block shapes per class from a sweep on MI355X (1024 x 1024 tiles):
// FP64 128 x 128 with 16 waves of 32 x 32, FP32 256 x 128 with 8 waves,
// FP16/BF16 256 x 256 with 16 waves, FP8 128 x 128 with 4 waves; tiles of
// 128 fall back to 128 x 128 blocks.
void launch_update(const Tiles &T, const Panel *const *Ps, int npan, int q, const int32_t *items, int nitems,
                   hipStream_t st, bool small)
{
    if (nitems <= 0 || npan < 1 || npan > 4) return;
    // "small": a launch beside the running updates (the look-ahead stream)
    // uses block shapes whose LDS fits in the slot one finished update block
    // frees; a 1024-thread block with 147 KB of LDS would wait for a whole
    // idle compute unit.
    const bool big = (T.b % 256) == 0 && !small;
    const Panel &P = *Ps[0];
    const Panel *P2 = npan > 1 ? Ps[1] : nullptr;  // the FP64 / FP32-MFMA updates take one pair at most
    switch (q) {
    case P64: launch_cm<double, 128, 128, 16, 4, 4>(T, P.p64, P2 ? P2->p64 : nullptr, items, nitems, st); break;
    case P32:
        if (T.lo32) {
            PanelSet<uint16_t> ps{};
            ps.n = npan;
            for (int h = 0; h < npan; ++h) ps.p[h] = Ps[h]->p32s;
            if (big) launch_split<256, 256, 64, 4, 4>(T, ps, items, nitems, st);
            else launch_split<128, 128, 64, 2, 2>(T, ps, items, nitems, st);
        } else if ((T.b % 256) == 0) {
            launch_cm<float, 256, 128, 16, 4, 2>(T, P.p32, P2 ? P2->p32 : nullptr, items, nitems, st);
        } else {
            launch_cm<float, 128, 128, 16, 2, 2>(T, P.p32, P2 ? P2->p32 : nullptr, items, nitems, st);
        }
        break;
    case P16: {
        PanelSet<uint16_t> ps{};
        ps.n = npan;
        for (int h = 0; h < npan; ++h) {
            ps.p[h] = Ps[h]->p16;
            ps.s[h] = Ps[h]->pscale;
        }
        if (T.lo16 == LO16_BF16) {
            if (big) launch_rm<RM_BF16, 256, 256, 64, 4, 4>(T, ps, q, items, nitems, st);
            else launch_rm<RM_BF16, 128, 128, 64, 2, 2>(T, ps, q, items, nitems, st);
        } else {
            if (big) launch_rm<RM_F16, 256, 256, 64, 4, 4>(T, ps, q, items, nitems, st);
            else launch_rm<RM_F16, 128, 128, 64, 2, 2>(T, ps, q, items, nitems, st);
        }
        break;
    }
    default: {
        PanelSet<uint8_t> ps{};
        ps.n = npan;
        for (int h = 0; h < npan; ++h) {
            ps.p[h] = Ps[h]->p8;
            ps.s[h] = Ps[h]->pscale;
            ps.x[h] = Ps[h]->p8x;
        }
        if (T.lo8) launch_rm<RM_FP8, 128, 128, 128, 2, 2, true>(T, ps, q, items, nitems, st);
        else launch_rm<RM_FP8, 128, 128, 128, 2, 2>(T, ps, q, items, nitems, st);
        break;
    }
    }
}

}  // namespace mpc
