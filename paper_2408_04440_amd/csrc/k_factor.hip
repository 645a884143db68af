// The factorization's tasks (Sec. V.A): POTRF of a diagonal tile, TRSM of the
// panel below it, and the SYRK/GEMM trailing update grouped per precision
// class, all for gfx950.
#include "common.h"
#include "gemm_core.h"
#include "launch.h"

namespace mpc {

// ---------------------------------------------------------------- POTRF
// Unblocked right-looking Cholesky of the NB x NB block at (j0, j0) of an FP64
// tile (column-major, leading dimension b), held in LDS.  A pivot that is not
// positive (or NaN) records its 1-based global column in *info (minimum over
// failures); the computation then continues on NaNs and every kernel still
// terminates.
template <int NB>
__global__ __launch_bounds__(256) void potrf_block_kernel(double *tile, int b, int j0, int64_t col0, int64_t n,
                                                          unsigned long long *info)
{
    __shared__ double a[NB][NB + 1];  // a[c][r] = tile(j0 + r, j0 + c)
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) {
        int r = e % NB, c = e / NB;
        a[c][r] = tile[(j0 + r) + (int64_t)(j0 + c) * b];
    }
    for (int c = 0; c < NB; ++c) {
        __syncthreads();
        if (tid == 0) {
            double d = a[c][c];
            if (!(d > 0.0)) {
                int64_t col = col0 + j0 + c;
                if (col < n) atomicMin(info, (unsigned long long)(col + 1));
            }
            a[c][c] = sqrt(d);
        }
        __syncthreads();
        const double piv = a[c][c];
        for (int r = c + 1 + tid; r < NB; r += 256) a[c][r] /= piv;
        __syncthreads();
        const int m = NB - c - 1;
        for (int e = tid; e < m * m; e += 256) {
            int r = c + 1 + e % m, cc = c + 1 + e / m;
            if (r >= cc) a[cc][r] -= a[c][r] * a[c][cc];
        }
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
        int r = e % NB, c = e / NB;
        tile[(j0 + r) + (int64_t)(j0 + c) * b] = (r >= c) ? a[c][r] : 0.0;
    }
}

// ---------------------------------------------------------------- TRSM
// X = W L^-T for strips of 64 rows (X L^T = W, L lower nL x nL, FP64).
// Column blocks of 32: the block's right-hand side W - X_left L_row^T is
// formed with FP64 MFMA from the already solved columns, then solved by
// substitution against the 32 x 32 diagonal block in LDS.
// mode 0: the panel of step k -- item I = k+1+blockIdx.y, W = tile (I,k) in
//         its work precision (FP64, or FP32 for lower classes), X = p64[I];
// mode 1: one FP64 strip set in place (W = X = xin, leading dimension ldin).
__global__ __launch_bounds__(256) void trsm_kernel(Tiles T, Panel P, int k, const double *L, int64_t ldl, int nL,
                                                   double *xin, int64_t ldin, int mode)
{
    __shared__ double ts[32][65];  // ts[c][r]
    __shared__ double lb[32][33];  // lb[c][r] = L(cb + r, cb + c)
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

    for (int cb = 0; cb < nL; cb += 32) {
        double4_t acc[2];
        acc[0] = (double4_t){0.0, 0.0, 0.0, 0.0};
        acc[1] = acc[0];
        const double *xa = X + (row0 + wave * 16 + gi);
        const double *lr0 = L + (cb + gi);
        for (int kk = 0; kk < cb; kk += 4) {
            double av = xa[(int64_t)(kk + gg) * ldx];
            double b0 = lr0[(int64_t)(kk + gg) * ldl];
            double b1 = lr0[16 + (int64_t)(kk + gg) * ldl];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[1], 0, 0, 0);
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int r = wave * 16 + acc_row<double>(gg, v), c = nb * 16 + gi;
                int64_t off = (int64_t)(row0 + r) + (int64_t)(cb + c) * ldw;
                double w = wf32 ? (double)((const float *)W)[off] : ((const double *)W)[off];
                ts[c][r] = w - acc[nb][v];
            }
        for (int e = tid; e < 32 * 32; e += 256) {
            int r = e & 31, c = e >> 5;
            lb[c][r] = L[(cb + r) + (int64_t)(cb + c) * ldl];
        }
        __syncthreads();
        if (tid < 64) {
            for (int c = 0; c < 32; ++c) {
                double xv = ts[c][tid];
                for (int cc = 0; cc < c; ++cc) xv -= ts[cc][tid] * lb[cc][c];
                ts[c][tid] = xv / lb[c][c];
            }
        }
        __syncthreads();
        for (int e = tid; e < 64 * 32; e += 256) {
            int r = e & 63, c = e >> 6;
            X[(int64_t)(row0 + r) + (int64_t)(cb + c) * ldx] = ts[c][r];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- SYRK inside a diagonal tile
// C -= X X^T on the lower 64 x 64 blocks of an M x M FP64 block (K = 64).
__global__ __launch_bounds__(256) void syrk_tile_kernel(const double *X, double *Cm, int b, int nblk)
{
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
        potrf_block_kernel<64><<<1, 256, 0, st>>>(tile, b, j0, (int64_t)k * b, T.n, info);
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
// One launch per class: every work item (I, J) of the step is a b x b tile
// update A_IJ -= L_Ik L_Jk^T from the class's panel copies.  Blocks are
// renumbered XCD-aware so the blocks of one item share an L2; an item with
// I == J (SYRK, always FP64) computes its lower blocks only.
template <typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void update_cm_kernel(Tiles Tt, const T *panel, const int32_t *items)
{
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
    typename CM<T>::acc_t acc[BM / 32][BN / 32];
#pragma unroll
    for (int m = 0; m < BM / 32; ++m)
#pragma unroll
        for (int n = 0; n < BN / 32; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[m][n][v] = 0;
    cm_block<T, BM, BN, BK>(panel + I * bb + tm * BM, b, panel + J * bb + tn * BN, b, b, acc, (T *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1, gi = lane & 15, gg = lane >> 4;
    T *C = (T *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes) + tm * BM + (int64_t)tn * BN * b;
#pragma unroll
    for (int m = 0; m < BM / 32; ++m)
#pragma unroll
        for (int n = 0; n < BN / 32; ++n) {
            int r = wm * (BM / 2) + m * 16, c = wn * (BN / 2) + n * 16 + gi;
            T *p = C + r + (int64_t)c * b;
#pragma unroll
            for (int v = 0; v < 4; ++v) p[acc_row<T>(gg, v)] -= acc[m][n][v];
        }
}

template <int KIND, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void update_rm_kernel(Tiles Tt, const typename RM<KIND>::T *panel,
                                                        const int32_t *pscale, int q, const int32_t *items)
{
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
    float4_t acc[BM / 32][BN / 32];
#pragma unroll
    for (int m = 0; m < BM / 32; ++m)
#pragma unroll
        for (int n = 0; n < BN / 32; ++n) acc[m][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
    rm_block<KIND, BM, BN, BK>(panel + I * bb + (int64_t)tm * BM * b, b, panel + J * bb + (int64_t)tn * BN * b, b, b,
                               acc, (uint8_t *)smem_raw);
    const int tsum = pscale[I * 4 + q] + pscale[J * 4 + q];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1, gi = lane & 15, gg = lane >> 4;
    float *C = (float *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes) + tm * BM + (int64_t)tn * BN * b;
#pragma unroll
    for (int m = 0; m < BM / 32; ++m)
#pragma unroll
        for (int n = 0; n < BN / 32; ++n) {
            int r = wm * (BM / 2) + m * 16 + 4 * gg, c = wn * (BN / 2) + n * 16 + gi;
            float *p = C + r + (int64_t)c * b;
#pragma unroll
            for (int v = 0; v < 4; ++v) p[v] -= ldexpf(acc[m][n][v], -tsum);
        }
}

void launch_update(const Tiles &T, const Panel &P, int q, const int32_t *items, int nitems, hipStream_t st)
{
    if (nitems <= 0) return;
    const int b = T.b;
    const int64_t bb = (int64_t)b * b;
    constexpr int BM = 128, BN = 128;
    const int64_t grid = (int64_t)nitems * (b / BM) * (b / BN);
    switch (q) {
    case P64:
        update_cm_kernel<double, BM, BN, 16><<<(unsigned)grid, 256, CMShape<double, BM, BN, 16>::SMEM, st>>>(
            T, P.p64, items);
        break;
    case P32:
        update_cm_kernel<float, BM, BN, 16><<<(unsigned)grid, 256, CMShape<float, BM, BN, 16>::SMEM, st>>>(
            T, P.p32, items);
        break;
    case P16:
        if (T.lo16 == LO16_BF16)
            update_rm_kernel<RM_BF16, BM, BN, 64><<<(unsigned)grid, 256, RMShape<RM_BF16, BM, BN, 64>::SMEM, st>>>(
                T, P.p16, P.pscale, q, items);
        else
            update_rm_kernel<RM_F16, BM, BN, 64><<<(unsigned)grid, 256, RMShape<RM_F16, BM, BN, 64>::SMEM, st>>>(
                T, P.p16, P.pscale, q, items);
        break;
    default:
        update_rm_kernel<RM_FP8, BM, BN, 128><<<(unsigned)grid, 256, RMShape<RM_FP8, BM, BN, 128>::SMEM, st>>>(
            T, P.p8, P.pscale, q, items);
        break;
    }
    (void)bb;
}

}  // namespace mpc
