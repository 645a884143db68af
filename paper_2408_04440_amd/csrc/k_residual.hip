// Backward error of the stored factor: R_IJ = Sigma_IJ - sum_{K<=J} L_IK L_JK^T
// for every lower tile, in FP64 with each stored tile exactly widened to FP64
// on its way into LDS; per-block sums of R^2 are reduced per tile in a fixed
// order.
#include "common.h"
#include "gemm_core.h"
#include "launch.h"

namespace mpc {

__device__ inline double source_at(const Tiles &T, const Source &S, int I, int J, int r, int c)
{
    int64_t i = (int64_t)I * T.b + r, j = (int64_t)J * T.b + c;
    if (S.dense) return S.dense[i + j * S.ld];  // i >= j: the lower part
    if (S.orig) return S.orig[tile_index(I, J) * (int64_t)T.b * T.b + r + (int64_t)c * T.b];
    double v = S.sigma[i] * S.sigma[j] * exp(-fabs(S.x[i] - S.x[j]) / S.rho);
    if (i == j) v += S.nugget;
    return v;
}

// 128 x 128 output block per workgroup, 16 waves of 32 x 32 (the FP64
// update's shape), K staged 16 columns at a time through LDS.
constexpr int RB = 128, RK = 16, RLD = RB + 16, RW = 4, RNT = 64 * RW * RW, RPER = RK * RB / RNT;

__global__ __launch_bounds__(RNT) void residual_kernel(Tiles T, Source S, const int32_t *items, double *partial)
{
    __shared__ double As[2][RK][RLD], Bs[2][RK][RLD];
    __shared__ double red[RNT];
    const int b = T.b, nsub = b / RB;
    const int item = blockIdx.x / (nsub * nsub), rem = blockIdx.x % (nsub * nsub);
    const int tm = rem % nsub, tn = rem / nsub;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % RW, wn = wave / RW, gi = lane & 15, gg = lane >> 4;
    constexpr int WT = RB / RW;  // 32
    double4_t acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const bool skip = (I == J && tn > tm);
    if (!skip) {
        const int nkt = b / RK;
        double ra[RPER], rb[RPER];
        for (int K = 0; K <= J; ++K) {
            const int ca = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
            const int cbc = (J == K) ? P64 : T.map[J + (int64_t)K * T.nt];
            const int ta = T.tscale[I + (int64_t)K * T.nt], tb = T.tscale[J + (int64_t)K * T.nt];
            const char *sa = T.slots + tile_index(I, K) * T.slot_bytes;
            const char *sb = T.slots + tile_index(J, K) * T.slot_bytes;
            auto gload = [&](int kt) {
#pragma unroll
                for (int c = 0; c < RPER; ++c) {
                    int e = tid + RNT * c;  // 0 .. RK*RB-1
                    int r = e % RB, col = e / RB;
                    int64_t off = (int64_t)(tm * RB + r) + (int64_t)(kt * RK + col) * b;
                    int64_t offb = (int64_t)(tn * RB + r) + (int64_t)(kt * RK + col) * b;
                    ra[c] = load_stored(sa, ca, T.lo16, ta, off);
                    rb[c] = load_stored(sb, cbc, T.lo16, tb, offb);
                }
            };
            auto sstore = [&](int buf) {
#pragma unroll
                for (int c = 0; c < RPER; ++c) {
                    int e = tid + RNT * c;
                    int r = e % RB, col = e / RB;
                    As[buf][col][r] = ra[c];
                    Bs[buf][col][r] = rb[c];
                }
            };
            gload(0);
            sstore(0);
            __syncthreads();
            for (int kt = 0; kt < nkt; ++kt) {
                const int cur = kt & 1;
                if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
                for (int s = 0; s < RK / 4; ++s) {
                    double fa[2], fb[2];
#pragma unroll
                    for (int m = 0; m < 2; ++m) fa[m] = As[cur][s * 4 + gg][wm * WT + m * 16 + gi];
#pragma unroll
                    for (int n = 0; n < 2; ++n) fb[n] = Bs[cur][s * 4 + gg][wn * WT + n * 16 + gi];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
#pragma unroll
                        for (int n = 0; n < 2; ++n)
                            acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[m], fb[n], acc[m][n], 0, 0, 0);
                }
                if (kt + 1 < nkt) sstore(cur ^ 1);
                __syncthreads();
            }
        }
    }
    double s2 = 0.0;
    if (!skip) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int r = tm * RB + wm * WT + m * 16 + acc_row<double>(gg, v), c = tn * RB + wn * WT + n * 16 + gi;
                    int64_t i = (int64_t)I * b + r, j = (int64_t)J * b + c;
                    if (i >= T.n || j >= T.n || i < j) continue;
                    double res = source_at(T, S, I, J, r, c) - acc[m][n][v];
                    double w = (i == j) ? 1.0 : (I == J ? 2.0 : 1.0);
                    s2 += w * res * res;
                }
    }
    red[tid] = s2;
    __syncthreads();
    for (int w = RNT / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
}

__global__ void residual_reduce_kernel(const int32_t *items, int nitems, int per_item, const double *partial, int nt,
                                       double *tile_res2)
{
    int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    double s = 0.0;
    for (int p = 0; p < per_item; ++p) s += partial[(int64_t)item * per_item + p];
    int32_t it = items[item];
    tile_res2[(it >> 16) + (int64_t)(it & 0xFFFF) * nt] = s;
}

// items: every lower tile as (I << 16 | J); scratch: partial sums
void launch_residual_items(const Tiles &T, const Source &S, const int32_t *items, int nitems, double *partial,
                           double *tile_res2, hipStream_t st)
{
    const int nsub = T.b / RB;
    residual_kernel<<<(unsigned)((int64_t)nitems * nsub * nsub), RNT, 0, st>>>(T, S, items, partial);
    residual_reduce_kernel<<<(nitems + 255) / 256, 256, 0, st>>>(items, nitems, nsub * nsub, partial, T.nt, tile_res2);
}

}  // namespace mpc
