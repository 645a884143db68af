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

// 128 x 128 output block per workgroup, 8 waves of 64 x 32 (two blocks share
// a compute unit: 144 KiB of LDS for the two, at most 128 registers a lane),
// K staged 16 columns at a time through LDS.
constexpr int RB = 128, RK = 16, RLD = RB + 16, RWM = 2, RWN = 4, RNT = 64 * RWM * RWN, RPER = RK * RB / RNT;
constexpr int RMB = RB / RWM / 16, RNB = RB / RWN / 16;  // MFMA tiles per wave: 4 x 2
static_assert(RNT <= 2 * RK * RLD, "the reduction reuses the A staging buffers");

__global__ __launch_bounds__(RNT) __attribute__((amdgpu_waves_per_eu(4))) void residual_kernel(Tiles T, Source S,
                                                                                              const int32_t *items,
                                                                                              double *partial)
{
    __shared__ double As[2][RK][RLD], Bs[2][RK][RLD];
    const int b = T.b, nsub = b / RB;
    const int item = blockIdx.x / (nsub * nsub), rem = blockIdx.x % (nsub * nsub);
    const int tm = rem % nsub, tn = rem / nsub;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % RWM, wn = wave / RWM, gi = lane & 15, gg = lane >> 4;
    constexpr int WTM = RB / RWM, WTN = RB / RWN;  // 64, 32
    double4_t acc[RMB][RNB];
#pragma unroll
    for (int m = 0; m < RMB; ++m)
#pragma unroll
        for (int n = 0; n < RNB; ++n) acc[m][n] = (double4_t){0.0, 0.0, 0.0, 0.0};

    const bool skip = (I == J && tn > tm);
    if (!skip) {
        const int nkt = b / RK;
        // raw stored codes in registers (the loads stay in flight across the
        // current slice's products), widened to FP64 only when staged
        uint64_t ra[RPER], rb[RPER];
        for (int K = 0; K <= J; ++K) {
            const int ca = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
            const int cbc = (J == K) ? P64 : T.map[J + (int64_t)K * T.nt];
            const int ta = T.tscale[I + (int64_t)K * T.nt], tb = T.tscale[J + (int64_t)K * T.nt];
            const char *sa = T.slots + tile_index(I, K) * T.slot_bytes;
            const char *sb = T.slots + tile_index(J, K) * T.slot_bytes;
            auto fetch = [&](const char *tile, int cls, int row0, int kt, uint64_t(&raw)[RPER]) {
                int off[RPER];  // within one tile: below b * b
#pragma unroll
                for (int c = 0; c < RPER; ++c) {
                    const int e = tid + RNT * c, r = e % RB, col = e / RB;
                    off[c] = (row0 + r) + (kt * RK + col) * b;
                }
                switch (cls) {
                case P64:
#pragma unroll
                    for (int c = 0; c < RPER; ++c) raw[c] = ((const uint64_t *)tile)[off[c]];
                    break;
                case P32:
#pragma unroll
                    for (int c = 0; c < RPER; ++c) raw[c] = ((const uint32_t *)tile)[off[c]];
                    break;
                case P16:
#pragma unroll
                    for (int c = 0; c < RPER; ++c) raw[c] = ((const uint16_t *)tile)[off[c]];
                    break;
                default:
#pragma unroll
                    for (int c = 0; c < RPER; ++c) raw[c] = ((const uint8_t *)tile)[off[c]];
                    break;
                }
            };
            auto widen = [&](uint64_t raw, int cls, int t) -> double {
                return cls == P64 ? __longlong_as_double((long long)raw) : decode_class((uint32_t)raw, cls, T.lo16, t);
            };
            auto gload = [&](int kt) {
                fetch(sa, ca, tm * RB, kt, ra);
                fetch(sb, cbc, tn * RB, kt, rb);
            };
            auto sstore = [&](int buf) {
#pragma unroll
                for (int c = 0; c < RPER; ++c) {
                    int e = tid + RNT * c;
                    int r = e % RB, col = e / RB;
                    As[buf][col][r] = widen(ra[c], ca, ta);
                    Bs[buf][col][r] = widen(rb[c], cbc, tb);
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
                    double fa[RMB], fb[RNB];
#pragma unroll
                    for (int m = 0; m < RMB; ++m) fa[m] = As[cur][s * 4 + gg][wm * WTM + m * 16 + gi];
#pragma unroll
                    for (int n = 0; n < RNB; ++n) fb[n] = Bs[cur][s * 4 + gg][wn * WTN + n * 16 + gi];
#pragma unroll
                    for (int m = 0; m < RMB; ++m)
#pragma unroll
                        for (int n = 0; n < RNB; ++n)
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
        for (int m = 0; m < RMB; ++m)
#pragma unroll
            for (int n = 0; n < RNB; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int r = tm * RB + wm * WTM + m * 16 + acc_row<double>(gg, v), c = tn * RB + wn * WTN + n * 16 + gi;
                    int64_t i = (int64_t)I * b + r, j = (int64_t)J * b + c;
                    if (i >= T.n || j >= T.n || i < j) continue;
                    double res = source_at(T, S, I, J, r, c) - acc[m][n][v];
                    double w = (i == j) ? 1.0 : (I == J ? 2.0 : 1.0);
                    s2 += w * res * res;
                }
    }
    // every wave is past the K loop's last barrier: the A staging buffers
    // are free for the reduction
    double *red = &As[0][0][0];
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
