// Covariance from samples: Sigma = scale * Xi Xi^T + nugget I, the estimator
// of the residual covariance (Sec. III.A.3, "Modeling the Temporal Dependence and
// Constructing a Covariance Matrix": the average of the R(T-P) outer products
// of the residual vectors, plus a small diagonal perturbation when there are
// fewer samples than L^2).  A tall-skinny SYRK on the FP64 MFMA: every lower
// tile (I, J) is one b x b output with K = the number of samples, written
// straight into the kept FP64 copy in the tile layout (as set_matrix does).
#include "common.h"
#include "gemm_core.h"
#include "launch.h"

namespace mpc {

// xp[i + k*ldp] = xi[i + k*ldxi] for i < n, k < m; zero elsewhere (rows up to
// NT*b, columns up to the padded sample count mp).
__global__ __launch_bounds__(256) void pack_samples_kernel(const double *xi, int64_t ldxi, int64_t n, int64_t m,
                                                           double *xp, int64_t ldp, int64_t mp)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ldp * mp) return;
    const int64_t i = e % ldp, k = e / ldp;
    xp[e] = (i < n && k < m) ? xi[i + k * ldxi] : 0.0;
}

// One 128 x 128 block of lower tile t: orig(I,J) = scale * Xp_I Xp_J^T
// (+ nugget on the diagonal below n); padding rows are zero.
typedef CMShape<double, 128, 128, 16, 4, 4> SYShape;

__global__ __launch_bounds__(1024) void syrk_samples_kernel(Tiles T, const double *xp, int64_t ldp, int mp,
                                                            double scale, double nugget, double *orig)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int b = T.b, per = (b / 128) * (b / 128);
    const int64_t lg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = lg / per;
    const int rem = (int)(lg % per);
    const int tm = rem % (b / 128), tn = rem / (b / 128);
    int I, J;
    tile_ij(t, I, J);
    double4_t acc[SYShape::MB][SYShape::NB];
#pragma unroll
    for (int m = 0; m < SYShape::MB; ++m)
#pragma unroll
        for (int q = 0; q < SYShape::NB; ++q) acc[m][q] = (double4_t){0.0, 0.0, 0.0, 0.0};
    cm_block<double, 128, 128, 16, 4, 4, true>(xp + (int64_t)I * b + tm * 128, ldp, xp + (int64_t)J * b + tn * 128, ldp,
                                               mp, acc, (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % 4, wn = wave / 4, gi = lane & 15, gg = lane >> 4;
    double *dst = orig + tile_index(I, J) * (int64_t)b * b;
#pragma unroll
    for (int m = 0; m < SYShape::MB; ++m)
#pragma unroll
        for (int q = 0; q < SYShape::NB; ++q) {
            const int r = tm * 128 + wm * 32 + m * 16 + gi;  // swapped operands: lane gi owns row r
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = tn * 128 + wn * 32 + q * 16 + acc_row<double>(gg, v);
                double val = scale * acc[m][q][v];
                if (I == J && r == c && (int64_t)I * b + r < T.n) val += nugget;
                dst[r + (int64_t)c * b] = val;
            }
        }
}

int launch_cov_samples(const Tiles &T, const double *xi, int64_t ldxi, int64_t m, double scale, double nugget,
                       double *xp, int64_t mp, double *orig, hipStream_t st)
{
    const int64_t ldp = (int64_t)T.nt * T.b;
    pack_samples_kernel<<<(unsigned)((ldp * mp + 255) / 256), 256, 0, st>>>(xi, ldxi, T.n, m, xp, ldp, mp);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)syrk_samples_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)SYShape::SMEM);
        attr = true;
    }
    const int64_t blocks = (int64_t)T.nt * (T.nt + 1) / 2 * (T.b / 128) * (T.b / 128);
    syrk_samples_kernel<<<(unsigned)blocks, 1024, SYShape::SMEM, st>>>(T, xp, ldp, (int)mp, scale, nugget, orig);
    return 0;
}

}  // namespace mpc
