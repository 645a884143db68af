// Products built on the stored factor: solves with Sigma (forward and
// backward tile substitution) and emulation draws Y = L Z (Sec. III.B), with
// the Philox4x32-10 / Box-Muller normal generator.
#include "common.h"
#include "launch.h"

namespace mpc {

// ---------------------------------------------------------------- normal draws
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the multiply/xor
// bijection with key schedule increments W0, W1.
__device__ inline void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Draw e (e = i + d*n, the column-major index of an n x ndraws array) comes
// from counter block e/4, output e%4: uniforms ((x >> 8) + 1) 2^-24 in (0,1],
// Box-Muller on (u0,u1) and (u2,u3) in FP32.  A launch writes the draws
// e0 <= e < e0 + count (e0 a multiple of n: whole columns starting at column
// e0/n) to Z with the column index taken relative to e0/n; each value depends
// only on e, so a range gives the same values as the whole sequence.
__global__ __launch_bounds__(256) void normal_kernel(uint64_t seed, int64_t e0, int64_t count, int64_t n, float *Z,
                                                     int64_t ldz, uint32_t *raw)
{
    const int64_t blk = e0 / 4 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (blk * 4 >= e0 + count) return;
    uint32_t c0 = (uint32_t)blk, c1 = (uint32_t)((uint64_t)blk >> 32), c2 = 0, c3 = 0;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint32_t o[4] = {c0, c1, c2, c3};
    float u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = (float)((o[q] >> 8) + 1u) * 5.9604644775390625e-8f;  // 2^-24
    const float twopi = 6.28318530717958647692f;
    float r0 = sqrtf(-2.0f * logf(u[0])), r1 = sqrtf(-2.0f * logf(u[2]));
    float s0, k0, s1, k1;
    sincosf(twopi * u[1], &s0, &k0);
    sincosf(twopi * u[3], &s1, &k1);
    float v[4] = {r0 * k0, r0 * s0, r1 * k1, r1 * s1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = blk * 4 + q;
        if (e < e0) continue;
        if (e >= e0 + count) break;
        const int64_t l = e - e0;
        if (Z) Z[(l % n) + (l / n) * ldz] = v[q];
        if (raw) raw[l] = o[q];
    }
}

static void launch_normal(uint64_t seed, int64_t e0, int64_t count, int64_t n, float *Z, int64_t ldz, uint32_t *raw,
                          hipStream_t st)
{
    const int64_t nb = (e0 + count + 3) / 4 - e0 / 4;  // counter blocks touched
    normal_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(seed, e0, count, n, Z, ldz, raw);
}

void launch_normal_draws(uint64_t seed, int64_t count, float *z, uint32_t *raw, hipStream_t st)
{
    launch_normal(seed, 0, count, count, z, count, raw, st);
}

void launch_normal_matrix(uint64_t seed, int64_t n, int ndraws, float *Z, int64_t ldz, hipStream_t st)
{
    launch_normal(seed, 0, n * ndraws, n, Z, ldz, nullptr, st);
}

void launch_normal_columns(uint64_t seed, int64_t n, int64_t d0, int nd, float *Z, int64_t ldz, hipStream_t st)
{
    launch_normal(seed, d0 * n, n * nd, n, Z, ldz, nullptr, st);
}

// ---------------------------------------------------------------- Y = L Z
// One 128 x 128 block of Y per workgroup of 16 waves (32 x 32 each): rows of
// tile row I, columns of draws; sum over K <= I of L_IK Z_K with FP32 MFMA,
// each stored tile widened (exactly, or rounded to FP32 for FP64 tiles) on its
// way into LDS.  The last tile rows, with the most tiles to walk, take the
// first blocks.
constexpr int SB = 128, SK = 16, SLD = SB + 4, SW = 4, SNT = 64 * SW * SW, SPER = SK * SB / SNT;

__global__ __launch_bounds__(SNT) void lower_apply_kernel(Tiles T, const float *Z, int64_t ldz, float *Y, int64_t ldy,
                                                          int ndraws)
{
    __shared__ float As[2][SK][SLD], Bs[2][SK][SLD];
    const int b = T.b, nsub = b / SB;
    const int I = T.nt - 1 - (int)(blockIdx.x / nsub), tm = blockIdx.x % nsub;
    const int s0 = blockIdx.y * SB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % SW, wn = wave / SW, gi = lane & 15, gg = lane >> 4;
    constexpr int WT = SB / SW;
    float4_t acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = (float4_t){0.f, 0.f, 0.f, 0.f};
    const int nkt = b / SK;
    float ra[SPER], rb[SPER];
    for (int K = 0; K <= I; ++K) {
        const int ca = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
        const int ta = T.tscale[I + (int64_t)K * T.nt];
        const char *sa = T.slots + tile_index(I, K) * T.slot_bytes;
        auto gload = [&](int kt) {
#pragma unroll
            for (int c = 0; c < SPER; ++c) {
                int e = tid + SNT * c;
                int r = e % SB, col = e / SB;
                ra[c] = (float)load_stored(sa, ca, T.lo16, ta, (int64_t)(tm * SB + r) + (int64_t)(kt * SK + col) * b);
                int kk = e % SK, s = e / SK;
                int64_t zr = (int64_t)K * b + kt * SK + kk;
                rb[c] = (zr < T.n && s0 + s < ndraws) ? Z[zr + (int64_t)(s0 + s) * ldz] : 0.0f;
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int c = 0; c < SPER; ++c) {
                int e = tid + SNT * c;
                As[buf][e / SB][e % SB] = ra[c];
                Bs[buf][e % SK][e / SK] = rb[c];
            }
        };
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nkt; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
            for (int s = 0; s < SK / 4; ++s) {
                float fa[2], fb[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) fa[m] = As[cur][s * 4 + gg][wm * WT + m * 16 + gi];
#pragma unroll
                for (int n = 0; n < 2; ++n) fb[n] = Bs[cur][s * 4 + gg][wn * WT + n * 16 + gi];
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int n = 0; n < 2; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[m], fb[n], acc[m][n], 0, 0, 0);
            }
            if (kt + 1 < nkt) sstore(cur ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t i = (int64_t)I * b + tm * SB + wm * WT + m * 16 + 4 * gg + v;
                int s = s0 + wn * WT + n * 16 + gi;
                if (i < T.n && s < ndraws) Y[i + (int64_t)s * ldy] = acc[m][n][v];
            }
}

void launch_lower_apply(const Tiles &T, const float *Z, int64_t ldz, float *Y, int64_t ldy, int ndraws, hipStream_t st)
{
    dim3 grid(T.nt * (T.b / SB), (ndraws + SB - 1) / SB);
    lower_apply_kernel<<<grid, SNT, 0, st>>>(T, Z, ldz, Y, ldy, ndraws);
}

// ---------------------------------------------------------------- solve
// Diagonal blocks: one wavefront per right-hand side, no barriers.  Lane l
// keeps rows i = l (mod 64) of the block in registers.
constexpr int MAXR = 2048 / 64;

__global__ __launch_bounds__(64) void diag_forward_kernel(Tiles T, int K, double *B, int64_t ldb)
{
    const int b = T.b, lane = threadIdx.x;
    const int vb = (int)min((int64_t)b, T.n - (int64_t)K * b);
    double *y = B + (int64_t)K * b + (int64_t)blockIdx.x * ldb;
    const double *L = (const double *)(T.slots + tile_index(K, K) * T.slot_bytes);
    double v[MAXR];
    const int nr = (vb + 63) / 64;
#pragma unroll
    for (int t = 0; t < MAXR; ++t) v[t] = (t < nr && lane + 64 * t < vb) ? y[lane + 64 * t] : 0.0;
    for (int c = 0; c < vb; ++c) {
        const int owner = c & 63, tc = c >> 6;
        double xc = 0.0;
#pragma unroll
        for (int t = 0; t < MAXR; ++t)
            if (t == tc) xc = v[t];
        xc = __shfl(xc, owner, 64) / L[c + (int64_t)c * b];
        const double *lc = L + (int64_t)c * b;
#pragma unroll
        for (int t = 0; t < MAXR; ++t) {
            int i = lane + 64 * t;
            if (t < nr && i > c && i < vb) v[t] -= lc[i] * xc;
            if (t == tc && lane == owner) v[t] = xc;
        }
    }
#pragma unroll
    for (int t = 0; t < MAXR; ++t)
        if (t < nr && lane + 64 * t < vb) y[lane + 64 * t] = v[t];
}

__global__ __launch_bounds__(64) void diag_backward_kernel(Tiles T, int K, double *B, int64_t ldb)
{
    const int b = T.b, lane = threadIdx.x;
    const int vb = (int)min((int64_t)b, T.n - (int64_t)K * b);
    double *y = B + (int64_t)K * b + (int64_t)blockIdx.x * ldb;
    const double *L = (const double *)(T.slots + tile_index(K, K) * T.slot_bytes);
    double x[MAXR];
    const int nr = (vb + 63) / 64;
#pragma unroll
    for (int t = 0; t < MAXR; ++t) x[t] = 0.0;
    // x_c = (y_c - sum_{i>c} L_ic x_i) / L_cc, c descending
    for (int c = vb - 1; c >= 0; --c) {
        const double *lc = L + (int64_t)c * b;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < MAXR; ++t) {
            int i = lane + 64 * t;
            if (t < nr && i > c && i < vb) s += lc[i] * x[t];
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        const double xc = (y[c] - s) / lc[c];
        const int owner = c & 63, tc = c >> 6;
#pragma unroll
        for (int t = 0; t < MAXR; ++t)
            if (t == tc && lane == owner) x[t] = xc;
    }
#pragma unroll
    for (int t = 0; t < MAXR; ++t)
        if (t < nr && lane + 64 * t < vb) y[lane + 64 * t] = x[t];
}

// B_I -= L_IK X_K for I > K: one thread per row (128 rows per block), 16
// right-hand sides per pass, X_K staged in LDS 128 rows at a time.
__global__ __launch_bounds__(128) void update_forward_kernel(Tiles T, int K, double *B, int64_t ldb, int nrhs)
{
    __shared__ double xs[128][17];
    const int b = T.b, per = b / 128;
    const int I = K + 1 + blockIdx.x / per;
    const int r = (blockIdx.x % per) * 128 + threadIdx.x;
    const int64_t gi = (int64_t)I * b + r;
    const int vk = (int)min((int64_t)b, T.n - (int64_t)K * b);
    const int cls = T.map[I + (int64_t)K * T.nt];
    const int ts = T.tscale[I + (int64_t)K * T.nt];
    const char *tile = T.slots + tile_index(I, K) * T.slot_bytes;
    for (int j0 = 0; j0 < nrhs; j0 += 16) {
        const int nj = min(16, nrhs - j0);
        double acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0;
        for (int c0 = 0; c0 < vk; c0 += 128) {
            __syncthreads();
            for (int e = threadIdx.x; e < 128 * 16; e += 128) {
                int c = e % 128, j = e / 128;
                xs[c][j] = (c0 + c < vk && j < nj) ? B[(int64_t)K * b + c0 + c + (int64_t)(j0 + j) * ldb] : 0.0;
            }
            __syncthreads();
            if (gi < T.n) {
                const int cmax = min(128, vk - c0);
                for (int c = 0; c < cmax; ++c) {
                    double l = load_stored(tile, cls, T.lo16, ts, (int64_t)r + (int64_t)(c0 + c) * b);
#pragma unroll
                    for (int j = 0; j < 16; ++j) acc[j] += l * xs[c][j];
                }
            }
        }
        if (gi < T.n)
            for (int j = 0; j < nj; ++j) B[gi + (int64_t)(j0 + j) * ldb] -= acc[j];
    }
}

// B_J -= L_KJ^T X_K for J < K: a 64-column chunk of tile (K, J) per block,
// staged 64 rows at a time through LDS.
__global__ __launch_bounds__(256) void update_backward_kernel(Tiles T, int K, double *B, int64_t ldb, int nrhs)
{
    __shared__ double ls[64][65];  // ls[c][r]
    __shared__ double xs[64][17];
    const int b = T.b, per = b / 64;
    const int J = blockIdx.x / per;
    const int c0 = (blockIdx.x % per) * 64;
    const int vk = (int)min((int64_t)b, T.n - (int64_t)K * b);
    const int cls = T.map[K + (int64_t)J * T.nt];
    const int ts = T.tscale[K + (int64_t)J * T.nt];
    const char *tile = T.slots + tile_index(K, J) * T.slot_bytes;
    const int col = threadIdx.x & 63, jg = threadIdx.x >> 6;  // 4 groups of 4 rhs
    for (int j0 = 0; j0 < nrhs; j0 += 16) {
        const int nj = min(16, nrhs - j0);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r0 = 0; r0 < vk; r0 += 64) {
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * 64; e += 256) {
                int r = e & 63, c = e >> 6;
                ls[c][r] = (r0 + r < vk) ? load_stored(tile, cls, T.lo16, ts, (int64_t)(r0 + r) + (int64_t)(c0 + c) * b) : 0.0;
            }
            for (int e = threadIdx.x; e < 64 * 16; e += 256) {
                int r = e & 63, j = e >> 6;
                xs[r][j] = (r0 + r < vk && j < nj) ? B[(int64_t)K * b + r0 + r + (int64_t)(j0 + j) * ldb] : 0.0;
            }
            __syncthreads();
            for (int r = 0; r < 64; ++r) {
                double l = ls[col][r];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += l * xs[r][jg * 4 + q];
            }
        }
        const int64_t gj = (int64_t)J * b + c0 + col;
        if (gj < T.n)
            for (int q = 0; q < 4; ++q)
                if (jg * 4 + q < nj) B[gj + (int64_t)(j0 + jg * 4 + q) * ldb] -= acc[q];
    }
}

void launch_solve(const Tiles &T, double *B, int64_t ldb, int nrhs, hipStream_t st)
{
    const int nt = T.nt, b = T.b;
    for (int K = 0; K < nt; ++K) {
        diag_forward_kernel<<<nrhs, 64, 0, st>>>(T, K, B, ldb);
        if (K + 1 < nt) update_forward_kernel<<<(nt - K - 1) * (b / 128), 128, 0, st>>>(T, K, B, ldb, nrhs);
    }
    for (int K = nt - 1; K >= 0; --K) {
        diag_backward_kernel<<<nrhs, 64, 0, st>>>(T, K, B, ldb);
        if (K > 0) update_backward_kernel<<<K * (b / 64), 256, 0, st>>>(T, K, B, ldb, nrhs);
    }
}

}  // namespace mpc
