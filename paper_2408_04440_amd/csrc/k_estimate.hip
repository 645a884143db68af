// Randomized estimate of the backward error ||Sigma - L L^T||_F: for probes
// V with independent N(0,1) entries, E ||E v||^2 = ||E||_F^2 (E symmetric), and
// E V = Sigma V - L (L^T V) costs O(N^2 k) instead of the N^3/3 of the exact
// residual.  Products in FP64 with each stored tile exactly widened; partial
// sums accumulate with FP64 atomics (the order does not matter for an
// estimate).  Buffers have NT*b rows, zero beyond n.
#include "common.h"
#include "launch.h"

namespace mpc {

constexpr int EK = 32;   // probes per pass (columns of V)
constexpr int EB = 64;   // rows / columns of a staged sub-block

__device__ inline double source_ij(const Tiles &T, const Source &S, int64_t i, int64_t j)
{
    if (i >= T.n || j >= T.n) return (i == j) ? 1.0 : 0.0;
    if (S.orig) {
        int64_t a = i >= j ? i : j, c = i >= j ? j : i;  // lower part of the kept copy
        int I = (int)(a / T.b), J = (int)(c / T.b);
        return S.orig[tile_index(I, J) * (int64_t)T.b * T.b + (a % T.b) + (c % T.b) * (int64_t)T.b];
    }
    double v = S.sigma[i] * S.sigma[j] * exp(-fabs(S.x[i] - S.x[j]) / S.rho);
    if (i == j) v += S.nugget;
    return v;
}

// SV[i, q] += sum_{j in chunk} Sigma_ij V[j, q]; one thread per row i, 256 rows
// x 16384 columns per block, V staged 128 rows at a time.
__global__ __launch_bounds__(256) void sigma_v_kernel(Tiles T, Source S, const double *V, int64_t ldv, double *SV)
{
    __shared__ double vs[128][EK + 1];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * 16384;
    const int64_t np = (int64_t)T.nt * T.b;
    double acc[EK];
#pragma unroll
    for (int q = 0; q < EK; ++q) acc[q] = 0.0;
    for (int64_t jc = j0; jc < j0 + 16384 && jc < np; jc += 128) {
        __syncthreads();
        for (int e = threadIdx.x; e < 128 * EK; e += 256) {
            int jj = e % 128, q = e / 128;
            vs[jj][q] = (jc + jj < np) ? V[jc + jj + q * ldv] : 0.0;
        }
        __syncthreads();
        if (i < np) {
            for (int jj = 0; jj < 128 && jc + jj < np; ++jj) {
                double s = source_ij(T, S, i, jc + jj);
#pragma unroll
                for (int q = 0; q < EK; ++q) acc[q] += s * vs[jj][q];
            }
        }
    }
    if (i < np)
#pragma unroll
        for (int q = 0; q < EK; ++q) atomicAdd(SV + i + q * ldv, acc[q]);
}

// Z[rows of I] = sum_{K <= I} L_IK W[rows of K] for one 64-row strip of tile row I.
__global__ __launch_bounds__(256) void l_apply_kernel(Tiles T, const double *W, int64_t ldw, double *Z)
{
    __shared__ double ls[EB][EB + 1];  // ls[c][r]
    __shared__ double ws[EB][EK + 1];
    const int b = T.b, per = b / EB;
    const int I = blockIdx.x / per, r0 = (blockIdx.x % per) * EB;
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;  // 4 groups of 8 probes
    double acc[EK / 4];
#pragma unroll
    for (int q = 0; q < EK / 4; ++q) acc[q] = 0.0;
    for (int K = 0; K <= I; ++K) {
        const int cls = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
        const int ts = T.tscale[I + (int64_t)K * T.nt];
        const char *tile = T.slots + tile_index(I, K) * T.slot_bytes;
        for (int c0 = 0; c0 < b; c0 += EB) {
            __syncthreads();
            for (int e = threadIdx.x; e < EB * EB; e += 256) {
                int rr = e % EB, cc = e / EB;
                ls[cc][rr] = load_stored(tile, cls, T.lo16, ts, (int64_t)(r0 + rr) + (int64_t)(c0 + cc) * b);
            }
            for (int e = threadIdx.x; e < EB * EK; e += 256) {
                int cc = e % EB, q = e / EB;
                ws[cc][q] = W[(int64_t)K * b + c0 + cc + q * ldw];
            }
            __syncthreads();
            for (int cc = 0; cc < EB; ++cc) {
                double l = ls[cc][r];
#pragma unroll
                for (int q = 0; q < EK / 4; ++q) acc[q] += l * ws[cc][g * (EK / 4) + q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < EK / 4; ++q) Z[(int64_t)I * b + r0 + r + (g * (EK / 4) + q) * ldw] = acc[q];
}

// W[rows of K] = sum_{I >= K} L_IK^T V[rows of I] for one 64-column strip of tile column K.
__global__ __launch_bounds__(256) void lt_apply_kernel(Tiles T, const double *V, int64_t ldv, double *W)
{
    __shared__ double ls[EB][EB + 1];  // ls[c][r]
    __shared__ double vs[EB][EK + 1];
    const int b = T.b, per = b / EB;
    const int K = blockIdx.x / per, c0 = (blockIdx.x % per) * EB;
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    double acc[EK / 4];
#pragma unroll
    for (int q = 0; q < EK / 4; ++q) acc[q] = 0.0;
    for (int I = K; I < T.nt; ++I) {
        const int cls = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
        const int ts = T.tscale[I + (int64_t)K * T.nt];
        const char *tile = T.slots + tile_index(I, K) * T.slot_bytes;
        for (int r0 = 0; r0 < b; r0 += EB) {
            __syncthreads();
            for (int e = threadIdx.x; e < EB * EB; e += 256) {
                int rr = e % EB, cc = e / EB;
                ls[cc][rr] = load_stored(tile, cls, T.lo16, ts, (int64_t)(r0 + rr) + (int64_t)(c0 + cc) * b);
            }
            for (int e = threadIdx.x; e < EB * EK; e += 256) {
                int rr = e % EB, q = e / EB;
                vs[rr][q] = V[(int64_t)I * b + r0 + rr + q * ldv];
            }
            __syncthreads();
            for (int rr = 0; rr < EB; ++rr) {
                double l = ls[c][rr];
#pragma unroll
                for (int q = 0; q < EK / 4; ++q) acc[q] += l * vs[rr][g * (EK / 4) + q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < EK / 4; ++q) W[(int64_t)K * b + c0 + c + (g * (EK / 4) + q) * ldv] = acc[q];
}

// Widen FP32 normals to FP64 probes, zero beyond n.
__global__ void probes_kernel(const float *z, int64_t n, int64_t np, double *V)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= np * EK) return;
    const int64_t i = e % np, q = e / np;
    V[e] = (i < n) ? (double)z[i + q * n] : 0.0;
}

// sum over rows < n and probes of (SV - Z)^2, one block, fixed order.
__global__ __launch_bounds__(1024) void residual_norm_kernel(const double *SV, const double *Z, int64_t n, int64_t np,
                                                             double *out)
{
    __shared__ double s[1024];
    double a = 0.0;
    for (int64_t e = threadIdx.x; e < np * EK; e += 1024) {
        int64_t i = e % np;
        if (i < n) {
            double d = SV[e] - Z[e];
            a += d * d;
        }
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// scratch: 3 * NT*b*EK doubles + n*EK floats.  Writes sum ||E v_q||^2 over
// the EK probes to *out (device).
void launch_estimate(const Tiles &T, const Source &S, uint64_t seed, double *scratch, float *zbuf, double *out,
                     hipStream_t st)
{
    const int64_t np = (int64_t)T.nt * T.b;
    double *V = scratch, *SV = scratch + np * EK, *W = scratch + 2 * np * EK, *Z = scratch;  // Z reuses V
    launch_normal_matrix(seed, T.n, EK, zbuf, T.n, st);
    probes_kernel<<<(unsigned)((np * EK + 255) / 256), 256, 0, st>>>(zbuf, T.n, np, V);
    (void)hipMemsetAsync(SV, 0, (size_t)np * EK * 8, st);
    sigma_v_kernel<<<dim3((unsigned)((np + 255) / 256), (unsigned)((np + 16383) / 16384)), 256, 0, st>>>(T, S, V, np, SV);
    const int per = T.b / EB;
    lt_apply_kernel<<<(unsigned)((int64_t)T.nt * per), 256, 0, st>>>(T, V, np, W);
    l_apply_kernel<<<(unsigned)((int64_t)T.nt * per), 256, 0, st>>>(T, W, np, Z);
    residual_norm_kernel<<<1, 1024, 0, st>>>(SV, Z, T.n, np, out);
}

int estimate_probes() { return EK; }

}  // namespace mpc
