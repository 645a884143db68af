// Randomized estimate of the backward error ||Sigma - L L^T||_F: for probes
// V with independent N(0,1) entries, E ||E v||^2 = ||E||_F^2 (E symmetric), and
// E V = Sigma V - L (L^T V) costs O(N^2 k) instead of the N^3/3 of the exact
// residual.  Every stored tile is widened exactly to FP64 and read once per
// product; the products run on the FP64 MFMA.  Buffers have NT*b rows,
// identity beyond n.
//
// Sigma V for the generator with nondecreasing coordinates uses the
// exponential kernel's separability: with u_j = sigma_j v_j and
// d_i = exp(-(x_i - x_{i-1})/rho),
//   F_i = sum_{j<=i} e^{-(x_i-x_j)/rho} u_j = d_i F_{i-1} + u_i,
//   H_i = sum_{j>=i} e^{-(x_j-x_i)/rho} u_j = d_{i+1} H_{i+1} + u_i,
//   (Sigma v)_i = sigma_i (F_i + H_i - u_i) + nugget v_i,
// evaluated as a chunked scan (local recursions, chunk carries, combination).
// Otherwise (an explicit matrix, or unsorted coordinates) Sigma V is the
// dense product with Sigma regenerated or read from the kept copy.
#include "common.h"
#include "gemm_core.h"
#include "launch.h"

namespace mpc {

constexpr int EK = 64;   // probes per pass (columns of V)
constexpr int EB = 64;   // rows / columns of an output block
constexpr int ER = 32;   // K rows staged per step
constexpr int SC = 256;  // rows per scan chunk

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

// ---------------------------------------------------------------- dense Sigma V
// SV[i, q0+q] += sum_{j in chunk} Sigma_ij V[j, q0+q] for 32 probes; one
// thread per row i, 256 rows x 16384 columns per block, V staged 128 rows at
// a time.
constexpr int DQ = 32;
__global__ __launch_bounds__(256) void sigma_v_kernel(Tiles T, Source S, const double *V, int64_t ldv, double *SV)
{
    __shared__ double vs[128][DQ + 1];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * 16384;
    const int64_t np = (int64_t)T.nt * T.b;
    double acc[DQ];
#pragma unroll
    for (int q = 0; q < DQ; ++q) acc[q] = 0.0;
    for (int64_t jc = j0; jc < j0 + 16384 && jc < np; jc += 128) {
        __syncthreads();
        for (int e = threadIdx.x; e < 128 * DQ; e += 256) {
            int jj = e % 128, q = e / 128;
            vs[jj][q] = (jc + jj < np) ? V[jc + jj + q * ldv] : 0.0;
        }
        __syncthreads();
        if (i < np) {
            for (int jj = 0; jj < 128 && jc + jj < np; ++jj) {
                double s = source_ij(T, S, i, jc + jj);
#pragma unroll
                for (int q = 0; q < DQ; ++q) acc[q] += s * vs[jj][q];
            }
        }
    }
    if (i < np)
#pragma unroll
        for (int q = 0; q < DQ; ++q) atomicAdd(SV + i + q * ldv, acc[q]);
}

// ---------------------------------------------------------------- scan Sigma V
// Local recursions of chunk c for probe q (rows s .. e, e < n):
//   f_i = d_i f_{i-1} + u_i (f_{s-1} = 0)   -> F buffer,
//   h_i = d_{i+1} h_{i+1} + u_i (h_{e+1} = 0) -> H buffer.
__global__ __launch_bounds__(64) void scan_local_kernel(Tiles T, Source S, const double *V, int64_t ldv, double *F,
                                                        double *H)
{
    const int c = blockIdx.x, q = threadIdx.x;
    const int64_t s = (int64_t)c * SC, e = min((int64_t)T.n, s + SC) - 1;
    const double *v = V + q * ldv;
    double f = 0.0;
    for (int64_t i = s; i <= e; ++i) {
        const double d = (i > s) ? exp(-(S.x[i] - S.x[i - 1]) / S.rho) : 0.0;
        f = d * f + S.sigma[i] * v[i];
        F[i + q * ldv] = f;
    }
    double h = 0.0;
    for (int64_t i = e; i >= s; --i) {
        const double d = (i < e) ? exp(-(S.x[i + 1] - S.x[i]) / S.rho) : 0.0;
        h = d * h + S.sigma[i] * v[i];
        H[i + q * ldv] = h;
    }
}

// Chunk carries for probe q: Fin[c] = F_{s_c - 1}, Hin[c] = H_{e_c + 1} (0
// at the ends), from the chunk-boundary values of the local recursions.
__global__ __launch_bounds__(64) void scan_carry_kernel(Tiles T, Source S, const double *F, const double *H,
                                                        int64_t ldv, int nchunk, double *Fin, double *Hin)
{
    const int q = threadIdx.x;
    double carry = 0.0;  // F at the last row of the previous chunk
    for (int c = 0; c < nchunk; ++c) {
        const int64_t s = (int64_t)c * SC, e = min((int64_t)T.n, s + SC) - 1;
        Fin[c * EK + q] = carry;
        const double dc = (c > 0) ? exp(-(S.x[e] - S.x[s - 1]) / S.rho) : 0.0;
        carry = F[e + q * ldv] + dc * carry;
    }
    carry = 0.0;  // H at the first row of the next chunk
    for (int c = nchunk - 1; c >= 0; --c) {
        const int64_t s = (int64_t)c * SC, e = min((int64_t)T.n, s + SC) - 1;
        Hin[c * EK + q] = carry;
        const double dc = (c < nchunk - 1) ? exp(-(S.x[e + 1] - S.x[s]) / S.rho) : 0.0;
        carry = H[s + q * ldv] + dc * carry;
    }
}

// SV_i = sigma_i (F_i + H_i - u_i) + nugget v_i with the carries applied;
// rows >= n are the identity's.  F may alias SV (each element read, then written).
__global__ __launch_bounds__(256) void scan_finish_kernel(Tiles T, Source S, const double *V, int64_t ldv,
                                                          const double *F, const double *H, const double *Fin,
                                                          const double *Hin, double *SV)
{
    const int64_t np = (int64_t)T.nt * T.b;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= np * EK) return;
    const int64_t i = e % np;
    const int q = (int)(e / np);
    const double v = V[i + q * ldv];
    if (i >= T.n) {
        SV[i + q * ldv] = v;
        return;
    }
    const int c = (int)(i / SC);
    const int64_t s = (int64_t)c * SC, ce = min((int64_t)T.n, s + SC) - 1;
    double Fi = F[i + q * ldv], Hi = H[i + q * ldv];
    if (c > 0) Fi += exp(-(S.x[i] - S.x[s - 1]) / S.rho) * Fin[c * EK + q];
    if (ce + 1 < T.n) Hi += exp(-(S.x[ce + 1] - S.x[i]) / S.rho) * Hin[c * EK + q];
    const double u = S.sigma[i] * v;
    SV[i + q * ldv] = S.sigma[i] * (Fi + Hi - u) + S.nugget * v;
}

// ---------------------------------------------------------------- L^T V, L W
// Both products walk a tile column (row) of the stored factor in steps of ER
// rows (columns) of K: each step's piece of L (widened to FP64) and of the
// probes is read into registers while the previous step is multiplied from
// LDS, then written to LDS once every wave is done with it (one LDS buffer,
// which leaves room for four blocks per compute unit).
constexpr int EPT = ER * EB / 256;  // elements of the L piece per thread
constexpr int QPT = ER * EK / 256;  // elements of the probe piece per thread
static_assert(ER * EB % 256 == 0 && ER * EK % 256 == 0, "staging split");

// The 2 x 2 MFMA tiles of a wave: acc[m][n] += B-piece(n)^T-ish products over
// the ER rows of one staged step, with swapped operands (lane gi owns output
// row c of the 32 x 32 wave tile, element v the probe acc_row(gg, v)).
__device__ inline void apply_step(const double (*ls)[EB + 1], const double (*vs)[EK + 1], int wm, int wn, int gi,
                                  int gg, double4_t (&acc)[2][2])
{
#pragma unroll
    for (int s = 0; s < ER / 4; ++s) {
        double fa[2], fb[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) fa[m] = ls[s * 4 + gg][wm * 32 + m * 16 + gi];
#pragma unroll
        for (int n = 0; n < 2; ++n) fb[n] = vs[s * 4 + gg][wn * 32 + n * 16 + gi];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[n], fa[m], acc[m][n], 0, 0, 0);
    }
}

// W[rows c0.. of tile column K] = sum_{I >= K} L_IK(:, c0:c0+64)^T V[rows of I]:
// block per (K, 64-column strip), four waves of 32 x 32 outputs (c x probe),
// K dimension = the rows r of L_IK, ER at a time.
__global__ __launch_bounds__(256) void lt_apply_kernel(Tiles T, const double *V, int64_t ldv, double *W)
{
    __shared__ double ls[ER][EB + 1];  // ls[r][c] = L_IK(r0 + r, c0 + c)
    __shared__ double vs[ER][EK + 1];  // vs[r][q] = V[I*b + r0 + r, q]
    const int b = T.b, per = b / EB, nrs = b / ER;
    const int K = blockIdx.x / per, c0 = (blockIdx.x % per) * EB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % 2, wn = wave / 2, gi = lane & 15, gg = lane >> 4;
    double4_t acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = (double4_t){0.0, 0.0, 0.0, 0.0};
    double lr[EPT], vr[QPT];
    auto fetch = [&](int st) {  // step st: tile I = K + st / nrs, rows r0 = (st % nrs) * ER
        const int I = K + st / nrs, r0 = (st % nrs) * ER;
        const int cls = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
        const int ts = T.tscale[I + (int64_t)K * T.nt];
        const char *tile = T.slots + tile_index(I, K) * T.slot_bytes;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j, r = e % ER, c = e / ER;
            lr[j] = load_stored(tile, cls, T.lo16, ts, (int64_t)(r0 + r) + (int64_t)(c0 + c) * b);
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int e = tid + 256 * j, r = e % ER, q = e / ER;
            vr[j] = V[(int64_t)I * b + r0 + r + q * ldv];
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j;
            ls[e % ER][e / ER] = lr[j];
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int e = tid + 256 * j;
            vs[e % ER][e / ER] = vr[j];
        }
    };
    const int nsteps = (T.nt - K) * nrs;
    fetch(0);
    put();
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        if (st + 1 < nsteps) fetch(st + 1);
        apply_step(ls, vs, wm, wn, gi, gg, acc);
        __syncthreads();
        if (st + 1 < nsteps) {
            put();
            __syncthreads();
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = wm * 32 + m * 16 + gi, q = wn * 32 + n * 16 + acc_row<double>(gg, v);
                W[(int64_t)K * b + c0 + c + q * ldv] = acc[m][n][v];
            }
}

// Z[rows r0.. of tile row I] = sum_{K <= I} L_IK(r0:r0+64, :) W[rows of K]:
// block per (I, 64-row strip), K dimension = the columns of L_IK, ER at a time.
// The last tile rows, with the most tiles to walk, take the first blocks so
// that the longest blocks start first.
__global__ __launch_bounds__(256) void l_apply_kernel(Tiles T, const double *W, int64_t ldw, double *Z)
{
    __shared__ double ls[ER][EB + 1];  // ls[c][r] = L_IK(r0 + r, c0 + c)
    __shared__ double ws[ER][EK + 1];  // ws[c][q] = W[K*b + c0 + c, q]
    const int b = T.b, per = b / EB, nrs = b / ER;
    const int I = T.nt - 1 - (int)(blockIdx.x / per), r0 = (blockIdx.x % per) * EB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % 2, wn = wave / 2, gi = lane & 15, gg = lane >> 4;
    double4_t acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = (double4_t){0.0, 0.0, 0.0, 0.0};
    double lr[EPT], wr[QPT];
    auto fetch = [&](int st) {  // step st: tile K = st / nrs, columns c0 = (st % nrs) * ER
        const int K = st / nrs, c0 = (st % nrs) * ER;
        const int cls = (I == K) ? P64 : T.map[I + (int64_t)K * T.nt];
        const int ts = T.tscale[I + (int64_t)K * T.nt];
        const char *tile = T.slots + tile_index(I, K) * T.slot_bytes;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j, r = e % EB, c = e / EB;
            lr[j] = load_stored(tile, cls, T.lo16, ts, (int64_t)(r0 + r) + (int64_t)(c0 + c) * b);
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int e = tid + 256 * j, c = e % ER, q = e / ER;
            wr[j] = W[(int64_t)K * b + c0 + c + q * ldw];
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j;
            ls[e / EB][e % EB] = lr[j];
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int e = tid + 256 * j;
            ws[e % ER][e / ER] = wr[j];
        }
    };
    const int nsteps = (I + 1) * nrs;
    fetch(0);
    put();
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        if (st + 1 < nsteps) fetch(st + 1);
        apply_step(ls, ws, wm, wn, gi, gg, acc);
        __syncthreads();
        if (st + 1 < nsteps) {
            put();
            __syncthreads();
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wm * 32 + m * 16 + gi, q = wn * 32 + n * 16 + acc_row<double>(gg, v);
                Z[(int64_t)I * b + r0 + r + q * ldw] = acc[m][n][v];
            }
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

int estimate_chunks(int64_t n) { return (int)((n + SC - 1) / SC); }

// scratch: 3 * NT*b*EK doubles + 2 * chunks*EK doubles; zbuf: n*EK floats.
// Writes sum ||E v_q||^2 over the EK probes to *out (device).  sorted: the
// generator's coordinates are nondecreasing (scan path for Sigma V).
void launch_estimate(const Tiles &T, const Source &S, bool sorted, uint64_t seed, double *scratch, float *zbuf,
                     double *out, hipStream_t st)
{
    const int64_t np = (int64_t)T.nt * T.b;
    double *V = scratch, *SV = scratch + np * EK, *W = scratch + 2 * np * EK, *Z = scratch;  // Z reuses V
    double *Fin = scratch + 3 * np * EK, *Hin = Fin + (int64_t)estimate_chunks(T.n) * EK;
    launch_normal_matrix(seed, T.n, EK, zbuf, T.n, st);
    const unsigned eb = (unsigned)((np * EK + 255) / 256);
    probes_kernel<<<eb, 256, 0, st>>>(zbuf, T.n, np, V);
    if (sorted && !S.orig) {
        const int nc = estimate_chunks(T.n);
        scan_local_kernel<<<nc, EK, 0, st>>>(T, S, V, np, SV, W);  // F -> SV, H -> W
        scan_carry_kernel<<<1, EK, 0, st>>>(T, S, SV, W, np, nc, Fin, Hin);
        scan_finish_kernel<<<eb, 256, 0, st>>>(T, S, V, np, SV, W, Fin, Hin, SV);
    } else {
        (void)hipMemsetAsync(SV, 0, (size_t)np * EK * 8, st);
        const dim3 g((unsigned)((np + 255) / 256), (unsigned)((np + 16383) / 16384));
        for (int q0 = 0; q0 < EK; q0 += DQ) sigma_v_kernel<<<g, 256, 0, st>>>(T, S, V + q0 * np, np, SV + q0 * np);
    }
    const int per = T.b / EB;
    lt_apply_kernel<<<(unsigned)((int64_t)T.nt * per), 256, 0, st>>>(T, V, np, W);
    l_apply_kernel<<<(unsigned)((int64_t)T.nt * per), 256, 0, st>>>(T, W, np, Z);
    residual_norm_kernel<<<1, 1024, 0, st>>>(SV, Z, T.n, np, out);
}

int estimate_probes() { return EK; }

}  // namespace mpc
