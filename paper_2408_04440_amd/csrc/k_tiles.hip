// Tile-level elementwise kernels: covariance generation and loading, tile
// norms, the sender-side conversion of a factored panel, log-determinant
// reduction and factor export.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace mpc {

// Sigma at row r, column c of tile (I, J); identity in the padding beyond n.
__device__ inline double source_value(const Tiles &T, const Source &S, int I, int J, int r, int c)
{
    int64_t i = (int64_t)I * T.b + r, j = (int64_t)J * T.b + c;
    if (i >= T.n || j >= T.n) return (i == j) ? 1.0 : 0.0;
    if (S.dense) return i >= j ? S.dense[i + j * S.ld] : S.dense[j + i * S.ld];
    if (S.orig) return S.orig[tile_index(I, J) * (int64_t)T.b * T.b + r + (int64_t)c * T.b];
    double v = S.sigma[i] * S.sigma[j] * exp(-fabs(S.x[i] - S.x[j]) / S.rho);
    if (i == j) v += S.nugget;
    return v;
}

// Frobenius norm squared and max |.| of the valid part of every lower tile;
// one block per tile, fixed-order reduction (deterministic).
__global__ __launch_bounds__(256) void norms_kernel(Tiles T, Source S, double *fro2, double *amax)
{
    __shared__ double ss[256], sm[256];
    int I, J;
    tile_ij(blockIdx.x, I, J);
    const int b = T.b, tid = threadIdx.x;
    double s = 0.0, m = 0.0;
    const int rmax = (int)min((int64_t)b, T.n - (int64_t)I * b), cmax = (int)min((int64_t)b, T.n - (int64_t)J * b);
    for (int c = 0; c < cmax; ++c)
        for (int r = tid; r < rmax; r += 256) {
            double v = source_value(T, S, I, J, r, c);
            s += v * v;
            m = fmax(m, fabs(v));
        }
    ss[tid] = s;
    sm[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            ss[tid] += ss[tid + w];
            sm[tid] = fmax(sm[tid], sm[tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        fro2[I + (int64_t)J * T.nt] = ss[0];
        amax[I + (int64_t)J * T.nt] = sm[0];
    }
}

// Write Sigma into the work tiles: FP64 for FP64-class and diagonal tiles,
// FP32 (rounded to nearest) for every lower class.
__global__ __launch_bounds__(256) void load_kernel(Tiles T, Source S)
{
    int I, J;
    tile_ij(blockIdx.y, I, J);
    const int b = T.b;
    const int cls = (I == J) ? P64 : T.map[I + (int64_t)J * T.nt];
    char *slot = T.slots + tile_index(I, J) * T.slot_bytes;
    const int64_t bb = (int64_t)b * b;
    for (int64_t e = (int64_t)blockIdx.x * 2048 + threadIdx.x; e < bb && e < (int64_t)(blockIdx.x + 1) * 2048; e += 256) {
        int r = (int)(e % b), c = (int)(e / b);
        double v = source_value(T, S, I, J, r, c);
        if (cls == P64) ((double *)slot)[e] = v;
        else ((float *)slot)[e] = (float)v;
    }
}

// Copy a caller matrix (column-major, lower part read) into FP64 tiles in the
// packed layout; diagonal tiles are filled symmetrically from their lower part.
__global__ __launch_bounds__(256) void copy_matrix_kernel(Tiles T, const double *A, int64_t lda, double *orig)
{
    int I, J;
    tile_ij(blockIdx.y, I, J);
    const int b = T.b;
    const int64_t bb = (int64_t)b * b;
    double *dst = orig + tile_index(I, J) * bb;
    for (int64_t e = (int64_t)blockIdx.x * 2048 + threadIdx.x; e < bb && e < (int64_t)(blockIdx.x + 1) * 2048; e += 256) {
        int r = (int)(e % b), c = (int)(e / b);
        int64_t i = (int64_t)I * b + r, j = (int64_t)J * b + c;
        double v = 0.0;
        if (i < T.n && j < T.n) v = (i >= j) ? A[i + j * lda] : A[j + i * lda];
        dst[e] = v;
    }
}

// Sender-side conversion of step k (one 64 x 64 sub-tile per block).
// The TRSM output X (FP64, in p64[I]) becomes the stored value S of tile
// (I,k) in its class -- FP64: X; FP32: (float)X; 16-bit/FP8: the scaled,
// rounded code of (float)X with t from max|(float)X| -- and every class q
// in qmask[I] gets its copy: FP64 S, FP32 (float)S (or, with the split
// products, its three BF16 parts), 16-bit/FP8 the code of S with the copy's
// own scale (row-major for the 16-bit, 8-bit and split copies).  With
// block-scaled FP8 (lo8 MX) every 32 columns of a row of the FP8 copy take
// their own scale from their own largest |S|, written as the E8M0 byte 127 - t.
__global__ __launch_bounds__(256) void convert_kernel(Tiles T, Panel P, int k, const uint8_t *qmask)
{
    __builtin_amdgcn_s_setprio(3);  // the panel chain: issue ahead of update waves sharing the SIMD
    __shared__ double xs[64][65];  // xs[c][r]
    __shared__ int xt[64][2];      // lo8 MX: scale exponent of row r, 32-column half h of the sub-tile
    const int b = T.b, nsub = b / 64;
    const int I = k + 1 + blockIdx.y;
    const int sr = blockIdx.x % nsub, sc = blockIdx.x / nsub;
    const int64_t bb = (int64_t)b * b;
    const int cls = T.map[I + (int64_t)k * T.nt];
    const int lo16 = T.lo16;
    const uint8_t mask = qmask[I];
    double *x64 = P.p64 + (int64_t)I * bb;
    char *slot = T.slots + tile_index(I, k) * T.slot_bytes;

    const double m = __longlong_as_double((long long)P.pmax[I]);
    int ts = 0;
    double mS = m;
    if (cls == P32) mS = (double)(float)m;
    else if (cls >= P16) {
        double mf = (double)(float)m;
        ts = scale_exp(mf, cls, lo16);
        mS = decode_class(encode_class(mf, cls, lo16, ts), cls, lo16, ts);
    }
    int tq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) tq[q] = scale_exp(mS, q, lo16);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        T.tscale[I + (int64_t)k * T.nt] = ts;
        for (int q = 0; q < 4; ++q) P.pscale[I * 4 + q] = tq[q];
    }

    for (int e = threadIdx.x; e < 4096; e += 256) {
        int r = e & 63, c = e >> 6;
        int64_t off = (int64_t)(sr * 64 + r) + (int64_t)(sc * 64 + c) * b;
        double X = x64[off];
        double Sv;
        if (cls == P64) {
            Sv = X;
            ((double *)slot)[off] = Sv;
        } else if (cls == P32) {
            float f = (float)X;
            Sv = (double)f;
            ((float *)slot)[off] = f;
        } else {
            double xf = (double)(float)X;
            uint32_t code = encode_class(xf, cls, lo16, ts);
            Sv = decode_class(code, cls, lo16, ts);
            if (cls == P16) ((uint16_t *)slot)[off] = (uint16_t)code;
            else ((uint8_t *)slot)[off] = (uint8_t)code;
        }
        xs[c][r] = Sv;
        if (mask & 1) x64[off] = Sv;
        if ((mask & 2) && !T.lo32) P.p32[(int64_t)I * bb + off] = (float)Sv;
    }
    const bool split = (mask & 2) && T.lo32;
    const bool mx = (mask & 8) && T.lo8;
    if ((mask & 12) || split) {
        __syncthreads();
        if (mx) {
            if (threadIdx.x < 128) {
                const int r = threadIdx.x & 63, h = threadIdx.x >> 6;
                double a = 0.0;
                for (int c = 0; c < 32; ++c) a = fmax(a, fabs(xs[h * 32 + c][r]));
                const int t = min(max(scale_exp(a, P8, lo16), -127), 127);  // 0 for an all-zero block
                xt[r][h] = t;
                P.p8x[(int64_t)I * (bb / 32) + (int64_t)(sr * 64 + r) * (b / 32) + sc * 2 + h] = (uint8_t)(127 - t);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < 4096; e += 256) {
            int c = e & 63, r = e >> 6;
            double Sv = xs[c][r];
            int64_t roff = (int64_t)(sr * 64 + r) * b + (sc * 64 + c);
            if (mask & 4) P.p16[(int64_t)I * bb + roff] = (uint16_t)encode_class(Sv, P16, lo16, tq[P16]);
            if (mask & 8)
                P.p8[(int64_t)I * bb + roff] = (uint8_t)encode_class(Sv, P8, lo16, mx ? xt[r][c >> 5] : tq[P8]);
            if (split) {  // FP32 copy as hi + mid + lo, each step exact in FP32
                const float f = (float)Sv;
                const uint16_t hi = f32_to_bf16(f);
                const float r1 = f - bf16_to_f32(hi);
                const uint16_t mid = f32_to_bf16(r1);
                const uint16_t lo = f32_to_bf16(r1 - bf16_to_f32(mid));
                uint16_t *d = P.p32s + (int64_t)I * 3 * bb + roff;
                d[0] = hi;
                d[bb] = mid;
                d[2 * bb] = lo;
            }
        }
    }
}

// 2 * sum_i log L_ii over i < n, one block, fixed-order reduction.
__global__ __launch_bounds__(1024) void logdet_kernel(Tiles T, double *out)
{
    __shared__ double s[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < T.n; i += 1024) {
        int K = (int)(i / T.b), r = (int)(i % T.b);
        const double *d = (const double *)(T.slots + tile_index(K, K) * T.slot_bytes);
        acc += log(d[r + (int64_t)r * T.b]);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = 2.0 * s[0];
}

// Dense copy of the factor's represented values (strict upper part zero).
__global__ __launch_bounds__(256) void get_factor_kernel(Tiles T, double *L, int64_t ldl)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= T.n) return;
    for (int64_t j = blockIdx.y; j < T.n; j += gridDim.y) {
        double v = 0.0;
        if (i >= j) {
            int I = (int)(i / T.b), J = (int)(j / T.b);
            int cls = (I == J) ? P64 : T.map[I + (int64_t)J * T.nt];
            const char *slot = T.slots + tile_index(I, J) * T.slot_bytes;
            v = load_stored(slot, cls, T.lo16, T.tscale[I + (int64_t)J * T.nt], (i % T.b) + (j % T.b) * (int64_t)T.b);
        }
        L[i + j * ldl] = v;
    }
}

__global__ __launch_bounds__(256) void zero_upper_kernel(double *tile, int b)
{
    const int c = blockIdx.x;
    for (int r = threadIdx.x; r < c; r += 256) tile[r + (int64_t)c * b] = 0.0;
}

// ---------------------------------------------------------------- launchers
static inline int64_t ntiles(const Tiles &T) { return (int64_t)T.nt * (T.nt + 1) / 2; }

void launch_norms(const Tiles &T, const Source &S, double *fro2, double *amax, hipStream_t st)
{
    norms_kernel<<<dim3((unsigned)ntiles(T)), 256, 0, st>>>(T, S, fro2, amax);
}

void launch_load(const Tiles &T, const Source &S, hipStream_t st)
{
    int64_t bb = (int64_t)T.b * T.b;
    load_kernel<<<dim3((unsigned)((bb + 2047) / 2048), (unsigned)ntiles(T)), 256, 0, st>>>(T, S);
}

void launch_copy_matrix(const Tiles &T, const double *A, int64_t lda, double *orig, hipStream_t st)
{
    int64_t bb = (int64_t)T.b * T.b;
    copy_matrix_kernel<<<dim3((unsigned)((bb + 2047) / 2048), (unsigned)ntiles(T)), 256, 0, st>>>(T, A, lda, orig);
}

void launch_convert(const Tiles &T, const Panel &P, int k, const uint8_t *qmask, hipStream_t st)
{
    int np = T.nt - k - 1;
    if (np <= 0) return;
    int nsub = T.b / 64;
    convert_kernel<<<dim3(nsub * nsub, np), 256, 0, st>>>(T, P, k, qmask);
}

void launch_logdet(const Tiles &T, double *out, hipStream_t st) { logdet_kernel<<<1, 1024, 0, st>>>(T, out); }

void launch_get_factor(const Tiles &T, double *L, int64_t ldl, hipStream_t st)
{
    get_factor_kernel<<<dim3((unsigned)((T.n + 255) / 256), (unsigned)std::min<int64_t>(T.n, 4096)), 256, 0, st>>>(T, L, ldl);
}

void launch_zero_upper_diag(const Tiles &T, int k, hipStream_t st)
{
    double *tile = (double *)(T.slots + tile_index(k, k) * T.slot_bytes);
    zero_upper_kernel<<<T.b, 256, 0, st>>>(tile, T.b);
}

}  // namespace mpc
