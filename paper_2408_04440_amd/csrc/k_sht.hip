// Spherical harmonic transform of fields on an equiangular grid (Sec. III.A.1,
// "Modeling in the Spherical Harmonic Domain"; the precomputation of
// Sec. III.A.2) and its inverse, used to turn emulated coefficient vectors
// back into fields (Sec. III.B), batched over time steps, and the C ABI of the
// transform object (include/mpchol.h).
//
// The paper's route, kept: G_m(theta_j) by FFT along longitude; G_m extended to
// colatitudes in (pi, 2 pi) with G_m(2 pi - theta) = (-1)^m G_m(theta) and an
// FFT along the extended colatitude gives K_{m,m'}; the coefficients follow
// from K through Wigner-d functions at pi/2, which are precomputed by a
// three-term recursion.  What is arranged differently for the GPU:
//   * the paper's two sums (over m' with I(m' + m'') and over m'' with
//     S_{l,m,m''}) are folded into one precomputed real table per order m,
//     using K_{m,-m'} = (-1)^m K_{m,m'} (so only m' >= 0 is kept), the
//     cancellation of the q = +-1 terms of I(q) under that symmetry, and the
//     parity structure d^l_{m'',0}(pi/2) = 0 for l + m'' odd (rows of degree l
//     only meet columns m' of the same parity).  Per order m and parity p the
//     forward transform is then a real GEMM
//         C[l, c] = sum_{m' = p mod 2} W^{m,p}[l, m'] Kr[m', c],
//     with the real and imaginary parts of K of all time steps as the columns
//     c (Re in c = t, Im in c = Tpad + t) and z_{l,m} = i^-m (C[l,t] + i C[l,Tpad+t]);
//   * the inverse uses the same parity blocks of
//     K_{m,m'} = 2 pi i^-m sum_l c_l d^l_{m',0} d^l_{m',m} z_{l,m};
//   * both GEMMs run on the FP64 MFMA block core shared with the
//     factorization; FFTs are in-place Stockham passes (radix 2, 3, 4, 5) in
//     LDS, several sequences per workgroup, real fields two rows per complex
//     sequence.
// Readings (the grid, the 1/2pi of the longitude synthesis, the real layout
// of the coefficient vector) are stated with the declarations in mpchol.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mpchol.h"
#include "common.h"
#include "gemm_core.h"

namespace mpc {
namespace sht {

constexpr int NTH = 256;   // threads of an FFT workgroup
constexpr int MAXV = 16;   // complex values per thread and pass: nseq * n <= NTH * MAXV
constexpr int MAXP = 16;   // passes of a plan
constexpr int MAXN = 4096; // longest transform
constexpr int MAXL = 1024; // band limit (2^-l of the edge value stays a normal double)

struct Plan {
    int n, np;
    int r[MAXP];
};

// GEMM block shape (FP64 MFMA, operands swapped so that column-major stores coalesce)
constexpr int GBM = 64, GBN = 128, GBK = 16, GWM = 2, GWN = 2;
typedef CMShape<double, GBM, GBN, GBK, GWM, GWN> GS;

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by i^e, e in 0..3
__device__ inline double2 ipow(double2 a, int e)
{
    switch (e & 3) {
    case 1: return make_double2(-a.y, a.x);
    case 2: return make_double2(-a.x, -a.y);
    case 3: return make_double2(a.y, -a.x);
    default: return a;
    }
}

// R-point DFT in place: V[q] = sum_r v[r] w^{q r}, w = e^{-2 pi i / R} (forward)
// or its conjugate (inverse); tw holds e^{-2 pi i k / n} for the transform length n.
template <int R>
__device__ inline void dft_small(double2 (&v)[R], const double2 *tw, int n, bool inv)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        double2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
        // w = -i forward, +i inverse
        double2 wd = inv ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, wd);
        v[3] = csub(d02, wd);
    } else {
        double2 in[R];
#pragma unroll
        for (int r = 0; r < R; ++r) in[r] = v[r];
        const int st = n / R;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double2 acc = in[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double2 w = tw[((q * r) % R) * st];
                if (inv) w.y = -w.y;
                acc = cadd(acc, cmul(in[r], w));
            }
            v[q] = acc;
        }
    }
}

// One Stockham pass of radix R over nseq sequences of length n held
// contiguously in LDS (in place: every butterfly reads its inputs before a
// barrier and writes its outputs after it).  Ns = product of earlier radices.
template <int R>
__device__ inline void fft_pass(double2 *buf, int nseq, int n, int Ns, const double2 *tw, bool inv)
{
    constexpr int MB = (MAXV + R - 1) / R;
    const int nb = n / R, total = nseq * nb;
    double2 v[MB][R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int idx = threadIdx.x + i * NTH;
        if (idx < total) {
            const int s = idx / nb, j = idx - s * nb;
            const double2 *src = buf + s * n + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[r * nb];
        }
    }
    __syncthreads();
    const int stride = n / (Ns * R);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int idx = threadIdx.x + i * NTH;
        if (idx < total) {
            const int s = idx / nb, j = idx - s * nb;
            const int k = j % Ns, step = k * stride;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double2 w = tw[r * step];
                if (inv) w.y = -w.y;
                v[i][r] = cmul(v[i][r], w);
            }
            dft_small<R>(v[i], tw, n, inv);
            double2 *dst = buf + s * n + (j / Ns) * Ns * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[q * Ns] = v[i][q];
        }
    }
    __syncthreads();
}

// X[k] = sum_j x[j] e^{-+2 pi i jk/n} for nseq sequences in LDS (no scaling).
__device__ inline void fft_run(double2 *buf, int nseq, const Plan &P, const double2 *tw, bool inv)
{
    int Ns = 1;
    for (int p = 0; p < P.np; ++p) {
        const int R = P.r[p];
        if (R == 4) fft_pass<4>(buf, nseq, P.n, Ns, tw, inv);
        else if (R == 2) fft_pass<2>(buf, nseq, P.n, Ns, tw, inv);
        else if (R == 3) fft_pass<3>(buf, nseq, P.n, Ns, tw, inv);
        else fft_pass<5>(buf, nseq, P.n, Ns, tw, inv);
        Ns *= R;
    }
}

__device__ inline void load_twiddles(double2 *tws, const double2 *twg, int n)
{
    for (int i = threadIdx.x; i < n; i += NTH) tws[i] = twg[i];
}

// ------------------------------------------------------------------ longitude
// Forward: rows q = t * ntheta + j of Z (nphi doubles each), two rows per
// complex sequence; G[(t L + m) ntheta + j] = (2 pi / nphi) sum_k Z e^{-i m phi_k}
// for m = 0..L-1.
__global__ __launch_bounds__(NTH) void phi_forward_kernel(const double *__restrict__ Z, int64_t rows, int ntheta,
                                                          int L, Plan P, const double2 *__restrict__ twg,
                                                          double2 *__restrict__ G, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int n = P.n;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + n;
    load_twiddles(tws, twg, n);
    const int64_t q0 = (int64_t)blockIdx.x * 2 * nseq;
    for (int idx = threadIdx.x; idx < nseq * n; idx += NTH) {
        const int s = idx / n, k = idx - s * n;
        const int64_t qa = q0 + 2 * s, qb = qa + 1;
        const double a = qa < rows ? Z[qa * n + k] : 0.0;
        const double b = qb < rows ? Z[qb * n + k] : 0.0;
        buf[idx] = make_double2(a, b);
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, false);
    const double sc = 2.0 * M_PI / n;
    const int nrow = 2 * nseq;
    for (int idx = threadIdx.x; idx < nrow * L; idx += NTH) {
        const int rr = idx % nrow, m = idx / nrow;
        const int64_t q = q0 + rr;
        if (q >= rows) continue;
        const int s = rr >> 1;
        const double2 X = buf[s * n + (m % n)], Y = buf[s * n + ((n - m % n) % n)];
        double2 val;
        if ((rr & 1) == 0) val = make_double2(0.5 * (X.x + Y.x), 0.5 * (X.y - Y.y));  // (X + conj Y) / 2
        else val = make_double2(0.5 * (X.y + Y.y), -0.5 * (X.x - Y.x));              // (X - conj Y) / 2i
        const int64_t t = q / ntheta, j = q - t * ntheta;
        G[(t * L + m) * ntheta + j] = cscale(val, sc);
    }
}

// Inverse: Z(theta_j, phi_k) = (1 / 2 pi) sum_{|m| < L} G_m(theta_j) e^{i m phi_k},
// G_{-m} = conj(G_m); two rows per complex sequence (their spectra are
// Hermitian, so the real and imaginary parts of one inverse FFT separate them).
__global__ __launch_bounds__(NTH) void phi_inverse_kernel(const double2 *__restrict__ G, int64_t rows, int ntheta,
                                                          int L, Plan P, const double2 *__restrict__ twg,
                                                          double *__restrict__ Z, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int n = P.n;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + n;
    load_twiddles(tws, twg, n);
    for (int idx = threadIdx.x; idx < nseq * n; idx += NTH) buf[idx] = make_double2(0.0, 0.0);
    __syncthreads();
    const int64_t q0 = (int64_t)blockIdx.x * 2 * nseq;
    const double sc = 1.0 / (2.0 * M_PI);
    for (int idx = threadIdx.x; idx < nseq * L; idx += NTH) {
        const int s = idx % nseq, m = idx / nseq;
        const int64_t qa = q0 + 2 * s, qb = qa + 1;
        double2 ga = make_double2(0.0, 0.0), gb = ga;
        if (qa < rows) {
            const int64_t t = qa / ntheta, j = qa - t * ntheta;
            ga = cscale(G[(t * L + m) * ntheta + j], sc);
        }
        if (qb < rows) {
            const int64_t t = qb / ntheta, j = qb - t * ntheta;
            gb = cscale(G[(t * L + m) * ntheta + j], sc);
        }
        if (m == 0) {  // G_0 of a real field is real
            buf[s * n] = make_double2(ga.x, gb.x);
        } else {
            buf[s * n + m] = make_double2(ga.x - gb.y, ga.y + gb.x);          // ga + i gb
            buf[s * n + n - m] = make_double2(ga.x + gb.y, -ga.y + gb.x);     // conj(ga) + i conj(gb)
        }
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, true);
    for (int idx = threadIdx.x; idx < nseq * n; idx += NTH) {
        const int s = idx / n, k = idx - s * n;
        const int64_t qa = q0 + 2 * s, qb = qa + 1;
        const double2 v = buf[idx];
        if (qa < rows) Z[qa * n + k] = v.x;
        if (qb < rows) Z[qb * n + k] = v.y;
    }
}

// ------------------------------------------------------------------ colatitude
struct Blocks {
    const int64_t *off;  // per (m, p): offset of the block
    int64_t ld;          // leading dimension
};

// Forward: for order m = blockIdx.y and nseq time steps, extend G_m to the
// M = 2 ntheta - 2 colatitudes 2 pi j / M with the parity (-1)^m (pole samples
// of odd orders taken as zero, the value that parity forces), FFT, and
// store K_{m,m'} / M for m' = 0..L-1 as GEMM operand rows: block (m, m' mod 2),
// row m' / 2, columns t (real part) and Tpad + t (imaginary part).
__global__ __launch_bounds__(NTH) void theta_forward_kernel(const double2 *__restrict__ G, int T, int ntheta, int L,
                                                            Plan P, const double2 *__restrict__ twg, double *B,
                                                            Blocks Bb, int Tpad, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int M = P.n;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + M;
    load_twiddles(tws, twg, M);
    const int m = blockIdx.y;
    const int t0 = blockIdx.x * nseq;
    const double par = (m & 1) ? -1.0 : 1.0;
    for (int idx = threadIdx.x; idx < nseq * M; idx += NTH) {
        const int s = idx / M, j = idx - s * M;
        const int t = t0 + s;
        double2 v = make_double2(0.0, 0.0);
        // odd orders vanish at the poles (the extension's symmetry forces it)
        const bool pole = (j == 0 || j == ntheta - 1) && (m & 1);
        if (t < T && !pole) {
            if (j < ntheta) v = G[((int64_t)t * L + m) * ntheta + j];
            else v = cscale(G[((int64_t)t * L + m) * ntheta + (M - j)], par);
        }
        buf[idx] = v;
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, false);
    const double sc = 1.0 / M;
    for (int idx = threadIdx.x; idx < nseq * L; idx += NTH) {
        const int s = idx % nseq, mp = idx / nseq;
        const int t = t0 + s;
        if (t >= T) continue;
        const double2 K = cscale(buf[s * M + mp], sc);
        double *row = B + Bb.off[2 * m + (mp & 1)] + (int64_t)(mp >> 1) * Bb.ld;
        row[t] = K.x;
        row[Tpad + t] = K.y;
    }
}

// Inverse: K_{m,m'} = i^-m (C[m'][t] + i C[m'][Tpad + t]) from the inverse GEMM's
// column-major blocks, K_{m,-m'} = (-1)^m K_{m,m'}; G_m(theta_j) = sum_m' K e^{i m' theta_j}
// by an inverse FFT over the M extended colatitudes, kept for j < ntheta.
__global__ __launch_bounds__(NTH) void theta_inverse_kernel(const double *__restrict__ Cinv, Blocks Cb,
                                                            const int *__restrict__ cld, int T, int ntheta, int L,
                                                            Plan P, const double2 *__restrict__ twg,
                                                            double2 *__restrict__ G, int Tpad, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int M = P.n;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + M;
    load_twiddles(tws, twg, M);
    for (int idx = threadIdx.x; idx < nseq * M; idx += NTH) buf[idx] = make_double2(0.0, 0.0);
    __syncthreads();
    const int m = blockIdx.y;
    const int t0 = blockIdx.x * nseq;
    const double par = (m & 1) ? -1.0 : 1.0;
    for (int idx = threadIdx.x; idx < nseq * L; idx += NTH) {
        const int s = idx / L, mp = idx - s * L;
        const int t = t0 + s;
        if (t >= T) continue;
        const int p = mp & 1;
        const double *c = Cinv + Cb.off[2 * m + p] + (mp >> 1);
        const int64_t ld = cld[2 * m + p];
        const double2 K = ipow(make_double2(c[(int64_t)t * ld], c[(int64_t)(Tpad + t) * ld]), (4 - (m & 3)) & 3);
        buf[s * M + mp] = K;
        if (mp > 0) buf[s * M + M - mp] = cscale(K, par);
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, true);
    for (int idx = threadIdx.x; idx < nseq * ntheta; idx += NTH) {
        const int s = idx / ntheta, j = idx - s * ntheta;
        const int t = t0 + s;
        if (t < T) G[((int64_t)t * L + m) * ntheta + j] = buf[s * M + j];
    }
}

// ------------------------------------------------------------------ contraction
__host__ __device__ inline int lstart(int m, int p) { return ((m & 1) == p) ? m : m + 1; }

struct Item {
    int16_t m, p;
    int32_t tm;
};

// Forward GEMM per (m, p, row block): C = W^{m,p} Kr^{m,p}; the epilogue rotates
// by i^-m and writes the real layout f[t L^2 + l^2 + l +- m].
__global__ __launch_bounds__(GS::NTH) void gemm_forward_kernel(const double *__restrict__ W, Blocks Wb,
                                                               const int *__restrict__ wrows,
                                                               const double *__restrict__ B, Blocks Bb,
                                                               const int *__restrict__ kpad,
                                                               const Item *__restrict__ items, int L, int T, int Tpad,
                                                               double *__restrict__ f)
{
    extern __shared__ __align__(16) char smem_raw[];
    const Item it = items[blockIdx.x];
    const int m = it.m, p = it.p, mp2 = 2 * m + p;
    const int tn = blockIdx.y;
    double4_t acc[GS::MB][GS::NB];
#pragma unroll
    for (int a = 0; a < GS::MB; ++a)
#pragma unroll
        for (int b = 0; b < GS::NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
    const int lda = wrows[mp2];
    cm_block<double, GBM, GBN, GBK, GWM, GWN, true>(W + Wb.off[mp2] + it.tm * GBM, lda,
                                                    B + Bb.off[mp2] + tn * GBN, Bb.ld, kpad[p], acc,
                                                    (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % GWM, wn = wave / GWM, gi = lane & 15, gg = lane >> 4;
    const int l0 = lstart(m, p);
    const int64_t LL = (int64_t)L * L;
    const int rot = m & 3;
    const double s2 = m > 0 ? M_SQRT2 : 1.0;
#pragma unroll
    for (int a = 0; a < GS::MB; ++a) {
        const int r = it.tm * GBM + wm * (GBM / GWM) + a * 16 + gi;
        const int l = l0 + 2 * r;
        if (l >= L) continue;
        const int64_t base = (int64_t)l * l + l;
#pragma unroll
        for (int b = 0; b < GS::NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = tn * GBN + wn * (GBN / GWN) + b * 16 + acc_row<double>(gg, v);
                const int part = c >= Tpad;
                const int t = part ? c - Tpad : c;
                if (t >= T) continue;
                double val = acc[a][b][v] * s2;
                if (m == 0) {
                    if (!part) f[t * LL + base] = val;
                    continue;
                }
                // z = i^-m (a + i b): Re z and Im z are each +- one of a, b
                bool re;
                if (!part) {
                    re = (rot == 0 || rot == 2);
                    if (rot == 1 || rot == 2) val = -val;
                } else {
                    re = (rot == 1 || rot == 3);
                    if (rot == 2 || rot == 3) val = -val;
                }
                f[t * LL + base + (re ? m : -m)] = val;
            }
    }
}

// Inverse operand: Bz^{m,p}[row (l - lstart) / 2][t] = Re z_{l,m}, [Tpad + t] = Im z_{l,m}
// from the real layout (one thread per coefficient of one time step).
__global__ void pack_inverse_kernel(const double *__restrict__ f, int T, int L, double *Bz, Blocks Zb, int Tpad)
{
    const int64_t LL = (int64_t)L * L;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= LL * T) return;
    const int t = (int)(g / LL);
    const int idx = (int)(g - (int64_t)t * LL);
    int l = (int)sqrt((double)idx);
    while (l * l > idx) --l;
    while ((l + 1) * (l + 1) <= idx) ++l;
    const int ms = idx - l * l - l;
    const int m = ms < 0 ? -ms : ms, p = l & 1;
    const int r = (l - lstart(m, p)) >> 1;
    double *row = Bz + Zb.off[2 * m + p] + (int64_t)r * Zb.ld;
    const double v = f[g];
    if (ms == 0) {
        row[t] = v;
        row[Tpad + t] = 0.0;
    } else if (ms > 0) {
        row[t] = v * M_SQRT1_2;
    } else {
        row[Tpad + t] = v * M_SQRT1_2;
    }
}

// Inverse GEMM per (m, p, row block of m'): Cinv^{m,p} = A^{m,p} Bz^{m,p}, stored
// column-major (rows m'/2 contiguous for each column c).
__global__ __launch_bounds__(GS::NTH) void gemm_inverse_kernel(const double *__restrict__ A, Blocks Ab,
                                                               const int *__restrict__ arows,
                                                               const int *__restrict__ akpad,
                                                               const double *__restrict__ Bz, Blocks Zb,
                                                               const Item *__restrict__ items, double *Cinv,
                                                               Blocks Cb, const int *__restrict__ cld)
{
    extern __shared__ __align__(16) char smem_raw[];
    const Item it = items[blockIdx.x];
    const int mp2 = 2 * it.m + it.p;
    const int tn = blockIdx.y;
    double4_t acc[GS::MB][GS::NB];
#pragma unroll
    for (int a = 0; a < GS::MB; ++a)
#pragma unroll
        for (int b = 0; b < GS::NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
    cm_block<double, GBM, GBN, GBK, GWM, GWN, true>(A + Ab.off[mp2] + it.tm * GBM, arows[mp2],
                                                    Bz + Zb.off[mp2] + tn * GBN, Zb.ld, akpad[mp2], acc,
                                                    (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % GWM, wn = wave / GWM, gi = lane & 15, gg = lane >> 4;
    const int64_t ld = cld[mp2];
    double *C = Cinv + Cb.off[mp2];
#pragma unroll
    for (int a = 0; a < GS::MB; ++a) {
        const int r = it.tm * GBM + wm * (GBM / GWM) + a * 16 + gi;
#pragma unroll
        for (int b = 0; b < GS::NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = tn * GBN + wn * (GBN / GWN) + b * 16 + acc_row<double>(gg, v);
                C[(int64_t)c * ld + r] = acc[a][b][v];
            }
    }
}

// ------------------------------------------------------------------ tables
__host__ __device__ inline int64_t wig_off(int l) { return (int64_t)l * (l + 1) * (2 * l + 1) / 6; }

// D[wig_off(l) + k (l+1) + m] = d^l_{k,m}(pi/2) for 0 <= k, m <= l < L: edge value
// d^l_{l,m} = (-1)^(l-m) 2^-l sqrt(C(2l, l+m)) (from m = l down by the ratio
// sqrt((l+m+1)/(l-m))), then the recursion in the first index
// sqrt((l+k)(l-k+1)) d_{k-1,m} = 2m d_{k,m} - sqrt((l-k)(l+k+1)) d_{k+1,m}, k = l..1.
__global__ void wigner_kernel(int L, double *D)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)L * (L + 1) / 2) return;
    int l = (int)((sqrt(8.0 * (double)g + 1.0) - 1.0) * 0.5);
    while ((int64_t)l * (l + 1) / 2 > g) --l;
    while ((int64_t)(l + 1) * (l + 2) / 2 <= g) ++l;
    const int m = (int)(g - (int64_t)l * (l + 1) / 2);
    double e = ldexp(1.0, -l);
    for (int mm = l - 1; mm >= m; --mm) e *= sqrt((double)(l + mm + 1) / (double)(l - mm));
    if ((l - m) & 1) e = -e;
    double *Dl = D + wig_off(l);
    const int ld = l + 1;
    Dl[(int64_t)l * ld + m] = e;
    double prev = 0.0, cur = e;
    for (int k = l; k >= 1; --k) {
        const double nxt = (2.0 * m * cur - sqrt((double)(l - k) * (l + k + 1)) * prev) / sqrt((double)(l + k) * (l - k + 1));
        Dl[(int64_t)(k - 1) * ld + m] = nxt;
        prev = cur;
        cur = nxt;
    }
}

__device__ inline double Ieven(int q) { return 2.0 / (1.0 - (double)q * (double)q); }

// Forward table W^{m,p}[r, col] (column-major, ld = wrows) for degree
// l = lstart(m,p) + 2r and m' = p + 2 col:
//   c_l sum_{k = l mod 2, k <= l} d^l_{k,0} d^l_{k,m} h(k, m', m),
// h = I(0) (k = 0, m' = 0), (1 + (-1)^m) I(k) (k > 0, m' = 0),
//     (1 + (-1)^m) I(m') (k = 0, m' > 0), 2 (I(k + m') + (-1)^m I(k - m')) otherwise.
__global__ void forward_table_kernel(int L, const double *__restrict__ D, double *W, Blocks Wb,
                                     const int *__restrict__ wrows, const int *__restrict__ kcols)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int R = (L - 1 - l0) / 2 + 1, Kc = kcols[p];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)R * Kc) return;
    const int r = (int)(g / Kc), col = (int)(g - (int64_t)r * Kc);
    const int l = l0 + 2 * r, mpr = p + 2 * col;
    const double sm = (m & 1) ? -1.0 : 1.0;
    const double *Dl = D + wig_off(l);
    const int ld = l + 1;
    double acc = 0.0;
    for (int k = l & 1; k <= l; k += 2) {
        double h;
        if (mpr == 0) h = (k == 0) ? Ieven(0) : (1.0 + sm) * Ieven(k);
        else h = (k == 0) ? (1.0 + sm) * Ieven(mpr) : 2.0 * (Ieven(k + mpr) + sm * Ieven(k - mpr));
        acc += Dl[(int64_t)k * ld] * Dl[(int64_t)k * ld + m] * h;
    }
    W[Wb.off[mp2] + (int64_t)col * wrows[mp2] + r] = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * acc;
}

// Inverse table A^{m,p}[r', col] (column-major, ld = arows) for m' = p + 2r' and
// degree l = lstart(m,p) + 2 col: 2 pi c_l d^l_{m',0} d^l_{m',m} (zero for m' > l).
__global__ void inverse_table_kernel(int L, const double *__restrict__ D, double *A, Blocks Ab,
                                     const int *__restrict__ arows, const int *__restrict__ kcols)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int R = (L - 1 - l0) / 2 + 1, Kr = kcols[p];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)R * Kr) return;
    const int col = (int)(g / Kr), rp = (int)(g - (int64_t)col * Kr);
    const int l = l0 + 2 * col, mpr = p + 2 * rp;
    double v = 0.0;
    if (mpr <= l) {
        const double *Dl = D + wig_off(l);
        v = 2.0 * M_PI * sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * Dl[(int64_t)mpr * (l + 1)] * Dl[(int64_t)mpr * (l + 1) + m];
    }
    A[Ab.off[mp2] + (int64_t)col * arows[mp2] + rp] = v;
}

}  // namespace sht
}  // namespace mpc

using namespace mpc;
using namespace mpc::sht;

// ---------------------------------------------------------------------- object
struct mpchol_sht {
    int dev = 0;
    hipStream_t st = nullptr;
    int L = 0, nth = 0, nph = 0, M = 0, tmax = 0, tmaxpad = 0;
    int nseq_phi = 1, nseq_th = 1;
    Plan Pphi{}, Pth{};
    double2 *tw_phi = nullptr, *tw_th = nullptr;
    // forward: W blocks (rows l, cols m'), operand Kr (rows m', cols c)
    double *W = nullptr, *Bk = nullptr;
    int64_t *w_off = nullptr, *b_off = nullptr;
    int *w_rows = nullptr, *kpad = nullptr;
    // inverse: A blocks (rows m', cols l), operand Bz (rows l, cols c), result Cinv (column-major)
    double *A = nullptr, *Bz = nullptr, *Cinv = nullptr;
    int64_t *a_off = nullptr, *z_off = nullptr, *c_off = nullptr;
    int *a_rows = nullptr, *a_kpad = nullptr;
    Item *items_f = nullptr, *items_i = nullptr;
    int nitems_f = 0, nitems_i = 0;
    double2 *G = nullptr;
    int64_t ldb = 0;
    size_t table_bytes = 0, work_bytes = 0;
};

namespace {

thread_local char g_sht_error[256] = "";

bool make_plan(int n, Plan &P)
{
    P.n = n;
    P.np = 0;
    int r = n;
    const int radices[4] = {4, 2, 3, 5};
    for (int R : radices)
        while (r % R == 0) {
            if (P.np == MAXP) return false;
            P.r[P.np++] = R;
            r /= R;
        }
    return r == 1;
}

// e^{-2 pi i k / n}, exact at multiples of n/4, reduced to the first half turn.
std::vector<double2> twiddles(int n)
{
    std::vector<double2> w(n);
    for (int k = 0; k < n; ++k) {
        double c, s;
        if ((4 * (int64_t)k) % n == 0) {
            const int q = (int)((4 * (int64_t)k) / n);
            const double cs[4][2] = {{1, 0}, {0, -1}, {-1, 0}, {0, 1}};
            c = cs[q][0];
            s = cs[q][1];
        } else if (2 * k < n) {
            const double a = 2.0 * M_PI * (double)k / (double)n;
            c = std::cos(a);
            s = -std::sin(a);
        } else {
            const double a = 2.0 * M_PI * (double)(n - k) / (double)n;
            c = std::cos(a);
            s = std::sin(a);
        }
        w[k] = make_double2(c, s);
    }
    return w;
}

int rup(int x, int a) { return (x + a - 1) / a * a; }

template <typename T> int dmalloc(T **p, size_t bytes, size_t &acc)
{
    if (hipMalloc((void **)p, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return MPCHOL_ENOMEM;
    }
    acc += bytes;
    return MPCHOL_OK;
}

template <typename T> int upload(T *d, const std::vector<T> &h, hipStream_t st)
{
    if (h.empty()) return MPCHOL_OK;
    return hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st) == hipSuccess ? MPCHOL_OK
                                                                                                      : MPCHOL_EHIP;
}

size_t fft_smem(int n, int nseq) { return (size_t)(nseq + 1) * n * sizeof(double2); }

void set_smem_attr(const void *k, size_t bytes)
{
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

extern "C" {

const char *mpchol_sht_last_error(void) { return g_sht_error; }

int mpchol_sht_destroy(mpchol_sht_t h)
{
    if (!h) return MPCHOL_OK;
    (void)hipSetDevice(h->dev);
    if (h->st) (void)hipStreamSynchronize(h->st);
    void *ps[] = {h->tw_phi, h->tw_th, h->W, h->Bk, h->w_off, h->b_off, h->w_rows, h->kpad, h->A, h->Bz, h->Cinv,
                  h->a_off, h->z_off, h->c_off, h->a_rows, h->a_kpad, h->items_f, h->items_i, h->G};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete h;
    return MPCHOL_OK;
}

int mpchol_sht_create(mpchol_sht_t *out, int32_t L, int32_t ntheta, int32_t nphi, int32_t tmax, int32_t device,
                      void *stream)
{
    if (!out) return MPCHOL_EINVAL;
    *out = nullptr;
    if (L < 1 || L > MAXL || ntheta < L + 1 || nphi < 2 * L - 1 || tmax < 1 || tmax > (1 << 20)) {
        snprintf(g_sht_error, sizeof(g_sht_error),
                 "invalid sizes: need 1 <= L <= %d, N_theta > L, N_phi >= 2L-1, 1 <= tmax <= 2^20", MAXL);
        return MPCHOL_EINVAL;
    }
    const int M = 2 * ntheta - 2;
    Plan Pphi, Pth;
    if (nphi > MAXN || M > MAXN || !make_plan(nphi, Pphi) || !make_plan(M, Pth)) {
        snprintf(g_sht_error, sizeof(g_sht_error),
                 "FFT lengths N_phi = %d and 2 N_theta - 2 = %d must be products of 2, 3 and 5, at most %d", nphi,
                 M, MAXN);
        return MPCHOL_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        snprintf(g_sht_error, sizeof(g_sht_error), "device %d not present", device);
        return MPCHOL_EHIP;
    }
    if (hipSetDevice(device) != hipSuccess) return MPCHOL_EHIP;
    mpchol_sht *h = new (std::nothrow) mpchol_sht();
    if (!h) return MPCHOL_ENOMEM;
    h->dev = device;
    h->st = (hipStream_t)stream;
    h->L = L;
    h->nth = ntheta;
    h->nph = nphi;
    h->M = M;
    h->tmax = tmax;
    h->tmaxpad = rup(tmax, GBN / 2);
    h->Pphi = Pphi;
    h->Pth = Pth;
    h->nseq_phi = std::max(1, std::min(4, NTH * MAXV / nphi));
    h->nseq_th = std::max(1, std::min(8, NTH * MAXV / M));
    h->ldb = 2 * (int64_t)h->tmaxpad;

    // block geometry per (m, p)
    const int nb = 2 * L;
    std::vector<int64_t> w_off(nb), b_off(nb), a_off(nb), z_off(nb), c_off(nb);
    std::vector<int> w_rows(nb), a_rows(nb), a_kpad(nb), kpad(2), kcols(2);
    std::vector<Item> items_f, items_i;
    for (int p = 0; p < 2; ++p) {
        kcols[p] = p == 0 ? (L + 1) / 2 : L / 2;  // m' in [0, L) of parity p
        kpad[p] = rup(std::max(kcols[p], 1), GBK);
    }
    int64_t wsz = 0, bsz = 0, asz = 0, zsz = 0, csz = 0;
    for (int m = 0; m < L; ++m)
        for (int p = 0; p < 2; ++p) {
            const int i = 2 * m + p, l0 = lstart(m, p);
            const int R = l0 < L ? (L - 1 - l0) / 2 + 1 : 0;
            w_rows[i] = rup(std::max(R, 1), GBM);
            w_off[i] = wsz;
            wsz += (int64_t)w_rows[i] * kpad[p];
            b_off[i] = bsz;
            bsz += (int64_t)kpad[p] * h->ldb;
            a_rows[i] = rup(std::max(kcols[p], 1), GBM);
            a_kpad[i] = rup(std::max(R, 1), GBK);
            a_off[i] = asz;
            asz += (int64_t)a_rows[i] * a_kpad[i];
            z_off[i] = zsz;
            zsz += (int64_t)a_kpad[i] * h->ldb;
            c_off[i] = csz;
            csz += (int64_t)a_rows[i] * h->ldb;
            if (R > 0) {
                for (int tm = 0; tm < w_rows[i] / GBM; ++tm) items_f.push_back(Item{(int16_t)m, (int16_t)p, tm});
                if (kcols[p] > 0)
                    for (int tm = 0; tm < a_rows[i] / GBM; ++tm) items_i.push_back(Item{(int16_t)m, (int16_t)p, tm});
            }
        }
    h->nitems_f = (int)items_f.size();
    h->nitems_i = (int)items_i.size();

    size_t tb = 0, wb = 0;
    int rc = MPCHOL_OK;
    double *D = nullptr;
    auto A_ = [&](int r) {
        if (rc == MPCHOL_OK) rc = r;
    };
    A_(dmalloc(&h->tw_phi, nphi * sizeof(double2), tb));
    A_(dmalloc(&h->tw_th, M * sizeof(double2), tb));
    A_(dmalloc(&h->W, wsz * 8, tb));
    A_(dmalloc(&h->A, asz * 8, tb));
    A_(dmalloc(&h->w_off, nb * 8, tb));
    A_(dmalloc(&h->b_off, nb * 8, tb));
    A_(dmalloc(&h->a_off, nb * 8, tb));
    A_(dmalloc(&h->z_off, nb * 8, tb));
    A_(dmalloc(&h->c_off, nb * 8, tb));
    A_(dmalloc(&h->w_rows, nb * 4, tb));
    A_(dmalloc(&h->a_rows, nb * 4, tb));
    A_(dmalloc(&h->a_kpad, nb * 4, tb));
    A_(dmalloc(&h->kpad, 2 * 4, tb));
    A_(dmalloc(&h->items_f, std::max<size_t>(1, items_f.size()) * sizeof(Item), tb));
    A_(dmalloc(&h->items_i, std::max<size_t>(1, items_i.size()) * sizeof(Item), tb));
    A_(dmalloc(&h->Bk, bsz * 8, wb));
    A_(dmalloc(&h->Bz, zsz * 8, wb));
    A_(dmalloc(&h->Cinv, csz * 8, wb));
    A_(dmalloc(&h->G, (size_t)tmax * L * ntheta * sizeof(double2), wb));
    size_t scratch = 0;
    A_(dmalloc(&D, (size_t)wig_off(L) * 8, scratch));
    int *kcols_d = nullptr;
    A_(dmalloc(&kcols_d, 2 * 4, scratch));
    h->table_bytes = tb;
    h->work_bytes = wb;
    if (rc != MPCHOL_OK) {
        snprintf(g_sht_error, sizeof(g_sht_error), "device allocation failed (tables %zu B, work %zu B)", tb, wb);
        if (D) (void)hipFree(D);
        if (kcols_d) (void)hipFree(kcols_d);
        mpchol_sht_destroy(h);
        return rc;
    }
    hipStream_t st = h->st;
    // zero padding: tables, operands (padded K rows must be zero) and the
    // inverse result (blocks without any degree stay zero)
    bool ok = hipMemsetAsync(h->W, 0, wsz * 8, st) == hipSuccess && hipMemsetAsync(h->A, 0, asz * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Bk, 0, bsz * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Bz, 0, zsz * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Cinv, 0, csz * 8, st) == hipSuccess;
    const std::vector<double2> twp = twiddles(nphi), twt = twiddles(M);
    if (ok)
        ok = upload(h->tw_phi, twp, st) == MPCHOL_OK && upload(h->tw_th, twt, st) == MPCHOL_OK &&
             upload(h->w_off, w_off, st) == MPCHOL_OK && upload(h->b_off, b_off, st) == MPCHOL_OK &&
             upload(h->a_off, a_off, st) == MPCHOL_OK && upload(h->z_off, z_off, st) == MPCHOL_OK &&
             upload(h->c_off, c_off, st) == MPCHOL_OK && upload(h->w_rows, w_rows, st) == MPCHOL_OK &&
             upload(h->a_rows, a_rows, st) == MPCHOL_OK && upload(h->a_kpad, a_kpad, st) == MPCHOL_OK &&
             upload(h->kpad, kpad, st) == MPCHOL_OK && upload(h->items_f, items_f, st) == MPCHOL_OK &&
             upload(h->items_i, items_i, st) == MPCHOL_OK && upload(kcols_d, kcols, st) == MPCHOL_OK;
    if (ok) {
        const int64_t nlm = (int64_t)L * (L + 1) / 2;
        wigner_kernel<<<(unsigned)((nlm + 255) / 256), 256, 0, st>>>(L, D);
        int64_t maxf = 0;
        for (int p = 0; p < 2; ++p) maxf = std::max<int64_t>(maxf, (int64_t)((L + 1) / 2) * kcols[p]);
        dim3 gt((unsigned)((maxf + 255) / 256), (unsigned)nb);
        forward_table_kernel<<<gt, 256, 0, st>>>(L, D, h->W, Blocks{h->w_off, 0}, h->w_rows, kcols_d);
        inverse_table_kernel<<<gt, 256, 0, st>>>(L, D, h->A, Blocks{h->a_off, 0}, h->a_rows, kcols_d);
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    }
    (void)hipFree(D);
    (void)hipFree(kcols_d);
    if (!ok) {
        snprintf(g_sht_error, sizeof(g_sht_error), "table set-up failed: %s", hipGetErrorString(hipGetLastError()));
        mpchol_sht_destroy(h);
        return MPCHOL_EHIP;
    }
    set_smem_attr((const void *)phi_forward_kernel, fft_smem(nphi, h->nseq_phi));
    set_smem_attr((const void *)phi_inverse_kernel, fft_smem(nphi, h->nseq_phi));
    set_smem_attr((const void *)theta_forward_kernel, fft_smem(M, h->nseq_th));
    set_smem_attr((const void *)theta_inverse_kernel, fft_smem(M, h->nseq_th));
    set_smem_attr((const void *)gemm_forward_kernel, GS::SMEM);
    set_smem_attr((const void *)gemm_inverse_kernel, GS::SMEM);
    *out = h;
    return MPCHOL_OK;
}

int mpchol_sht_info(mpchol_sht_t h, int64_t *table_bytes, int64_t *work_bytes, int64_t *gemm_flops_per_step)
{
    if (!h) return MPCHOL_EINVAL;
    if (table_bytes) *table_bytes = (int64_t)h->table_bytes;
    if (work_bytes) *work_bytes = (int64_t)h->work_bytes;
    if (gemm_flops_per_step) {
        // unpadded: per (m, p) rows x (m' of parity p) x 2 columns x 2 flops
        int64_t fl = 0;
        for (int m = 0; m < h->L; ++m)
            for (int p = 0; p < 2; ++p) {
                const int l0 = lstart(m, p);
                const int64_t R = l0 < h->L ? (h->L - 1 - l0) / 2 + 1 : 0;
                const int64_t Kc = p == 0 ? (h->L + 1) / 2 : h->L / 2;
                fl += 4 * R * Kc;
            }
        *gemm_flops_per_step = fl;
    }
    return MPCHOL_OK;
}

int mpchol_sht_forward(mpchol_sht_t h, const double *Z, int64_t T, double *f)
{
    if (!h || T < 0 || T > h->tmax) return MPCHOL_EINVAL;
    if (T == 0) return MPCHOL_OK;
    if (!Z || !f) return MPCHOL_EINVAL;
    if (hipSetDevice(h->dev) != hipSuccess) return MPCHOL_EHIP;
    hipStream_t st = h->st;
    const int Tpad = rup((int)T, GBN / 2);
    const int64_t rows = T * h->nth;
    const int nrow = 2 * h->nseq_phi;
    phi_forward_kernel<<<(unsigned)((rows + nrow - 1) / nrow), NTH, fft_smem(h->nph, h->nseq_phi), st>>>(
        Z, rows, h->nth, h->L, h->Pphi, h->tw_phi, h->G, h->nseq_phi);
    dim3 gt((unsigned)((T + h->nseq_th - 1) / h->nseq_th), (unsigned)h->L);
    theta_forward_kernel<<<gt, NTH, fft_smem(h->M, h->nseq_th), st>>>(h->G, (int)T, h->nth, h->L, h->Pth, h->tw_th,
                                                                    h->Bk, Blocks{h->b_off, h->ldb}, Tpad,
                                                                    h->nseq_th);
    dim3 gg((unsigned)h->nitems_f, (unsigned)(2 * Tpad / GBN));
    gemm_forward_kernel<<<gg, GS::NTH, GS::SMEM, st>>>(h->W, Blocks{h->w_off, 0}, h->w_rows, h->Bk,
                                                       Blocks{h->b_off, h->ldb}, h->kpad, h->items_f, h->L, (int)T,
                                                       Tpad, f);
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_sht_inverse(mpchol_sht_t h, const double *f, int64_t T, double *Z)
{
    if (!h || T < 0 || T > h->tmax) return MPCHOL_EINVAL;
    if (T == 0) return MPCHOL_OK;
    if (!Z || !f) return MPCHOL_EINVAL;
    if (hipSetDevice(h->dev) != hipSuccess) return MPCHOL_EHIP;
    hipStream_t st = h->st;
    const int Tpad = rup((int)T, GBN / 2);
    const int64_t ncoef = T * (int64_t)h->L * h->L;
    pack_inverse_kernel<<<(unsigned)((ncoef + 255) / 256), 256, 0, st>>>(f, (int)T, h->L, h->Bz,
                                                                        Blocks{h->z_off, h->ldb}, Tpad);
    dim3 gg((unsigned)h->nitems_i, (unsigned)(2 * Tpad / GBN));
    gemm_inverse_kernel<<<gg, GS::NTH, GS::SMEM, st>>>(h->A, Blocks{h->a_off, 0}, h->a_rows, h->a_kpad, h->Bz,
                                                       Blocks{h->z_off, h->ldb}, h->items_i, h->Cinv,
                                                       Blocks{h->c_off, 0}, h->a_rows);
    dim3 gt((unsigned)((T + h->nseq_th - 1) / h->nseq_th), (unsigned)h->L);
    theta_inverse_kernel<<<gt, NTH, fft_smem(h->M, h->nseq_th), st>>>(h->Cinv, Blocks{h->c_off, 0}, h->a_rows,
                                                                    (int)T, h->nth, h->L, h->Pth, h->tw_th, h->G,
                                                                    Tpad, h->nseq_th);
    const int64_t rows = T * h->nth;
    const int nrow = 2 * h->nseq_phi;
    phi_inverse_kernel<<<(unsigned)((rows + nrow - 1) / nrow), NTH, fft_smem(h->nph, h->nseq_phi), st>>>(
        h->G, rows, h->nth, h->L, h->Pphi, h->tw_phi, Z, h->nseq_phi);
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

}  // extern "C"
