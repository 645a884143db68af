// Spherical harmonic transform of fields on an equiangular grid (Sec. III.A.1,
// "Modeling in the Spherical Harmonic Domain"; the precomputation of
// Sec. III.A.2) and its inverse, used to turn emulated coefficient vectors
// back into fields (Sec. III.B), batched over time steps, and the C ABI of the
// transform object (include/mpchol.h).
//
// The paper's route: G_m(theta_j) by FFT along longitude; G_m extended to
// colatitudes in (pi, 2 pi) with G_m(2 pi - theta) = (-1)^m G_m(theta) and an
// FFT along the extended colatitude gives K_{m,m'}; the coefficients follow
// from K through Wigner-d functions at pi/2, precomputed by a three-term
// recursion.  Every step after the longitude FFT is linear in G_m and the
// same for all time steps, so on the GPU the steps are composed once, at
// set-up, into one real table per order m (Sec. III.A.2 precomputes the
// Wigner-d part; here the colatitude DFT and both sums are precomputed too):
//   * the two sums (over m' with I(m' + m'') and over m'' with S_{l,m,m''})
//     fold into a table over m' >= 0, using K_{m,-m'} = (-1)^m K_{m,m'}, the
//     cancellation of the q = +-1 terms of I(q) under that symmetry, and
//     d^l_{m'',0}(pi/2) = 0 for l + m'' odd (degree l meets only m' = l mod 2);
//   * the colatitude DFT of the extended G_m, written out with that symmetry,
//     weighs G_m(theta_j) by 2 cos(m' theta_j) (m even) or -2i sin(m' theta_j)
//     (m odd, pole samples zero); composed with the folded table it gives
//     z_{l,m} = i^{-m-(m mod 2)} sum_j a_{l,j} G_m(theta_j) with a real;
//   * a_{l, pi - theta} = (-1)^{l+m} a_{l,theta}, so only the northern half of
//     the colatitudes is kept: rows j and N_theta - 1 - j are transformed
//     together (two real rows per complex FFT) and enter as
//     G_j + G_{N-1-j} (l + m even) or G_j - G_{N-1-j} (l + m odd).
// Per order m and degree parity p the forward transform is then one real FP64
// MFMA GEMM over all time steps of a batch (columns 2t and 2t + 1 hold the
// real and imaginary parts), and the inverse the mirror image with the table
// 2 pi Y_lm(theta_j, 0) (up to the sign i^{m - (m mod 2)}), composed the same
// way from the paper's K_{m,m'} = 2 pi i^-m sum_l c_l d^l_{m',0} d^l_{m',m} z_{l,m}
// and G_m(theta) = sum_m' K_{m,m'} e^{i m' theta}.  GEMM work per time step
// stays about L^3 flops; the colatitude FFT leaves the per-field path.
// Readings (the grid, the 1/2pi of the longitude synthesis, the poles, the
// real layout of the coefficient vector) are stated with the declarations in
// mpchol.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/mpchol.h"
#include "common.h"
#include "gemm_core.h"

namespace mpc {
namespace sht {

constexpr int NTH = 512;   // threads of an FFT workgroup
constexpr int MAXV = 8;    // complex values per thread and pass: nseq * n <= NTH * MAXV
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
__host__ __device__ inline int lstart(int m, int p) { return ((m & 1) == p) ? m : m + 1; }

// Forward: sequence g = j' T + t (j' < H = ceil(N_theta / 2)) packs rows j' and
// N_theta - 1 - j' of field t (the second row zero at the equator of an odd
// grid); with A, B their spectra times 2 pi / N_phi, block (m, q) of Gb gets
// row j', columns 2t, 2t + 1: A + B (q = 0) and A - B (q = 1), m = 0..L-1.
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4, 8))) void phi_forward_kernel(
    const double *__restrict__ Z, int T, int ntheta, int L, Plan P, const double2 *__restrict__ twg, double *Gb,
    int64_t blk, int64_t ld, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int n = P.n;
    const int H = (ntheta + 1) / 2;
    const int64_t nsq = (int64_t)H * T;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + n;
    load_twiddles(tws, twg, n);
    const int64_t g0 = (int64_t)blockIdx.x * nseq;
    double2 vin[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        const int idx = threadIdx.x + i * NTH;
        vin[i] = make_double2(0.0, 0.0);
        if (idx < nseq * n) {
            const int s = idx / n, k = idx - s * n;
            const int64_t g = g0 + s;
            if (g < nsq) {
                const int jp = (int)(g / T), t = (int)(g - (int64_t)jp * T);
                const int js = ntheta - 1 - jp;
                const double *zt = Z + (int64_t)t * ntheta * n;
                vin[i].x = zt[(int64_t)jp * n + k];
                if (js != jp) vin[i].y = zt[(int64_t)js * n + k];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        const int idx = threadIdx.x + i * NTH;
        if (idx < nseq * n) buf[idx] = vin[i];
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, false);
    const double sc = M_PI / n;  // (2 pi / n) / 2 of the two-row separation
    for (int idx = threadIdx.x; idx < nseq * L; idx += NTH) {
        const int s = idx % nseq, m = idx / nseq;
        const int64_t g = g0 + s;
        if (g >= nsq) continue;
        const int jp = (int)(g / T), t = (int)(g - (int64_t)jp * T);
        const double2 X = buf[s * n + m], Y = buf[s * n + (n - m) % n];
        // A = (X + conj Y) / 2, B = (X - conj Y) / 2i, both times 2 pi / n
        const double2 a = make_double2(sc * (X.x + Y.x), sc * (X.y - Y.y));
        const double2 b = make_double2(sc * (X.y + Y.y), -sc * (X.x - Y.x));
        double2 gs = cadd(a, b), ga = csub(a, b);
        if (ntheta - 1 - jp == jp) ga = make_double2(0.0, 0.0);
        *(double2 *)(Gb + (2 * m) * blk + jp * ld + 2 * t) = gs;
        *(double2 *)(Gb + (2 * m + 1) * blk + jp * ld + 2 * t) = ga;
    }
}

// Inverse: for the pair of rows (j', N_theta - 1 - j') of field t, with E and O
// the results of the even (l + m even) and odd blocks of order m,
// G_m = i^{m mod 2 - m} (E + O) on row j' and i^{m mod 2 - m} (E - O) on its
// mirror; Z = (1 / 2 pi) sum_{|m| < L} G_m e^{i m phi}, G_{-m} = conj(G_m), both
// rows from one inverse FFT (their spectra are Hermitian).
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(4, 8))) void phi_inverse_kernel(
    const double *__restrict__ Ob, int64_t blk, int64_t ld, int T, int ntheta, int L, Plan P,
    const double2 *__restrict__ twg, double *__restrict__ Z, int nseq)
{
    extern __shared__ __align__(16) char smem_raw[];
    const int n = P.n;
    const int H = (ntheta + 1) / 2;
    const int64_t nsq = (int64_t)H * T;
    double2 *tws = (double2 *)smem_raw;
    double2 *buf = tws + n;
    load_twiddles(tws, twg, n);
    for (int idx = threadIdx.x; idx < nseq * n; idx += NTH) buf[idx] = make_double2(0.0, 0.0);
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * nseq;
    const double sc = 1.0 / (2.0 * M_PI);
    for (int idx = threadIdx.x; idx < nseq * L; idx += NTH) {
        const int s = idx % nseq, m = idx / nseq;
        const int64_t g = g0 + s;
        if (g >= nsq) continue;
        const int jp = (int)(g / T), t = (int)(g - (int64_t)jp * T);
        const int p0 = m & 1;  // degree parity of the block with l + m even
        const double2 E = *(const double2 *)(Ob + (2 * m + p0) * blk + jp * ld + 2 * t);
        const double2 O = *(const double2 *)(Ob + (2 * m + (p0 ^ 1)) * blk + jp * ld + 2 * t);
        const int e = ((m & 1) - m) & 3;
        const double2 ga = cscale(ipow(cadd(E, O), e), sc);
        double2 gb = cscale(ipow(csub(E, O), e), sc);
        if (ntheta - 1 - jp == jp) gb = make_double2(0.0, 0.0);
        if (m == 0) {  // G_0 of a real field is real
            buf[s * n] = make_double2(ga.x, gb.x);
        } else {
            buf[s * n + m] = make_double2(ga.x - gb.y, ga.y + gb.x);       // ga + i gb
            buf[s * n + n - m] = make_double2(ga.x + gb.y, -ga.y + gb.x);  // conj(ga) + i conj(gb)
        }
    }
    __syncthreads();
    fft_run(buf, nseq, P, tws, true);
    for (int idx = threadIdx.x; idx < nseq * n; idx += NTH) {
        const int s = idx / n, k = idx - s * n;
        const int64_t g = g0 + s;
        if (g >= nsq) continue;
        const int jp = (int)(g / T), t = (int)(g - (int64_t)jp * T);
        const int js = ntheta - 1 - jp;
        double *zt = Z + (int64_t)t * ntheta * n;
        const double2 v = buf[idx];
        zt[(int64_t)jp * n + k] = v.x;
        if (js != jp) zt[(int64_t)js * n + k] = v.y;
    }
}

// ------------------------------------------------------------------ contraction
struct Item {
    int16_t m, p;
    int32_t tm;
};

// Forward GEMM per (m, p, row block): C^{m,p} = A^{m,p} Gq, q = (p + m) mod 2, over
// the northern colatitudes, written row-major (rows r, columns 2t / 2t + 1
// contiguous) into block (m, p) of Cf.
__global__ __launch_bounds__(GS::NTH) void gemm_forward_kernel(const double *__restrict__ Af,
                                                               const int64_t *__restrict__ aoff,
                                                               const int *__restrict__ arows,
                                                               const double *__restrict__ Gb, int64_t gblk,
                                                               int64_t ldb, int Kp, const Item *__restrict__ items,
                                                               double *Cf, int64_t cblk)
{
    extern __shared__ __align__(16) char smem_raw[];
    const Item it = items[blockIdx.x];
    const int m = it.m, p = it.p, mp2 = 2 * m + p, q = (p + m) & 1;
    const int tn = blockIdx.y;
    double4_t acc[GS::MB][GS::NB];
#pragma unroll
    for (int a = 0; a < GS::MB; ++a)
#pragma unroll
        for (int b = 0; b < GS::NB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
    cm_block<double, GBM, GBN, GBK, GWM, GWN, false>(Af + aoff[mp2] + it.tm * GBM, arows[mp2],
                                                     Gb + (2 * m + q) * gblk + tn * GBN, ldb, Kp, acc,
                                                     (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % GWM, wn = wave / GWM, gi = lane & 15, gg = lane >> 4;
    double *C = Cf + mp2 * cblk;
#pragma unroll
    for (int a = 0; a < GS::MB; ++a)
#pragma unroll
        for (int b = 0; b < GS::NB; ++b) {
            const int c = tn * GBN + wn * (GBN / GWN) + b * 16 + gi;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = it.tm * GBM + wm * (GBM / GWM) + a * 16 + acc_row<double>(gg, v);
                C[(int64_t)row * ldb + c] = acc[a][b][v];
            }
        }
}

// Degree of pair pr of a chunk starting at degree la, where degree l holds the
// l + 1 pairs (l, 0..l): the largest l with (l (l+1) - la (la+1)) / 2 <= pr.
__device__ inline int pair_degree(int pr, int la)
{
    const double u = 2.0 * pr + (double)la * (la + 1);
    int l = (int)((sqrt(4.0 * u + 1.0) - 1.0) * 0.5);
    while (l * (l + 1) > u) --l;
    while ((l + 1) * (l + 2) <= u) ++l;
    return l;
}

constexpr int TNT = 1024;  // threads of a transpose workgroup

// Transposes between the coefficient vectors f (T x L^2, degree-major) and the
// per-order GEMM blocks (rows r = (l - lstart(m,p)) / 2, columns 2t / 2t + 1),
// through LDS: a workgroup owns TT time steps and a chunk of whole degrees
// [l_a, l_b) (at most CH coefficients), reads one side contiguously and writes
// the other in runs of 2 TT doubles.
//
// Forward: z_{l,m} = i^{-m-(m mod 2)} (C[r][2t] + i C[r][2t + 1]); f gets z_{l,0}
// and sqrt(2) Re / Im z_{l,m} at l^2 + l +- m.
__global__ __launch_bounds__(TNT) void unpack_forward_kernel(const double *__restrict__ Cf, int64_t cblk, int64_t ldb,
                                      const int *__restrict__ chunk_l, int T, int L, int TT, int CH,
                                      double *__restrict__ f)
{
    extern __shared__ __align__(16) char smem_raw[];
    double *buf = (double *)smem_raw;  // [TT][CH], raw (a at l^2+l+m, b at l^2+l-m)
    const int la = chunk_l[blockIdx.x], lb = chunk_l[blockIdx.x + 1];
    const int i0 = la * la, ni = lb * lb - i0;
    const int t0 = blockIdx.y * TT;
    const int tt = min(TT, T - t0);
    // gather: one (l, m >= 0) pair and 2 tt columns per 2 tt threads
    const int npair = (lb * (lb + 1) - la * (la + 1)) / 2;  // sum over l of (l + 1)
    for (int g = threadIdx.x; g < npair * 2 * tt; g += blockDim.x) {
        const int col = g % (2 * tt), pr = g / (2 * tt);
        const int l = pair_degree(pr, la);
        const int m = pr - (l * (l + 1) - la * (la + 1)) / 2, p = l & 1, r = (l - lstart(m, p)) >> 1;
        const int t = t0 + col / 2, part = col & 1;
        const double v = Cf[(2 * m + p) * cblk + (int64_t)r * ldb + 2 * t + part];
        const int idx = l * l + l + (part ? -m : m) - i0;
        if (m > 0 || part == 0) buf[(col / 2) * CH + idx] = v;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < tt * ni; g += blockDim.x) {
        const int ts = g / ni, idx = g - ts * ni;
        const int gi_ = idx + i0;
        int l = (int)sqrt((double)gi_);
        while (l * l > gi_) --l;
        while ((l + 1) * (l + 1) <= gi_) ++l;
        const int ms = gi_ - l * l - l, m = ms < 0 ? -ms : ms;
        double v;
        if (m == 0) {
            v = buf[ts * CH + idx];
        } else {
            const double a = buf[ts * CH + (l * l + l + m - i0)], b = buf[ts * CH + (l * l + l - m - i0)];
            const int rot = (m + (m & 1)) & 3;  // z = i^-rot (a + i b)
            double re, im;
            switch (rot) {
            case 0: re = a; im = b; break;
            case 1: re = b; im = -a; break;
            case 2: re = -a; im = -b; break;
            default: re = -b; im = a; break;
            }
            v = M_SQRT2 * (ms > 0 ? re : im);
        }
        f[(int64_t)(t0 + ts) * L * L + gi_] = v;
    }
}

// Inverse operand Bz^{m,p}[r][2t] = Re z_{l,m}, [r][2t + 1] = Im z_{l,m} for
// l = lstart + 2r, from f through LDS (same tiling as the forward unpack).
__global__ __launch_bounds__(TNT) void pack_inverse_kernel(const double *__restrict__ f, const int *__restrict__ chunk_l, int T, int L,
                                    int TT, int CH, double *Bz, const int64_t *__restrict__ zoff, int64_t ldb)
{
    extern __shared__ __align__(16) char smem_raw[];
    double *buf = (double *)smem_raw;  // [TT][CH]
    const int la = chunk_l[blockIdx.x], lb = chunk_l[blockIdx.x + 1];
    const int i0 = la * la, ni = lb * lb - i0;
    const int t0 = blockIdx.y * TT;
    const int tt = min(TT, T - t0);
    for (int g = threadIdx.x; g < tt * ni; g += blockDim.x) {
        const int ts = g / ni, idx = g - ts * ni;
        buf[ts * CH + idx] = f[(int64_t)(t0 + ts) * L * L + i0 + idx];
    }
    __syncthreads();
    const int npair = (lb * (lb + 1) - la * (la + 1)) / 2;
    for (int g = threadIdx.x; g < npair * 2 * tt; g += blockDim.x) {
        const int col = g % (2 * tt), pr = g / (2 * tt);
        const int l = pair_degree(pr, la);
        const int m = pr - (l * (l + 1) - la * (la + 1)) / 2, p = l & 1, r = (l - lstart(m, p)) >> 1;
        const int ts = col / 2, part = col & 1;
        double v;
        if (m == 0) v = part ? 0.0 : buf[ts * CH + l * l + l - i0];
        else v = buf[ts * CH + l * l + l + (part ? -m : m) - i0] * M_SQRT1_2;
        Bz[zoff[2 * m + p] + (int64_t)r * ldb + 2 * (t0 + ts) + part] = v;
    }
}

// Inverse GEMM per (m, p, row block of j'): E/O^{m,p}[j'][c] = V^{m,p} Bz^{m,p},
// written row-major (columns contiguous) into block (m, p) of Ob.
__global__ __launch_bounds__(GS::NTH) void gemm_inverse_kernel(const double *__restrict__ V,
                                                               const int64_t *__restrict__ voff, int64_t ldv,
                                                               const int *__restrict__ kpadz,
                                                               const double *__restrict__ Bz,
                                                               const int64_t *__restrict__ zoff, int64_t ldb,
                                                               const Item *__restrict__ items, double *Ob,
                                                               int64_t oblk)
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
    cm_block<double, GBM, GBN, GBK, GWM, GWN, false>(V + voff[mp2] + it.tm * GBM, ldv, Bz + zoff[mp2] + tn * GBN,
                                                     ldb, kpadz[mp2], acc, (double *)smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % GWM, wn = wave / GWM, gi = lane & 15, gg = lane >> 4;
    double *O = Ob + mp2 * oblk;
#pragma unroll
    for (int a = 0; a < GS::MB; ++a)
#pragma unroll
        for (int b = 0; b < GS::NB; ++b) {
            const int c = tn * GBN + wn * (GBN / GWN) + b * 16 + gi;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = it.tm * GBM + wm * (GBM / GWM) + a * 16 + acc_row<double>(gg, v);
                O[(int64_t)row * ldb + c] = acc[a][b][v];
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

// Folded table W^{m,p}[r, col] (row-major, ld = kc) for degree l = lstart(m,p) + 2r
// and m' = p + 2 col:  c_l sum_{k = l mod 2, k <= l} d^l_{k,0} d^l_{k,m} h(k, m', m),
// h = I(0) (k = 0, m' = 0), (1 + (-1)^m) I(k) (k > 0, m' = 0),
//     (1 + (-1)^m) I(m') (k = 0, m' > 0), 2 (I(k + m') + (-1)^m I(k - m')) otherwise.
__global__ void folded_table_kernel(int L, const double *__restrict__ D, double *W, int64_t blk, int kc)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int R = (L - 1 - l0) / 2 + 1, Kc = p == 0 ? (L + 1) / 2 : L / 2;
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
    W[mp2 * blk + (int64_t)r * kc + col] = sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * acc;
}

// S table S^{m,p}[r', col] (row-major, ld = rc) for m' = p + 2r' and degree
// l = lstart(m,p) + 2 col: 2 pi c_l d^l_{m',0} d^l_{m',m} (zero for m' > l).
__global__ void s_table_kernel(int L, const double *__restrict__ D, double *S, int64_t blk, int rc)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int R = (L - 1 - l0) / 2 + 1, Kr = p == 0 ? (L + 1) / 2 : L / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)R * Kr) return;
    const int rp = (int)(g / R), col = (int)(g - (int64_t)rp * R);
    const int l = l0 + 2 * col, mpr = p + 2 * rp;
    double v = 0.0;
    if (mpr <= l) {
        const double *Dl = D + wig_off(l);
        v = 2.0 * M_PI * sqrt((2.0 * l + 1.0) / (4.0 * M_PI)) * Dl[(int64_t)mpr * (l + 1)] * Dl[(int64_t)mpr * (l + 1) + m];
    }
    S[mp2 * blk + (int64_t)rp * rc + col] = v;
}

// Forward table A^{m,p}[j'][r] (column-major, ld = arows): the folded table
// composed with the colatitude DFT of the extended G_m,
//   a_{l,j'} = (1 / M) sum_{m' = p mod 2} W^{m,p}[r][m'/2] kap_{m mod 2}[m'][j'],
// kap_0 = 1 at the pole row, 2 cos(m' theta_j') elsewhere; kap_1 = 0 at the pole,
// 2 sin(m' theta_j') elsewhere (the -i of odd orders goes to the epilogue).  The
// equator column of rows with l + m odd is exactly zero.
__global__ void compose_forward_kernel(int L, int ntheta, const double *__restrict__ W, int64_t wblk, int kc,
                                       const double *__restrict__ kap, double *Af, const int64_t *__restrict__ aoff,
                                       const int *__restrict__ arows)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int H = (ntheta + 1) / 2, M = 2 * ntheta - 2;
    const int R = (L - 1 - l0) / 2 + 1, Kc = p == 0 ? (L + 1) / 2 : L / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)R * H) return;
    const int jp = (int)(g / R), r = (int)(g - (int64_t)jp * R);
    double v = 0.0;
    if (!((ntheta & 1) && jp == H - 1 && ((p + m) & 1))) {
        const double *w = W + mp2 * wblk + (int64_t)r * kc;
        const double *kp = kap + ((int64_t)(m & 1) * L) * H + jp;
        for (int col = 0; col < Kc; ++col) v += w[col] * kp[(int64_t)(p + 2 * col) * H];
        v /= M;
    }
    Af[aoff[mp2] + (int64_t)jp * arows[mp2] + r] = v;
}

// Inverse table V^{m,p}[r][j'] (column-major over j', ld = ldv): the S table
// composed with the colatitude synthesis G_m(theta) = sum_m' K_{m,m'} e^{i m' theta},
//   v_{j',l} = sum_{m' = p mod 2} S^{m,p}[m'/2][r] lam_{m mod 2}[m'][j'],
// lam_0 = 1 (m' = 0), 2 cos(m' theta_j'); lam_1 = 0 (m' = 0), 2 sin(m' theta_j')
// (the i of odd orders goes to the longitude kernel).
__global__ void compose_inverse_kernel(int L, int ntheta, const double *__restrict__ S, int64_t sblk, int rc,
                                       const double *__restrict__ lam, double *V, const int64_t *__restrict__ voff,
                                       int64_t ldv)
{
    const int mp2 = blockIdx.y, m = mp2 >> 1, p = mp2 & 1;
    const int l0 = lstart(m, p);
    if (l0 >= L) return;
    const int H = (ntheta + 1) / 2;
    const int R = (L - 1 - l0) / 2 + 1, Kr = p == 0 ? (L + 1) / 2 : L / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)R * H) return;
    const int r = (int)(g / H), jp = (int)(g - (int64_t)r * H);
    const double *sp = S + mp2 * sblk + r;
    const double *lp = lam + ((int64_t)(m & 1) * L) * H + jp;
    double v = 0.0;
    for (int rp = 0; rp < Kr; ++rp) v += sp[(int64_t)rp * rc] * lp[(int64_t)(p + 2 * rp) * H];
    V[voff[mp2] + (int64_t)r * ldv + jp] = v;
}

}  // namespace sht
}  // namespace mpc

using namespace mpc;
using namespace mpc::sht;

// ---------------------------------------------------------------------- object
struct mpchol_sht {
    int dev = 0;
    hipStream_t st = nullptr;
    int L = 0, nth = 0, nph = 0, H = 0, tmax = 0, tmaxpad = 0;
    int kph = 0;      // forward K extent: H padded to GBK
    int64_t vrows = 0; // inverse row extent: H padded to GBM
    int nseq = 1;
    Plan Pphi{};
    double2 *tw = nullptr;
    double *Af = nullptr, *V = nullptr;               // composed tables
    int64_t *a_off = nullptr, *v_off = nullptr, *z_off = nullptr;
    int *a_rows = nullptr, *z_kpad = nullptr;
    Item *items_f = nullptr, *items_i = nullptr;
    int nitems_f = 0, nitems_i = 0;
    double *Gb = nullptr, *Bz = nullptr, *Ob = nullptr;  // work: folded G, packed z, GEMM results
    int *chunk_l = nullptr;                              // degree chunks of the f transposes
    int nchunk = 0, TT = 1, CH = 0;
    int64_t ldb = 0, gblk = 0, oblk = 0;
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

// cos(k pi x / y) and sin(k pi x / y) with the argument reduced exactly to
// [0, pi/2] through integer arithmetic (x k mod 2y).
void cossin_pi_ratio(int64_t num, int64_t den, double &c, double &s)
{
    int64_t a = num % (2 * den);  // angle = pi a / den in [0, 2 pi)
    double sc = 1.0, ss = 1.0;
    if (a >= den) {  // pi + b: cos -> -cos, sin -> -sin
        a -= den;
        sc = -sc;
        ss = -ss;
    }
    if (2 * a > den) {  // pi - b: cos -> -cos, sin -> sin
        a = den - a;
        sc = -sc;
    }
    if (a == 0) {
        c = sc;
        s = 0.0;
    } else if (2 * a == den) {
        c = 0.0;
        s = ss;
    } else {
        const double ang = M_PI * (double)a / (double)den;
        c = sc * std::cos(ang);
        s = ss * std::sin(ang);
    }
}

int rup(int x, int a) { return (x + a - 1) / a * a; }
int64_t rup64(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

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

// Raise a kernel's dynamic-LDS limit to at least `bytes` (never lower it: an
// object created earlier with larger transforms keeps launching).
void set_smem_attr(const void *k, size_t bytes)
{
    static std::vector<std::pair<const void *, size_t>> seen;
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    for (auto &e : seen)
        if (e.first == k) {
            if (bytes <= e.second) return;
            e.second = bytes;
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            return;
        }
    seen.emplace_back(k, bytes);
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
    void *ps[] = {h->tw, h->Af, h->V, h->a_off, h->v_off, h->z_off, h->a_rows, h->z_kpad, h->items_f, h->items_i,
                  h->Gb, h->Bz, h->Ob, h->chunk_l};
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
    Plan Pphi;
    if (nphi > MAXN || !make_plan(nphi, Pphi)) {
        snprintf(g_sht_error, sizeof(g_sht_error), "FFT length N_phi = %d must be a product of 2, 3 and 5, at most %d",
                 nphi, MAXN);
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
    h->H = (ntheta + 1) / 2;
    h->tmax = tmax;
    h->tmaxpad = rup(tmax, GBN / 2);
    h->Pphi = Pphi;
    h->nseq = std::max(1, std::min(8, NTH * MAXV / nphi));
    h->ldb = 2 * (int64_t)h->tmaxpad;
    h->kph = rup(h->H, GBK);
    h->vrows = rup64(h->H, GBM);
    h->gblk = (int64_t)h->kph * h->ldb;
    h->oblk = h->vrows * h->ldb;
    const int H = h->H;

    // block geometry per (m, p): degrees l = lstart(m,p) + 2r, r < R
    const int nb = 2 * L;
    std::vector<int64_t> a_off(nb), v_off(nb), z_off(nb);
    std::vector<int> a_rows(nb), z_kpad(nb);
    std::vector<Item> items_f, items_i;
    const int kc = rup((L + 1) / 2, 2), rc = rup((L + 1) / 2, 2);  // row lengths of the temporary tables
    int64_t asz = 0, vsz = 0, zsz = 0;
    for (int m = 0; m < L; ++m)
        for (int p = 0; p < 2; ++p) {
            const int i = 2 * m + p, l0 = lstart(m, p);
            const int R = l0 < L ? (L - 1 - l0) / 2 + 1 : 0;
            a_rows[i] = rup(std::max(R, 1), GBM);
            a_off[i] = asz;
            asz += (int64_t)a_rows[i] * h->kph;
            z_kpad[i] = rup(std::max(R, 1), GBK);
            v_off[i] = vsz;
            vsz += (int64_t)z_kpad[i] * h->vrows;
            z_off[i] = zsz;
            zsz += (int64_t)z_kpad[i] * h->ldb;
            if (R > 0) {
                for (int tm = 0; tm < a_rows[i] / GBM; ++tm) items_f.push_back(Item{(int16_t)m, (int16_t)p, tm});
                for (int tm = 0; tm < h->vrows / GBM; ++tm) items_i.push_back(Item{(int16_t)m, (int16_t)p, tm});
            }
        }
    h->nitems_f = (int)items_f.size();
    h->nitems_i = (int)items_i.size();
    // f transposes: chunks of whole degrees of at most CH coefficients, TT time
    // steps per workgroup, TT * CH doubles of LDS (64 KB)
    h->CH = std::max(1024, rup(2 * L - 1, 256));
    h->TT = std::max(1, 8192 / h->CH);
    std::vector<int> chunk_l{0};
    for (int l = 0; l < L; ++l) {
        const int la = chunk_l.back();
        if ((l + 1) * (l + 1) - la * la > h->CH) chunk_l.push_back(l);
    }
    chunk_l.push_back(L);
    h->nchunk = (int)chunk_l.size() - 1;
    // colatitude weights of the composition, [m mod 2][m'][j']
    std::vector<double> kap(2 * (size_t)L * H), lam(2 * (size_t)L * H);
    for (int mp = 0; mp < L; ++mp)
        for (int jp = 0; jp < H; ++jp) {
            double c, s;
            cossin_pi_ratio((int64_t)mp * jp, ntheta - 1, c, s);  // m' theta_j' = pi m' j' / (N_theta - 1)
            const size_t e = (size_t)mp * H + jp, o = (size_t)L * H + e;
            kap[e] = jp == 0 ? 1.0 : 2.0 * c;
            kap[o] = jp == 0 ? 0.0 : 2.0 * s;
            lam[e] = mp == 0 ? 1.0 : 2.0 * c;
            lam[o] = mp == 0 ? 0.0 : 2.0 * s;
        }

    size_t tb = 0, wb = 0, scratch = 0;
    int rc_ = MPCHOL_OK;
    auto chk = [&](int r) {
        if (rc_ == MPCHOL_OK) rc_ = r;
    };
    double *D = nullptr, *Wt = nullptr, *St = nullptr, *kap_d = nullptr, *lam_d = nullptr;
    const int64_t wblk = (int64_t)rup((L + 1) / 2, 1) * kc, sblk = (int64_t)rup((L + 1) / 2, 1) * rc;
    chk(dmalloc(&h->tw, nphi * sizeof(double2), tb));
    chk(dmalloc(&h->Af, asz * 8, tb));
    chk(dmalloc(&h->V, vsz * 8, tb));
    chk(dmalloc(&h->a_off, nb * 8, tb));
    chk(dmalloc(&h->v_off, nb * 8, tb));
    chk(dmalloc(&h->z_off, nb * 8, tb));
    chk(dmalloc(&h->a_rows, nb * 4, tb));
    chk(dmalloc(&h->z_kpad, nb * 4, tb));
    chk(dmalloc(&h->items_f, std::max<size_t>(1, items_f.size()) * sizeof(Item), tb));
    chk(dmalloc(&h->items_i, std::max<size_t>(1, items_i.size()) * sizeof(Item), tb));
    chk(dmalloc(&h->Gb, (size_t)nb * h->gblk * 8, wb));
    chk(dmalloc(&h->Bz, zsz * 8, wb));
    chk(dmalloc(&h->Ob, (size_t)nb * h->oblk * 8, wb));
    chk(dmalloc(&h->chunk_l, chunk_l.size() * 4, tb));
    chk(dmalloc(&D, (size_t)wig_off(L) * 8, scratch));
    chk(dmalloc(&Wt, (size_t)nb * wblk * 8, scratch));
    chk(dmalloc(&St, (size_t)nb * sblk * 8, scratch));
    chk(dmalloc(&kap_d, kap.size() * 8, scratch));
    chk(dmalloc(&lam_d, lam.size() * 8, scratch));
    h->table_bytes = tb;
    h->work_bytes = wb;
    auto free_tmp = [&]() {
        void *ts[] = {D, Wt, St, kap_d, lam_d};
        for (void *p : ts)
            if (p) (void)hipFree(p);
    };
    if (rc_ != MPCHOL_OK) {
        snprintf(g_sht_error, sizeof(g_sht_error), "device allocation failed (tables %zu B, work %zu B)", tb, wb);
        free_tmp();
        mpchol_sht_destroy(h);
        return rc_;
    }
    hipStream_t st = h->st;
    // zero padding: padded K rows/columns of tables and operands must be zero,
    // and result blocks of (m, p) without any degree (m = L - 1, one parity)
    // are read as zero by the longitude kernel
    bool ok = hipMemsetAsync(h->Af, 0, asz * 8, st) == hipSuccess && hipMemsetAsync(h->V, 0, vsz * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Gb, 0, (size_t)nb * h->gblk * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Bz, 0, zsz * 8, st) == hipSuccess &&
              hipMemsetAsync(h->Ob, 0, (size_t)nb * h->oblk * 8, st) == hipSuccess;
    const std::vector<double2> twp = twiddles(nphi);
    if (ok)
        ok = upload(h->tw, twp, st) == MPCHOL_OK && upload(h->a_off, a_off, st) == MPCHOL_OK &&
             upload(h->v_off, v_off, st) == MPCHOL_OK && upload(h->z_off, z_off, st) == MPCHOL_OK &&
             upload(h->a_rows, a_rows, st) == MPCHOL_OK && upload(h->z_kpad, z_kpad, st) == MPCHOL_OK &&
             upload(h->items_f, items_f, st) == MPCHOL_OK && upload(h->items_i, items_i, st) == MPCHOL_OK &&
             upload(h->chunk_l, chunk_l, st) == MPCHOL_OK &&
             upload(kap_d, kap, st) == MPCHOL_OK && upload(lam_d, lam, st) == MPCHOL_OK;
    if (ok) {
        const int64_t nlm = (int64_t)L * (L + 1) / 2;
        wigner_kernel<<<(unsigned)((nlm + 255) / 256), 256, 0, st>>>(L, D);
        const int64_t half = (L + 1) / 2;
        dim3 gt((unsigned)((half * half + 255) / 256), (unsigned)nb);
        folded_table_kernel<<<gt, 256, 0, st>>>(L, D, Wt, wblk, kc);
        s_table_kernel<<<gt, 256, 0, st>>>(L, D, St, sblk, rc);
        dim3 gc((unsigned)((half * H + 255) / 256), (unsigned)nb);
        compose_forward_kernel<<<gc, 256, 0, st>>>(L, ntheta, Wt, wblk, kc, kap_d, h->Af, h->a_off, h->a_rows);
        compose_inverse_kernel<<<gc, 256, 0, st>>>(L, ntheta, St, sblk, rc, lam_d, h->V, h->v_off, h->vrows);
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    }
    free_tmp();
    if (!ok) {
        snprintf(g_sht_error, sizeof(g_sht_error), "table set-up failed: %s", hipGetErrorString(hipGetLastError()));
        mpchol_sht_destroy(h);
        return MPCHOL_EHIP;
    }
    set_smem_attr((const void *)phi_forward_kernel, fft_smem(nphi, h->nseq));
    set_smem_attr((const void *)phi_inverse_kernel, fft_smem(nphi, h->nseq));
    set_smem_attr((const void *)gemm_forward_kernel, GS::SMEM);
    set_smem_attr((const void *)gemm_inverse_kernel, GS::SMEM);
    set_smem_attr((const void *)unpack_forward_kernel, (size_t)h->TT * h->CH * 8);
    set_smem_attr((const void *)pack_inverse_kernel, (size_t)h->TT * h->CH * 8);
    *out = h;
    return MPCHOL_OK;
}

int mpchol_sht_info(mpchol_sht_t h, int64_t *table_bytes, int64_t *work_bytes, int64_t *gemm_flops_per_step)
{
    if (!h) return MPCHOL_EINVAL;
    if (table_bytes) *table_bytes = (int64_t)h->table_bytes;
    if (work_bytes) *work_bytes = (int64_t)h->work_bytes;
    if (gemm_flops_per_step) {
        // unpadded: per (m, p) degrees x northern colatitudes x 2 columns x 2 flops
        int64_t fl = 0;
        for (int m = 0; m < h->L; ++m)
            for (int p = 0; p < 2; ++p) {
                const int l0 = lstart(m, p);
                const int64_t R = l0 < h->L ? (h->L - 1 - l0) / 2 + 1 : 0;
                fl += 4 * R * h->H;
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
    const int64_t nsq = (int64_t)h->H * T;
    phi_forward_kernel<<<(unsigned)((nsq + h->nseq - 1) / h->nseq), NTH, fft_smem(h->nph, h->nseq), st>>>(
        Z, (int)T, h->nth, h->L, h->Pphi, h->tw, h->Gb, h->gblk, h->ldb, h->nseq);
    dim3 gg((unsigned)h->nitems_f, (unsigned)(2 * Tpad / GBN));
    gemm_forward_kernel<<<gg, GS::NTH, GS::SMEM, st>>>(h->Af, h->a_off, h->a_rows, h->Gb, h->gblk, h->ldb, h->kph,
                                                       h->items_f, h->Ob, h->oblk);
    dim3 gu((unsigned)h->nchunk, (unsigned)((T + h->TT - 1) / h->TT));
    unpack_forward_kernel<<<gu, TNT, (size_t)h->TT * h->CH * 8, st>>>(h->Ob, h->oblk, h->ldb, h->chunk_l, (int)T,
                                                                      h->L, h->TT, h->CH, f);
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
    dim3 gp((unsigned)h->nchunk, (unsigned)((T + h->TT - 1) / h->TT));
    pack_inverse_kernel<<<gp, TNT, (size_t)h->TT * h->CH * 8, st>>>(f, h->chunk_l, (int)T, h->L, h->TT, h->CH, h->Bz,
                                                                    h->z_off, h->ldb);
    dim3 gg((unsigned)h->nitems_i, (unsigned)(2 * Tpad / GBN));
    gemm_inverse_kernel<<<gg, GS::NTH, GS::SMEM, st>>>(h->V, h->v_off, h->vrows, h->z_kpad, h->Bz, h->z_off, h->ldb,
                                                       h->items_i, h->Ob, h->oblk);
    const int64_t nsq = (int64_t)h->H * T;
    phi_inverse_kernel<<<(unsigned)((nsq + h->nseq - 1) / h->nseq), NTH, fft_smem(h->nph, h->nseq), st>>>(
        h->Ob, h->oblk, h->ldb, (int)T, h->nth, h->L, h->Pphi, h->tw, Z, h->nseq);
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

}  // extern "C"
