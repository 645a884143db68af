/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the mixed-precision tile Cholesky of the
 * spherical-harmonic covariance (paper Sec. III.A.3, Sec. III.D, Sec. V.A).
 * Only tests/, the package's smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP path and must never
 * be called by it.
 *
 * Conventions: column-major storage, lower-triangular factors, FP64 unless a
 * function says otherwise, 0-based indices.  Every function follows the
 * plain definition of what it computes, or the tile algorithm's steps in the
 * paper's order (POTRF, TRSM, sender-side conversion, SYRK/GEMM; Sec. V.A).
 *
 * Parity status of each group is stated in its header comment.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_F64 0
#define ORC_F32 1
#define ORC_BF16 2
#define ORC_F16 3
#define ORC_E4M3 4

/* precision classes of a tile (the map's codes) */
#define ORC_P64 0
#define ORC_P32 1
#define ORC_P16 2
#define ORC_P8 3

/* ------------------------------------------------------------------------
 * Workload entries.  Exponential (Markov) kernel on the ordered coordinate
 * of the coefficient index, scaled by sigma, with a diagonal perturbation
 * that keeps the matrix positive definite (Sec. III.A.3 adds such a
 * perturbation when the sample covariance is rank deficient).
 * Pinned by: symmetric, unit-correlation diagonal, closed forms below.
 * ---------------------------------------------------------------------- */
double orc_cov_entry(const double *sigma, const double *x, double rho, double nugget, int64_t i, int64_t j)
{
    double v = sigma[i] * sigma[j] * exp(-fabs(x[i] - x[j]) / rho);
    if (i == j) v += nugget;
    return v;
}

void orc_cov_dense(int64_t n, const double *sigma, const double *x, double rho, double nugget, double *A, int64_t lda)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            A[i + j * lda] = orc_cov_entry(sigma, x, rho, nugget, i, j);
}

/* ------------------------------------------------------------------------
 * Covariance from samples (the estimator of the residual covariance in Sec.
 * III.A.3, "Modeling the Temporal Dependence and Constructing a Covariance
 * Matrix": the average of the outer products of the R(T-P) residual vectors,
 * plus a small diagonal perturbation when there are fewer samples than L^2):
 *   S_ij = scale * sum_k xi_ik xi_jk + nugget * delta_ij,
 * xi column-major n x m (leading dimension ldxi), terms summed in k order,
 * S full (both triangles) column-major.
 * Pinned by: xi = [I 0] (S = (scale + nugget) I), a rank-one xi (closed
 * form), and xi = L0 H with a Sylvester-Hadamard H (H H^T = m I): with
 * scale = 1/m, S = L0 L0^T exactly.
 * ---------------------------------------------------------------------- */
void orc_cov_samples(int64_t n, int64_t m, const double *xi, int64_t ldxi, double scale, double nugget, double *S,
                     int64_t lds)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = 0; k < m; ++k) acc += xi[i + k * ldxi] * xi[j + k * ldxi];
            double v = scale * acc + ((i == j) ? nugget : 0.0);
            S[i + j * lds] = v;
            S[j + i * lds] = v;
        }
}

/* ------------------------------------------------------------------------
 * O1: exact FP64 Cholesky, A = L L^T with L lower and positive diagonal
 * (the factorization of Sec. III.A.3).  Right-looking, one column at a time:
 *   L_kk = sqrt(A_kk); L_ik = A_ik / L_kk; A_ij -= L_ik L_jk (i >= j > k).
 * Returns 0, or the 1-based column of the first non-positive pivot
 * (LAPACK potrf convention).  The strict upper part is set to zero.
 * Pinned by: brute-force 2x2/3x3 factors, L0 L0^T with integer L0, the
 * Markov closed form, LAPACK dpotrf.
 * ---------------------------------------------------------------------- */
int64_t orc_potrf(int64_t n, double *A, int64_t lda)
{
    for (int64_t k = 0; k < n; ++k) {
        double d = A[k + k * lda];
        if (!(d > 0.0)) return k + 1;
        double lkk = sqrt(d);
        A[k + k * lda] = lkk;
        for (int64_t i = k + 1; i < n; ++i) A[i + k * lda] /= lkk;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t j = k + 1; j < n; ++j) {
            double ljk = A[j + k * lda];
            double *cj = A + j * lda;
            const double *ck = A + k * lda;
            for (int64_t i = j; i < n; ++i) cj[i] -= ck[i] * ljk;
        }
    }
    for (int64_t j = 1; j < n; ++j)
        for (int64_t i = 0; i < j; ++i) A[i + j * lda] = 0.0;
    return 0;
}

/* OpenMP threads the oracle's parallel loops use. */
int orc_threads(void) { return omp_get_max_threads(); }

/* log det(A) = 2 * sum_i log L_ii, summed in index order. */
double orc_logdet(int64_t n, const double *L, int64_t ldl)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += log(L[i + i * ldl]);
    return 2.0 * s;
}

/* Solve A X = B with A = L L^T: forward substitution L y = b, then backward
 * substitution L^T x = y, column by column of B (overwritten by X). */
void orc_potrs(int64_t n, const double *L, int64_t ldl, int64_t nrhs, double *B, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + r * ldb;
        /* forward: b_i = (b_i - sum_{k<i} l_ik y_k) / l_ii, terms taken in k order */
        for (int64_t k = 0; k < n; ++k) {
            b[k] /= L[k + k * ldl];
            for (int64_t i = k + 1; i < n; ++i) b[i] -= L[i + k * ldl] * b[k];
        }
        /* backward: x_i = (y_i - sum_{k>i} l_ki x_k) / l_ii */
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int64_t k = i + 1; k < n; ++k) s -= L[k + i * ldl] * b[k];
            b[i] = s / L[i + i * ldl];
        }
    }
}

/* Residual of a factor: returns ||A - L L^T||_F over the full symmetric
 * matrix; ||A||_F goes to *anorm.  Entry by entry:
 *   r_ij = a_ij - sum_{k <= min(i,j)} l_ik l_jk. */
double orc_residual_fro(int64_t n, const double *A, int64_t lda, const double *L, int64_t ldl, double *anorm)
{
    double rs = 0.0, as = 0.0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : rs, as)
    for (int64_t j = 0; j < n; ++j) {
        double *s = calloc((size_t)n, sizeof(double));
        /* s_i = sum_{k <= j} l_ik l_jk for i >= j, terms taken in k order */
        for (int64_t k = 0; k <= j; ++k) {
            double ljk = L[j + k * ldl];
            for (int64_t i = j; i < n; ++i) s[i] += L[i + k * ldl] * ljk;
        }
        for (int64_t i = j; i < n; ++i) {
            double a = A[i + j * lda];
            double r = a - s[i];
            double w = (i == j) ? 1.0 : 2.0;
            rs += w * r * r;
            as += w * a * a;
        }
        free(s);
    }
    if (anorm) *anorm = sqrt(as);
    return sqrt(rs);
}

/* Squared Frobenius norm of the residual per b x b tile (I, J), I >= J,
 * written to out[I + J*nt] (strict-lower entries of a diagonal tile count
 * twice, as in the full symmetric matrix); rows/columns < n only. */
void orc_tile_residual2(int64_t n, int64_t b, const double *A, int64_t lda, const double *L, int64_t ldl, double *out)
{
    int64_t nt = (n + b - 1) / b;
    double *colsum = calloc((size_t)n * nt, sizeof(double));
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j) {
        double *s = calloc((size_t)n, sizeof(double));
        for (int64_t k = 0; k <= j; ++k) {
            double ljk = L[j + k * ldl];
            for (int64_t i = j; i < n; ++i) s[i] += L[i + k * ldl] * ljk;
        }
        for (int64_t i = j; i < n; ++i) {
            double r = A[i + j * lda] - s[i];
            colsum[j + (i / b) * n] += (i == j ? 1.0 : ((i / b) == (j / b) ? 2.0 : 1.0)) * r * r;
        }
        free(s);
    }
    for (int64_t t = 0; t < nt * nt; ++t) out[t] = 0.0;
    for (int64_t I = 0; I < nt; ++I)
        for (int64_t j = 0; j < n; ++j) {
            int64_t J = j / b;
            if (I >= J) out[I + J * nt] += colsum[j + I * n];
        }
    free(colsum);
}

/* Y = L Z for lower-triangular L (n x n) and Z (n x m), FP64; each y_i sums
 * l_ik z_k in k order. */
void orc_lower_matmul(int64_t n, const double *L, int64_t ldl, int64_t m, const double *Z, int64_t ldz, double *Y, int64_t ldy)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < m; ++c) {
        double *y = Y + c * ldy;
        for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double zk = Z[k + c * ldz];
            for (int64_t i = k; i < n; ++i) y[i] += L[i + k * ldl] * zk;
        }
    }
}

/* ------------------------------------------------------------------------
 * Closed forms of the exponential (Markov) kernel on sorted coordinates,
 * Sigma = D K D + delta I with D = diag(sigma), K_ij = exp(-|x_i - x_j|/rho).
 * With a_j = exp(-(x_j - x_{j-1})/rho), s_0 = 1, s_j = sqrt(1 - a_j^2):
 *   chol(D K D)_ij = sigma_i exp(-(x_i - x_j)/rho) s_j          (i >= j)
 *   K^-1 = T tridiagonal, T_jj = 1/s_j^2 + a_{j+1}^2/s_{j+1}^2,
 *          T_{j,j+1} = -a_{j+1}/s_{j+1}^2   (terms past n-1 dropped)
 *   logdet(Sigma) = N log delta + logdet(D^2/delta + T) + sum_j log s_j^2
 *   Sigma^-1 b = D^-1 T (D^2/delta + T)^-1 (D b / delta)
 * and for delta = 0: logdet = 2 sum log sigma + sum log s_j^2, x = D^-1 T D^-1 b.
 * The tridiagonal systems use an LDL^T recurrence (SPD, no pivoting).
 * These are the independent pins of the factor, logdet and solve at every
 * size of the workload.
 * ---------------------------------------------------------------------- */
static double mk_a(const double *x, double rho, int64_t j) { return exp(-(x[j] - x[j - 1]) / rho); }

double orc_markov_L(const double *sigma, const double *x, double rho, int64_t i, int64_t j)
{
    if (i < j) return 0.0;
    double sj = 1.0;
    if (j > 0) {
        double a = mk_a(x, rho, j);
        sj = sqrt(1.0 - a * a);
    }
    return sigma[i] * exp(-(x[i] - x[j]) / rho) * sj;
}

/* log(1 - a_j^2) = log(s_j^2), computed as log(-expm1(-2 dx / rho)) for accuracy */
static double mk_logs2(const double *x, double rho, int64_t j) { return log(-expm1(-2.0 * (x[j] - x[j - 1]) / rho)); }
static double mk_s2(const double *x, double rho, int64_t j) { return -expm1(-2.0 * (x[j] - x[j - 1]) / rho); }

/* Diagonal and super-diagonal of T = K^-1. */
static void mk_T(int64_t n, const double *x, double rho, double *td, double *te)
{
    for (int64_t j = 0; j < n; ++j) {
        double inv_s2 = (j == 0) ? 1.0 : 1.0 / mk_s2(x, rho, j);
        double nxt = 0.0;
        if (j + 1 < n) {
            double a = mk_a(x, rho, j + 1);
            nxt = a * a / mk_s2(x, rho, j + 1);
            te[j] = -a / mk_s2(x, rho, j + 1);
        }
        td[j] = inv_s2 + nxt;
    }
}

double orc_markov_logdet(int64_t n, const double *sigma, const double *x, double rho, double nugget)
{
    double s = 0.0;
    for (int64_t j = 1; j < n; ++j) s += mk_logs2(x, rho, j);
    if (nugget == 0.0) {
        for (int64_t i = 0; i < n; ++i) s += 2.0 * log(sigma[i]);
        return s;
    }
    double *td = malloc(sizeof(double) * n), *te = malloc(sizeof(double) * n);
    mk_T(n, x, rho, td, te);
    double ld = 0.0, dprev = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double m = sigma[j] * sigma[j] / nugget + td[j];
        double d = (j == 0) ? m : m - te[j - 1] * te[j - 1] / dprev;
        ld += log(d);
        dprev = d;
    }
    free(td);
    free(te);
    return s + (double)n * log(nugget) + ld;
}

void orc_markov_solve(int64_t n, const double *sigma, const double *x, double rho, double nugget, int64_t nrhs, double *B, int64_t ldb)
{
    double *td = malloc(sizeof(double) * n), *te = malloc(sizeof(double) * n);
    double *dd = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    mk_T(n, x, rho, td, te);
    if (nugget != 0.0) {
        for (int64_t j = 0; j < n; ++j) {
            double m = sigma[j] * sigma[j] / nugget + td[j];
            dd[j] = (j == 0) ? m : m - te[j - 1] * te[j - 1] / dd[j - 1];
        }
    }
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + r * ldb;
        if (nugget != 0.0) {
            /* w = D b / delta, then w = M^-1 w with M = L D L^T tridiagonal */
            for (int64_t j = 0; j < n; ++j) w[j] = sigma[j] * b[j] / nugget;
            for (int64_t j = 1; j < n; ++j) w[j] -= (te[j - 1] / dd[j - 1]) * w[j - 1];
            for (int64_t j = 0; j < n; ++j) w[j] /= dd[j];
            for (int64_t j = n - 2; j >= 0; --j) w[j] -= (te[j] / dd[j]) * w[j + 1];
        } else {
            for (int64_t j = 0; j < n; ++j) w[j] = b[j] / sigma[j];
        }
        /* b = D^-1 T w */
        for (int64_t j = 0; j < n; ++j) {
            double s = td[j] * w[j];
            if (j > 0) s += te[j - 1] * w[j - 1];
            if (j + 1 < n) s += te[j] * w[j + 1];
            b[j] = s / sigma[j];
        }
    }
    free(td);
    free(te);
    free(dd);
    free(w);
}

/* ------------------------------------------------------------------------
 * Floating-point formats of the precision classes (Sec. III.D: DP, SP, HP;
 * FP8 is OCP E4M3FN).  A format is (p significand bits incl. the hidden
 * one, minimum normal exponent emin, largest finite value).  Rounding is
 * round-to-nearest, ties to even, with gradual underflow; values beyond the
 * largest finite one saturate (E4M3FN has no infinity) or become infinity.
 * Pinned by: numpy's float32/float16 casts, brute force over every E4M3FN
 * code decoded from the bit definition, bf16 brute force on sampled inputs.
 * ---------------------------------------------------------------------- */
static void fmt_params(int fmt, int *p, int *emin, double *maxf, int *sat)
{
    switch (fmt) {
    case ORC_F32: *p = 24; *emin = -126; *maxf = ldexp(2.0 - ldexp(1.0, -23), 127); *sat = 0; break;
    case ORC_BF16: *p = 8; *emin = -126; *maxf = ldexp(2.0 - ldexp(1.0, -7), 127); *sat = 0; break;
    case ORC_F16: *p = 11; *emin = -14; *maxf = 65504.0; *sat = 0; break;
    case ORC_E4M3: *p = 4; *emin = -6; *maxf = 448.0; *sat = 1; break;
    default: *p = 53; *emin = -1022; *maxf = INFINITY; *sat = 0; break;
    }
}

double orc_round(double v, int fmt)
{
    if (fmt == ORC_F64 || v == 0.0 || !isfinite(v)) return v;
    int p, emin, sat;
    double maxf;
    fmt_params(fmt, &p, &emin, &maxf, &sat);
    double a = fabs(v);
    int e = ilogb(a);
    if (e < emin) e = emin;
    double ulp = ldexp(1.0, e - (p - 1));
    double q = a / ulp;          /* exact: division by a power of two */
    double r = nearbyint(q);     /* ties to even in the default rounding mode */
    double res = r * ulp;
    if (res > maxf) res = sat ? maxf : INFINITY;
    return copysign(res, v);
}

/* Value of an E4M3FN byte from the format's bit definition:
 * sign s, exponent e (4 bits, bias 7), mantissa m (3 bits);
 * e = 0: subnormal m/8 * 2^-6; e = 15 and m = 7: NaN; else (1 + m/8) 2^(e-7). */
double orc_e4m3_decode(uint8_t code)
{
    int s = code >> 7, e = (code >> 3) & 15, m = code & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = (m / 8.0) * ldexp(1.0, -6);
    else v = (1.0 + m / 8.0) * ldexp(1.0, e - 7);
    return s ? -v : v;
}

double orc_unit_roundoff(int fmt)
{
    switch (fmt) {
    case ORC_F32: return ldexp(1.0, -24);
    case ORC_BF16: return ldexp(1.0, -8);
    case ORC_F16: return ldexp(1.0, -11);
    case ORC_E4M3: return ldexp(1.0, -4);
    default: return ldexp(1.0, -53);
    }
}

/* Per-tile power-of-two scale for the narrow-range formats: the largest
 * integer t with amax * 2^t <= largest finite value.  FP16 and E4M3 are
 * scaled; FP64, FP32 and BF16 (FP32's exponent range) use t = 0, as does an
 * all-zero tile, and a tile whose maximum is not finite (no such t exists). */
int orc_scale_exp(double amax, int fmt)
{
    if (!(fmt == ORC_F16 || fmt == ORC_E4M3) || !(amax > 0.0) || !isfinite(amax)) return 0;
    double maxf = (fmt == ORC_F16) ? 65504.0 : 448.0;
    int t = ilogb(maxf) - ilogb(amax);
    while (ldexp(amax, t) > maxf) --t;
    while (ldexp(amax, t + 1) <= maxf) ++t;
    return t;
}

/* ------------------------------------------------------------------------
 * Block-scaled FP8 copies, after the OCP Microscaling formats: one shared
 * power-of-two scale per block of 32 consecutive elements -- here the
 * elements of a row along the K direction of the products that read the
 * copy.  Block exponent: t = orc_scale_exp(block max |v|, E4M3) clamped to
 * [-127, 127] (the range of an E8M0 scale), so no element saturates; each
 * element becomes round_e4m3(round_f32(v 2^t)) and represents that code
 * times 2^-t.  (The OCP recipe takes floor(log2 max) - 8 and saturates
 * elements above 448; the choice here is the per-tile rule applied per
 * block.)
 * Pinned by: brute force of the exponent choice; exactness for values of at
 * most four significant bits at any exponent per block; equality with the
 * per-tile copy when every block holds the tile's maximum; the per-element
 * E4M3 rounding bound.
 * ---------------------------------------------------------------------- */
int orc_mx_block_exp(double amax)
{
    int t = orc_scale_exp(amax, ORC_E4M3);
    return t < -127 ? -127 : (t > 127 ? 127 : t);
}

/* X: rows x cols (column-major, leading dimension ld); the last block of a
 * row is shorter when cols is not a multiple of 32.  out (leading dimension
 * ldo) = the represented values of the copy; texp (optional)
 * [r + (c / 32) * rows] = the block exponents. */
void orc_mx_quantize(int64_t rows, int64_t cols, const double *X, int64_t ld, double *out, int64_t ldo, int32_t *texp)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c0 = 0; c0 < cols; c0 += 32) {
            const int64_t ce = c0 + 32 < cols ? c0 + 32 : cols;
            double m = 0.0;
            for (int64_t c = c0; c < ce; ++c)
                if (fabs(X[r + c * ld]) > m) m = fabs(X[r + c * ld]);
            int t = orc_mx_block_exp(m);
            if (texp) texp[r + (c0 / 32) * rows] = t;
            for (int64_t c = c0; c < ce; ++c)
                out[r + c * ldo] = ldexp(orc_round((double)(float)ldexp(X[r + c * ld], t), ORC_E4M3), -t);
        }
}

/* ------------------------------------------------------------------------
 * Precision maps (Sec. III.D tile-centric and band-based mixed precision).
 * Norm rule: tile (I,J), I > J, takes the lowest allowed class p with
 *   ||Sigma_IJ||_F * u_p <= eps * ||Sigma||_F / NT,
 * tiles with |I - J| <= band stay FP64, the diagonal is always FP64.
 * Classes: 0 FP64, 1 FP32, 2 16-bit (BF16 or FP16), 3 FP8 E4M3.
 * ---------------------------------------------------------------------- */
static int class_fmt(int cls, int lo16)
{
    switch (cls) {
    case ORC_P32: return ORC_F32;
    case ORC_P16: return lo16;
    case ORC_P8: return ORC_E4M3;
    default: return ORC_F64;
    }
}

/* Tile Frobenius norms squared and max-abs over the valid part of the
 * lower tiles: fro2[I + J*nt], amax[I + J*nt]; returns ||A||_F of the full
 * symmetric matrix (strict-lower tiles counted twice). */
double orc_tile_norms(int64_t n, int64_t b, const double *A, int64_t lda, double *fro2, double *amax)
{
    int64_t nt = (n + b - 1) / b;
    double tot = 0.0;
    for (int64_t J = 0; J < nt; ++J)
        for (int64_t I = 0; I < nt; ++I) {
            double s = 0.0, m = 0.0;
            if (I >= J)
                for (int64_t j = J * b; j < (J + 1) * b && j < n; ++j)
                    for (int64_t i = I * b; i < (I + 1) * b && i < n; ++i) {
                        double a = A[i + j * lda];
                        s += a * a;
                        if (fabs(a) > m) m = fabs(a);
                    }
            fro2[I + J * nt] = s;
            amax[I + J * nt] = m;
            if (I > J) tot += 2.0 * s;
            else if (I == J) tot += s;
        }
    return sqrt(tot);
}

void orc_map_norm(int64_t nt, const double *fro2, double total_fro, double eps, int band, unsigned allowed, int lo16, uint8_t *map)
{
    double thr = eps * total_fro / (double)nt;
    for (int64_t J = 0; J < nt; ++J)
        for (int64_t I = 0; I < nt; ++I) {
            uint8_t c = ORC_P64;
            if (I > J && (I - J) > band) {
                double f = sqrt(fro2[I + J * nt]);
                for (int cls = ORC_P8; cls >= ORC_P32; --cls) {
                    if (!(allowed & (1u << cls))) continue;
                    if (f * orc_unit_roundoff(class_fmt(cls, lo16)) <= thr) { c = (uint8_t)cls; break; }
                }
            }
            map[I + J * nt] = (I >= J) ? c : 0;
        }
}

/* Band rule (Sec. IV.B's precision variants DP/SP, DP/SP/HP and DP/HP; the
 * band-based mixed precision of Sec. III.D).  Tiles with I - J <= band (the
 * diagonal included) are FP64.  variant 1 (DP/SP): every other lower tile
 * FP32; variant 3 (DP/HP): every other lower tile 16-bit; variant 2
 * (DP/SP/HP): tiles with band < I - J <= w32 FP32 and the rest 16-bit, where
 * w32 is the smallest width whose FP32 band holds at least 5% of the
 * nt(nt-1)/2 strict-lower tiles (every off-band tile when no width reaches
 * it).  A class outside `allowed` is raised to the nearest more precise
 * allowed class (FP64 is always allowed).  The 5% count visits the tiles
 * one by one. */
void orc_map_band(int64_t nt, int band, int variant, unsigned allowed, uint8_t *map)
{
    const double total = (double)nt * (double)(nt - 1) / 2.0;
    int64_t w32 = band;
    if (variant == 2)
        for (w32 = band; w32 < nt - 1; ++w32) {
            int64_t cnt = 0;
            for (int64_t J = 0; J < nt; ++J)
                for (int64_t I = J + 1; I < nt; ++I)
                    if (I - J > band && I - J <= w32) ++cnt;
            if ((double)cnt >= 0.05 * total) break;
        }
    for (int64_t J = 0; J < nt; ++J)
        for (int64_t I = 0; I < nt; ++I) {
            int c = ORC_P64;
            if (I > J && I - J > band) {
                if (variant == 1) c = ORC_P32;
                else if (variant == 2) c = (I - J <= w32) ? ORC_P32 : ORC_P16;
                else c = ORC_P16;
                while (c > ORC_P64 && !(allowed & (1u << c))) --c;
            }
            map[I + J * nt] = (I >= J) ? (uint8_t)c : 0;
        }
}

/* ------------------------------------------------------------------------
 * FP64-class products emulated with exact integer products (the Ozaki
 * scheme II of Ozaki, Uchino and Imamura: scale each row to integers, form
 * the integer product exactly, scale back).  Definition, for D = A B^T with
 * A (m x k) and B (n x k):
 *   - row r of an operand X: mu_r = max_c |X_rc|; e_r = 0 if mu_r = 0, else
 *     e_r = 53 - E_r with mu_r = f 2^E_r, f in [1/2, 1), so that
 *     mu_r 2^e_r lies in [2^52, 2^53);
 *   - integers x_rc = rint(X_rc 2^e_r) (round to nearest even; |x| <= 2^53);
 *   - P_rs = sum_c a_rc b_sc, exact (here in 128-bit integers: each term is
 *     below 2^106 in magnitude, the sum below 2^116 for k <= 1024);
 *   - D_rs = round_f64(P_rs) 2^-(e_r + f_s), one rounding to nearest even.
 * The integer product does not depend on a summation order; how it is
 * formed (by residues on the GPU) is not part of the definition.
 * Pinned by: brute force with Python integers and its correctly rounded
 * int-to-float conversion (bit for bit, including conversion halfway
 * cases), exactness on integer inputs, and the error bound
 * |D_rs - (A B^T)_rs| <= 2k 2^-53 mu_r nu_s (1 + 2^-52) + |(A B^T)_rs| 2^-53
 * (each scaled entry moves by at most half a unit, 2^-53 of its row max).
 * ---------------------------------------------------------------------- */
static int ozaki_row_exp(double mu)
{
    if (!(mu > 0.0)) return 0;
    int E;
    frexp(mu, &E);
    return 53 - E;
}

/* Row exponent of row r of the column-major block X (len entries, stride ld). */
int orc_ozaki_row_exp(const double *X, int64_t ld, int64_t len)
{
    double mu = 0.0;
    for (int64_t c = 0; c < len; ++c)
        if (fabs(X[c * ld]) > mu) mu = fabs(X[c * ld]);
    return ozaki_row_exp(mu);
}

/* The integer of entry x scaled by 2^e (round to nearest even). */
static int64_t ozaki_int(double x, int e) { return (int64_t)nearbyint(ldexp(x, e)); }

static double ozaki_value(__int128 P, int e)
{
    return ldexp((double)P, -e);  /* the 128-bit to double conversion rounds to nearest even */
}

/* D (m x n, ldd) = A B^T by the definition above; A (m x k, lda), B (n x k, ldb),
 * all column-major. */
void orc_ozaki_gemm(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                    double *D, int64_t ldd)
{
    int64_t *a = malloc(sizeof(int64_t) * (size_t)(m * k + 1)), *bq = malloc(sizeof(int64_t) * (size_t)(n * k + 1));
    int *ea = malloc(sizeof(int) * (size_t)(m + 1)), *eb = malloc(sizeof(int) * (size_t)(n + 1));
    for (int64_t r = 0; r < m; ++r) {
        ea[r] = orc_ozaki_row_exp(A + r, lda, k);
        for (int64_t c = 0; c < k; ++c) a[r * k + c] = ozaki_int(A[r + c * lda], ea[r]);
    }
    for (int64_t s = 0; s < n; ++s) {
        eb[s] = orc_ozaki_row_exp(B + s, ldb, k);
        for (int64_t c = 0; c < k; ++c) bq[s * k + c] = ozaki_int(B[s + c * ldb], eb[s]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s)
        for (int64_t r = 0; r < m; ++r) {
            __int128 P = 0;
            for (int64_t c = 0; c < k; ++c) P += (__int128)a[r * k + c] * bq[s * k + c];
            D[r + s * ldd] = ozaki_value(P, ea[r] + eb[s]);
        }
    free(a);
    free(bq);
    free(ea);
    free(eb);
}

/* ------------------------------------------------------------------------
 * O2: the mixed-precision tile Cholesky replayed on the CPU with explicit
 * rounding (Sec. III.D with the task graph and sender-side conversion of
 * Sec. V.A).  The matrix is padded to NT*b with an identity block.
 *   - Work tiles: FP64 for the diagonal and FP64-class tiles, FP32 (values
 *     rounded to float) for every lower class.
 *   - For k = 0..NT-1:
 *     POTRF(k,k) in FP64 (plain right-looking, as O1);
 *     TRSM(I,k) = W_Ik L_kk^-T by forward substitution in FP64, rounded to
 *       the work precision; a 16-bit/FP8 tile then takes its scale t from
 *       the max |value| and is stored as round_q(round_f32(v * 2^t)) * 2^-t;
 *     conversion at the sender: each panel tile gets one copy per consumer
 *       class: FP64 = stored value; FP32 = round_f32(stored);
 *       16-bit/FP8 = round_q(round_f32(stored * 2^t_q)) with its own scale t_q;
 *     SYRK(I,I) and FP64-class GEMM(I,J): W -= C64_I C64_J^T in FP64;
 *       with lo64 = 1, an FP64-class GEMM of a tile with |I-J| > band64 is
 *       W -= D(C64_I, C64_J), the exact-integer-product emulation defined
 *       above (row scales of each panel tile taken once, at its conversion);
 *       SYRK and the tiles within band64 of the diagonal keep FP64 sums;
 *     FP32-class GEMM: acc = sum of float products (float adds, k order),
 *       W = round_f32(W - acc);
 *       with lo32 = 1 the FP32 operands are split into three BF16 parts,
 *       v = hi + mid + lo (hi = bf16(v), mid = bf16(v - hi), lo = bf16(v - hi
 *       - mid), each step exact in FP32), and acc sums the six significant
 *       part products -- pairs (mid,mid), (hi,lo), (lo,hi), (hi,mid),
 *       (mid,hi), (hi,hi) in this order, each over k -- as exact float
 *       products with float adds (the split-product scheme of Henry, Tang and
 *       Heinecke, ARITH 2019, with the three smallest products dropped);
 *     16-bit/FP8-class GEMM: acc as above on the scaled copies,
 *       W = round_f32(W - acc * 2^-(t_I + t_J));
 *       with lo8 = 1 the FP8 copies are block-scaled (orc_mx_quantize over
 *       the rows of each panel tile) and acc sums the float products of the
 *       represented values, W = round_f32(W - acc).
 * order = 0 sums the update products in increasing c, order = 1 in
 * decreasing c: two valid executions whose difference calibrates how far
 * another summation order (the GPU's) may move the result.
 * Output: Lhat (n x n, the represented values of the stored factor),
 * tscale[I + J*nt] = stored scale exponent of tile (I,J).  Returns 0 or the
 * 1-based global column of a failing pivot.
 * Parity: the HIP path sums in a different order, so agreement is to a
 * rounding-level tolerance, not bitwise.
 * ---------------------------------------------------------------------- */
#define IDX(i, j) ((i) + (size_t)(j) * (size_t)np)

/* Part (0 hi, 1 mid, 2 lo) of the three-way BF16 split of the float value v. */
float orc_split3(double v, int part)
{
    const float f = (float)v;
    const float hi = (float)orc_round(f, ORC_BF16);
    if (part == 0) return hi;
    const float r1 = f - hi;
    const float mid = (float)orc_round(r1, ORC_BF16);
    if (part == 1) return mid;
    return (float)orc_round(r1 - mid, ORC_BF16);
}

int64_t orc_mp_factor(int64_t n, int64_t b, const double *A, int64_t lda, const uint8_t *map, int lo16,
                      double *Lhat, int64_t ldl, int32_t *tscale, int order, int lo32, int lo64, int band64, int lo8)
{
    int64_t nt = (n + b - 1) / b, np = nt * b;
    double *W = malloc(sizeof(double) * (size_t)np * np);
    /* panel copies per consumer class: values (scaled for 16-bit/FP8) */
    double *C[4];
    for (int c = 0; c < 4; ++c) C[c] = malloc(sizeof(double) * (size_t)np * b);
    /* with lo32: the three BF16 parts of each FP32 copy, made once per panel
     * tile at conversion (the same values orc_split3 gives at every use) */
    float *S3[3] = {NULL, NULL, NULL};
    if (lo32)
        for (int p = 0; p < 3; ++p) S3[p] = malloc(sizeof(float) * (size_t)np * b);
    int *tq = malloc(sizeof(int) * nt * 4);
    /* with lo64: the integers and row exponents of each FP64 panel copy */
    int64_t *Z64 = lo64 ? malloc(sizeof(int64_t) * (size_t)np * b) : NULL;
    int *ez = lo64 ? malloc(sizeof(int) * (size_t)np) : NULL;
    int64_t info = 0;

    for (int64_t t = 0; t < nt * nt; ++t) tscale[t] = 0;
    for (int64_t j = 0; j < np; ++j)
        for (int64_t i = 0; i < np; ++i) {
            double v = (i < n && j < n) ? A[i + j * lda] : (i == j ? 1.0 : 0.0);
            int64_t I = i / b, J = j / b;
            if (I > J && map[I + J * nt] != ORC_P64) v = (double)(float)v;
            W[IDX(i, j)] = v;
        }

    for (int64_t k = 0; k < nt && !info; ++k) {
        int64_t k0 = k * b;
        /* POTRF(k,k) */
        for (int64_t c = 0; c < b; ++c) {
            double d = W[IDX(k0 + c, k0 + c)];
            if (!(d > 0.0)) { info = k0 + c + 1; break; }
            double l = sqrt(d);
            W[IDX(k0 + c, k0 + c)] = l;
            for (int64_t i = c + 1; i < b; ++i) W[IDX(k0 + i, k0 + c)] /= l;
            for (int64_t j = c + 1; j < b; ++j)
                for (int64_t i = j; i < b; ++i) W[IDX(k0 + i, k0 + j)] -= W[IDX(k0 + i, k0 + c)] * W[IDX(k0 + j, k0 + c)];
        }
        if (info) break;
        for (int64_t j = 0; j < b; ++j)
            for (int64_t i = 0; i < j; ++i) W[IDX(k0 + i, k0 + j)] = 0.0;

        /* TRSM(I,k) and storage rounding */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t I = k + 1; I < nt; ++I) {
            int cls = map[I + k * nt];
            int64_t i0 = I * b;
            /* x_rc = (w_rc - sum_{cc<c} x_r,cc l_c,cc) / l_cc, terms in cc order */
            for (int64_t c = 0; c < b; ++c) {
                for (int64_t cc = 0; cc < c; ++cc) {
                    double l = W[IDX(k0 + c, k0 + cc)];
                    for (int64_t r = 0; r < b; ++r) W[IDX(i0 + r, k0 + c)] -= W[IDX(i0 + r, k0 + cc)] * l;
                }
                double d = W[IDX(k0 + c, k0 + c)];
                for (int64_t r = 0; r < b; ++r) W[IDX(i0 + r, k0 + c)] /= d;
            }
            if (cls != ORC_P64) {
                double m = 0.0;
                for (int64_t c = 0; c < b; ++c)
                    for (int64_t r = 0; r < b; ++r) {
                        double v = (double)(float)W[IDX(i0 + r, k0 + c)];
                        W[IDX(i0 + r, k0 + c)] = v;
                        if (fabs(v) > m) m = fabs(v);
                    }
                if (cls != ORC_P32) {
                    int fmt = class_fmt(cls, lo16);
                    int t = orc_scale_exp(m, fmt);
                    tscale[I + k * nt] = t;
                    for (int64_t c = 0; c < b; ++c)
                        for (int64_t r = 0; r < b; ++r) {
                            double v = W[IDX(i0 + r, k0 + c)];
                            W[IDX(i0 + r, k0 + c)] = ldexp(orc_round((double)(float)ldexp(v, t), fmt), -t);
                        }
                }
            }
            /* sender-side copies for every consumer class */
            double m = 0.0;
            for (int64_t c = 0; c < b; ++c)
                for (int64_t r = 0; r < b; ++r) {
                    double v = W[IDX(i0 + r, k0 + c)];
                    if (fabs(v) > m) m = fabs(v);
                }
            for (int q = 0; q < 4; ++q) {
                int fmt = class_fmt(q, lo16);
                int t = orc_scale_exp(m, fmt);
                tq[I * 4 + q] = t;
                for (int64_t c = 0; c < b; ++c)
                    for (int64_t r = 0; r < b; ++r) {
                        double v = W[IDX(i0 + r, k0 + c)];
                        double cv;
                        if (q == ORC_P64) cv = v;
                        else if (q == ORC_P32) cv = (double)(float)v;
                        else cv = orc_round((double)(float)ldexp(v, t), fmt);
                        C[q][(i0 + r) + (size_t)c * np] = cv;
                        if (q == ORC_P32 && lo32)
                            for (int p = 0; p < 3; ++p) S3[p][(i0 + r) + (size_t)c * np] = orc_split3(cv, p);
                    }
                if (q == ORC_P8 && lo8) {
                    tq[I * 4 + q] = 0;
                    orc_mx_quantize(b, b, W + IDX(i0, k0), np, C[q] + i0, np, NULL);
                }
            }
            if (lo64)
                for (int64_t r = 0; r < b; ++r) {
                    const double *row = C[ORC_P64] + i0 + r;
                    ez[i0 + r] = orc_ozaki_row_exp(row, np, b);
                    for (int64_t c = 0; c < b; ++c) Z64[(i0 + r) * b + c] = ozaki_int(row[(size_t)c * np], ez[i0 + r]);
                }
        }

        /* SYRK / GEMM updates of the trailing tiles */
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t I = k + 1; I < nt; ++I) {
            for (int64_t J = k + 1; J <= I; ++J) {
                int cls = (I == J) ? ORC_P64 : map[I + J * nt];
                int64_t i0 = I * b, j0 = J * b;
                const double *CI = C[cls], *CJ = C[cls];
                double acc64[b > 0 ? b : 1];
                float acc32[b > 0 ? b : 1];
                for (int64_t s = 0; s < b; ++s) {
                    /* acc_r = sum_c C_I[r,c] C_J[s,c], terms in c order */
                    if (cls == ORC_P64 && lo64 && I - J > band64) {
                        /* exact integer products of the scaled panel rows, one rounding each */
                        const int64_t *bz = Z64 + (j0 + s) * b;
                        for (int64_t r = 0; r < b; ++r) {
                            const int64_t *az = Z64 + (i0 + r) * b;
                            __int128 P = 0;
                            for (int64_t c = 0; c < b; ++c) P += (__int128)az[c] * bz[c];
                            W[IDX(i0 + r, j0 + s)] -= ozaki_value(P, ez[i0 + r] + ez[j0 + s]);
                        }
                    } else if (cls == ORC_P64) {
                        for (int64_t r = 0; r < b; ++r) acc64[r] = 0.0;
                        for (int64_t cc = 0; cc < b; ++cc) {
                            int64_t c = order ? b - 1 - cc : cc;
                            double bj = CJ[(j0 + s) + (size_t)c * np];
                            const double *ci = CI + i0 + (size_t)c * np;
                            for (int64_t r = 0; r < b; ++r) acc64[r] += ci[r] * bj;
                        }
                        for (int64_t r = 0; r < b; ++r) W[IDX(i0 + r, j0 + s)] -= acc64[r];
                    } else if (cls == ORC_P32 && lo32) {
                        static const int pa[6] = {1, 0, 2, 0, 1, 0}, pb[6] = {1, 2, 0, 1, 0, 0};
                        for (int64_t r = 0; r < b; ++r) acc32[r] = 0.0f;
                        for (int t = 0; t < 6; ++t)
                            for (int64_t cc = 0; cc < b; ++cc) {
                                int64_t c = order ? b - 1 - cc : cc;
                                float bj = S3[pb[t]][(j0 + s) + (size_t)c * np];
                                const float *ci = S3[pa[t]] + i0 + (size_t)c * np;
                                for (int64_t r = 0; r < b; ++r) acc32[r] += ci[r] * bj;
                            }
                        for (int64_t r = 0; r < b; ++r) {
                            float w = (float)W[IDX(i0 + r, j0 + s)];
                            W[IDX(i0 + r, j0 + s)] = (double)(w - acc32[r]);
                        }
                    } else {
                        for (int64_t r = 0; r < b; ++r) acc32[r] = 0.0f;
                        for (int64_t cc = 0; cc < b; ++cc) {
                            int64_t c = order ? b - 1 - cc : cc;
                            float bj = (float)CJ[(j0 + s) + (size_t)c * np];
                            const double *ci = CI + i0 + (size_t)c * np;
                            for (int64_t r = 0; r < b; ++r) acc32[r] += (float)ci[r] * bj;
                        }
                        for (int64_t r = 0; r < b; ++r) {
                            float w = (float)W[IDX(i0 + r, j0 + s)];
                            if (cls == ORC_P32 || (cls == ORC_P8 && lo8)) w = w - acc32[r];
                            else w = w - ldexpf(acc32[r], -(tq[I * 4 + cls] + tq[J * 4 + cls]));
                            W[IDX(i0 + r, j0 + s)] = (double)w;
                        }
                    }
                }
            }
        }
    }

    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Lhat[i + j * ldl] = (i >= j) ? W[IDX(i, j)] : 0.0;
    for (int c = 0; c < 4; ++c) free(C[c]);
    for (int p = 0; p < 3; ++p) free(S3[p]);
    free(tq);
    free(Z64);
    free(ez);
    free(W);
    return info;
}

/* ------------------------------------------------------------------------
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), and the normal
 * draws z of the emulation step xi = V z (Sec. III.B).
 * Draw e (column-major index of an n x ndraws array) uses block e / 4,
 * counter {block_lo, block_hi, 0, 0}, key {seed_lo, seed_hi}; the four
 * 32-bit outputs give uniforms u_q = ((x_q >> 8) + 1) * 2^-24 in (0, 1], and
 * Box-Muller pairs (u0,u1) -> (r cos, r sin)(2 pi u1), r = sqrt(-2 log u0),
 * likewise (u2,u3); draw e takes entry e mod 4.
 * Pinned by: the generator's published known-answer vectors.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_normal_draws(uint64_t seed, int64_t count, double *z, uint32_t *raw)
{
    const double twopi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < (count + 3) / 4; ++blk) {
        uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)((uint64_t)blk >> 32), 0u, 0u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        double u[4], v[4];
        for (int q = 0; q < 4; ++q) u[q] = ((double)(o[q] >> 8) + 1.0) * ldexp(1.0, -24);
        double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
        v[0] = r0 * cos(twopi * u[1]);
        v[1] = r0 * sin(twopi * u[1]);
        v[2] = r1 * cos(twopi * u[3]);
        v[3] = r1 * sin(twopi * u[3]);
        for (int q = 0; q < 4; ++q) {
            int64_t e = blk * 4 + q;
            if (e < count) {
                if (z) z[e] = v[q];
                if (raw) raw[e] = o[q];
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * Learned precision selector reference (FP64).  A multilayer perceptron
 * 8 -> 64 -> 64 -> 4 with ReLU and a softmax over the classes
 * {FP64, FP32, 16-bit, FP8}.  Parameter vector layout (row-major, out x in):
 *   W1[64*8], b1[64], W2[64*64], b2[64], W3[4*64], b3[4]   (4932 values).
 * Loss per sample with label y and probabilities p:
 *   w_y * (-log p_y) + alpha * sum_{c > y} p_c
 * (class weights w_y; the second term charges probability put on classes
 * of lower precision than the label, which would be unsafe); the batch loss
 * is the mean.  Adam (Kingma & Ba 2015) with bias correction.
 * Pinned by: a hand-computed forward case and central finite differences.
 * ---------------------------------------------------------------------- */
#define H1 64
#define H2 64
#define NF 8
#define NC 4
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H1 * NF)
#define OFF_W2 (OFF_B1 + H1)
#define OFF_B2 (OFF_W2 + H2 * H1)
#define OFF_W3 (OFF_B2 + H2)
#define OFF_B3 (OFF_W3 + NC * H2)
#define NPARAM (OFF_B3 + NC)

int64_t orc_mlp_nparam(void) { return NPARAM; }

static void mlp_fwd1(const double *P, const double *x, double *h1, double *h2, double *z)
{
    for (int o = 0; o < H1; ++o) {
        double s = P[OFF_B1 + o];
        for (int i = 0; i < NF; ++i) s += P[OFF_W1 + o * NF + i] * x[i];
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < H2; ++o) {
        double s = P[OFF_B2 + o];
        for (int i = 0; i < H1; ++i) s += P[OFF_W2 + o * H1 + i] * h1[i];
        h2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < NC; ++o) {
        double s = P[OFF_B3 + o];
        for (int i = 0; i < H2; ++i) s += P[OFF_W3 + o * H2 + i] * h2[i];
        z[o] = s;
    }
}

void orc_mlp_forward(const double *P, int64_t nb, const double *X, double *logits)
{
    double h1[H1], h2[H2];
    for (int64_t s = 0; s < nb; ++s) mlp_fwd1(P, X + s * NF, h1, h2, logits + s * NC);
}

double orc_mlp_loss_grad(const double *P, int64_t nb, const double *X, const int32_t *y, const double *cw, double alpha,
                         double *grad)
{
    double h1[H1], h2[H2], z[NC], p[NC], dz[NC], dh2[H2], dh1[H1];
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * NPARAM);
    for (int64_t s = 0; s < nb; ++s) {
        const double *x = X + s * NF;
        int lab = y[s];
        mlp_fwd1(P, x, h1, h2, z);
        double zm = z[0];
        for (int c = 1; c < NC; ++c) zm = z[c] > zm ? z[c] : zm;
        double se = 0.0;
        for (int c = 0; c < NC; ++c) se += exp(z[c] - zm);
        double pu = 0.0;
        for (int c = 0; c < NC; ++c) {
            p[c] = exp(z[c] - zm) / se;
            if (c > lab) pu += p[c];
        }
        loss += cw[lab] * (-(z[lab] - zm - log(se))) + alpha * pu;
        if (!grad) continue;
        for (int c = 0; c < NC; ++c) {
            double g = cw[lab] * (p[c] - (c == lab ? 1.0 : 0.0));
            g += alpha * p[c] * ((c > lab ? 1.0 : 0.0) - pu);
            dz[c] = g / (double)nb;
        }
        for (int i = 0; i < H2; ++i) dh2[i] = 0.0;
        for (int o = 0; o < NC; ++o) {
            grad[OFF_B3 + o] += dz[o];
            for (int i = 0; i < H2; ++i) {
                grad[OFF_W3 + o * H2 + i] += dz[o] * h2[i];
                dh2[i] += dz[o] * P[OFF_W3 + o * H2 + i];
            }
        }
        for (int i = 0; i < H1; ++i) dh1[i] = 0.0;
        for (int o = 0; o < H2; ++o) {
            double g = h2[o] > 0.0 ? dh2[o] : 0.0;
            grad[OFF_B2 + o] += g;
            for (int i = 0; i < H1; ++i) {
                grad[OFF_W2 + o * H1 + i] += g * h1[i];
                dh1[i] += g * P[OFF_W2 + o * H1 + i];
            }
        }
        for (int o = 0; o < H1; ++o) {
            double g = h1[o] > 0.0 ? dh1[o] : 0.0;
            grad[OFF_B1 + o] += g;
            for (int i = 0; i < NF; ++i) grad[OFF_W1 + o * NF + i] += g * x[i];
        }
    }
    return loss / (double)nb;
}

void orc_adam_step(int64_t np_, double *P, const double *g, double *m, double *v, int64_t step, double lr, double b1,
                   double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < np_; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        P[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
