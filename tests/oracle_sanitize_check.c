/* Host driver of the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer: every entry point of oracle.c on small cases with a ragged last
 * tile (n = 77, tiles of 16), each class and option of the mixed-precision
 * replay, the Ozaki products, the draws and the MLP.  Exits non-zero on the
 * first failed check; the sanitizers abort on any invalid access or
 * undefined operation.  Built and run by tests/test_host_logic.py. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_cov_dense(int64_t n, const double *sigma, const double *x, double rho, double nugget, double *A, int64_t lda);
void orc_cov_samples(int64_t n, int64_t m, const double *xi, int64_t ldxi, double scale, double nugget, double *S,
                     int64_t lds);
int64_t orc_potrf(int64_t n, double *A, int64_t lda);
double orc_logdet(int64_t n, const double *L, int64_t ldl);
void orc_potrs(int64_t n, const double *L, int64_t ldl, int64_t nrhs, double *B, int64_t ldb);
double orc_residual_fro(int64_t n, const double *A, int64_t lda, const double *L, int64_t ldl, double *anorm);
void orc_tile_residual2(int64_t n, int64_t b, const double *A, int64_t lda, const double *L, int64_t ldl, double *out);
void orc_lower_matmul(int64_t n, const double *L, int64_t ldl, int64_t m, const double *Z, int64_t ldz, double *Y,
                      int64_t ldy);
double orc_markov_logdet(int64_t n, const double *sigma, const double *x, double rho, double nugget);
void orc_markov_solve(int64_t n, const double *sigma, const double *x, double rho, double nugget, int64_t nrhs,
                      double *B, int64_t ldb);
double orc_round(double v, int fmt);
double orc_e4m3_decode(uint8_t code);
double orc_unit_roundoff(int fmt);
int orc_scale_exp(double amax, int fmt);
double orc_tile_norms(int64_t n, int64_t b, const double *A, int64_t lda, double *fro2, double *amax);
void orc_map_norm(int64_t nt, const double *fro2, double total_fro, double eps, int band, unsigned allowed, int lo16,
                  uint8_t *map);
void orc_map_band(int64_t nt, int band, int variant, unsigned allowed, uint8_t *map);
int orc_ozaki_row_exp(const double *X, int64_t ld, int64_t len);
void orc_ozaki_gemm(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                    double *D, int64_t ldd);
float orc_split3(double v, int part);
int64_t orc_mp_factor(int64_t n, int64_t b, const double *A, int64_t lda, const uint8_t *map, int lo16, double *Lhat,
                      int64_t ldl, int32_t *tscale, int order, int lo32, int lo64, int band64, int lo8);
int orc_mx_block_exp(double amax);
void orc_mx_quantize(int64_t rows, int64_t cols, const double *X, int64_t ld, double *out, int64_t ldo, int32_t *texp);
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
void orc_normal_draws(uint64_t seed, int64_t count, double *z, uint32_t *raw);
int64_t orc_mlp_nparam(void);
void orc_mlp_forward(const double *P, int64_t nb, const double *X, double *logits);
double orc_mlp_loss_grad(const double *P, int64_t nb, const double *X, const int32_t *y, const double *cw, double alpha,
                         double *grad);
void orc_adam_step(int64_t np_, double *P, const double *g, double *m, double *v, int64_t step, double lr, double b1,
                   double b2, double eps);

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand(void)  /* uniform [0, 1), 53 bits */
{
    rs = rs * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(void)
{
    const int64_t n = 77, b = 16, nt = (n + b - 1) / b;
    double *sigma = malloc(n * sizeof(double)), *x = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        sigma[i] = 0.5 + urand();
        x[i] = (i ? x[i - 1] : 0.0) + 0.05 + urand();
    }
    double *A = malloc(n * n * sizeof(double)), *L = malloc(n * n * sizeof(double));
    orc_cov_dense(n, sigma, x, 5.0, 1e-8, A, n);
    memcpy(L, A, n * n * sizeof(double));
    CHECK(orc_potrf(n, L, n) == 0);
    const double ld = orc_logdet(n, L, n), mk = orc_markov_logdet(n, sigma, x, 5.0, 1e-8);
    CHECK(fabs(ld - mk) <= 1e-8 * fabs(mk));
    double anorm = 0.0;
    CHECK(orc_residual_fro(n, A, n, L, n, &anorm) <= 1e-13 * anorm);
    double *tr = malloc(nt * nt * sizeof(double));
    orc_tile_residual2(n, b, A, n, L, n, tr);
    const int64_t nr = 3;
    double *B = malloc(n * nr * sizeof(double)), *B2 = malloc(n * nr * sizeof(double));
    for (int64_t i = 0; i < n * nr; ++i) B[i] = B2[i] = urand() - 0.5;
    orc_potrs(n, L, n, nr, B, n);
    orc_markov_solve(n, sigma, x, 5.0, 1e-8, nr, B2, n);
    for (int64_t i = 0; i < n * nr; ++i) CHECK(fabs(B[i] - B2[i]) <= 1e-6 * (1.0 + fabs(B2[i])));
    const int64_t m = 5;
    double *Z = malloc(n * m * sizeof(double)), *Y = malloc(n * m * sizeof(double));
    for (int64_t i = 0; i < n * m; ++i) Z[i] = urand() - 0.5;
    orc_lower_matmul(n, L, n, m, Z, n, Y, n);
    double *xi = malloc(n * 9 * sizeof(double)), *S = malloc(n * n * sizeof(double));
    for (int64_t i = 0; i < n * 9; ++i) xi[i] = urand() - 0.5;
    orc_cov_samples(n, 9, xi, n, 1.0 / 9.0, 1e-3, S, n);

    for (int fmt = 1; fmt <= 4; ++fmt) {
        CHECK(orc_unit_roundoff(fmt) > 0.0);
        for (int i = 0; i < 64; ++i) {
            const double v = (urand() - 0.5) * ldexp(1.0, (int)(urand() * 60) - 30);
            CHECK(!isnan(orc_round(v, fmt)));  // FP16 overflows to infinity
            (void)orc_scale_exp(fabs(v) + 1e-300, fmt);
        }
    }
    for (int c = 0; c < 256; ++c) (void)orc_e4m3_decode((uint8_t)c);
    {  /* block-scaled copy with a ragged last block, and the exponent clamp */
        double X[3 * 45], Q[3 * 45];
        int32_t te[3 * 2];
        for (int i = 0; i < 3 * 45; ++i) X[i] = (urand() - 0.5) * ldexp(1.0, (int)(urand() * 60) - 30);
        orc_mx_quantize(3, 45, X, 3, Q, 3, te);
        for (int i = 0; i < 3 * 45; ++i) {  /* relative bound, or half the subnormal spacing of the block */
            const int t = te[i % 3 + (i / 3 / 32) * 3];
            CHECK(fabs(Q[i] - X[i]) <= fmax(0.0626 * fabs(X[i]), ldexp(1.0, -10 - t)));
        }
        CHECK(orc_mx_block_exp(0.0) == 0 && orc_mx_block_exp(1e-300) == 127 && orc_mx_block_exp(1e300) == -127);
    }
    for (int p = 0; p < 3; ++p) (void)orc_split3(urand() - 0.5, p);

    double *fro2 = malloc(nt * nt * sizeof(double)), *amax = malloc(nt * nt * sizeof(double));
    const double tot = orc_tile_norms(n, b, A, n, fro2, amax);
    uint8_t *map = malloc(nt * nt);
    double *Lh = malloc(n * n * sizeof(double));
    int32_t *ts = malloc(nt * nt * sizeof(int32_t));
    for (int variant = 0; variant < 3; ++variant) orc_map_band(nt, 1, variant, 0xFu, map);
    for (int lo16 = 0; lo16 <= 1; ++lo16) {
        orc_map_norm(nt, fro2, sqrt(tot), 1e-4, 0, 0xFu, lo16, map);
        for (int64_t J = 0; J < nt; ++J)
            for (int64_t I = J + 1; I < nt; ++I) map[I + J * nt] = (uint8_t)((I + 2 * J + lo16) % 4);
        for (int order = 0; order <= 1; ++order)
            for (int lo32 = 0; lo32 <= 1; ++lo32)
                for (int lo64 = 0; lo64 <= 1; ++lo64) {
                    const int lo8 = (order + lo32 + lo64) & 1;
                    memset(Lh, 0, n * n * sizeof(double));
                    CHECK(orc_mp_factor(n, b, A, n, map, lo16, Lh, n, ts, order, lo32, lo64, 1, lo8) == 0);
                    double an2 = 0.0;
                    CHECK(orc_residual_fro(n, A, n, Lh, n, &an2) <= 0.1 * an2);
                }
    }

    const int64_t om = 7, on = 5, ok = 33;
    double *Oa = malloc(om * ok * sizeof(double)), *Ob = malloc(on * ok * sizeof(double)), *Od = malloc(om * on * sizeof(double));
    for (int64_t i = 0; i < om * ok; ++i) Oa[i] = (urand() - 0.5) * ldexp(1.0, (int)(urand() * 20) - 10);
    for (int64_t i = 0; i < on * ok; ++i) Ob[i] = (urand() - 0.5) * ldexp(1.0, (int)(urand() * 20) - 10);
    (void)orc_ozaki_row_exp(Oa, om, ok);
    orc_ozaki_gemm(om, on, ok, Oa, om, Ob, on, Od, om);
    for (int64_t i = 0; i < om; ++i)
        for (int64_t j = 0; j < on; ++j) {
            double s = 0.0, sa = 0.0;
            for (int64_t k = 0; k < ok; ++k) {
                s += Oa[i + k * om] * Ob[j + k * on];
                sa += fabs(Oa[i + k * om] * Ob[j + k * on]);
            }
            CHECK(fabs(Od[i + j * om] - s) <= 1e-13 * sa);
        }

    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    double *zd = malloc(37 * sizeof(double));
    uint32_t *raw = malloc(40 * sizeof(uint32_t));
    orc_normal_draws(11, 37, zd, raw);
    for (int i = 0; i < 37; ++i) CHECK(isfinite(zd[i]));

    const int64_t np_ = orc_mlp_nparam(), nb = 9;
    double *P = malloc(np_ * sizeof(double)), *g = malloc(np_ * sizeof(double));
    double *m1 = calloc(np_, sizeof(double)), *m2 = calloc(np_, sizeof(double));
    double *X = malloc(nb * 8 * sizeof(double)), *lg = malloc(nb * 4 * sizeof(double));
    int32_t *y = malloc(nb * sizeof(int32_t));
    const double cw[4] = {1.0, 2.0, 0.5, 1.5};
    for (int64_t i = 0; i < np_; ++i) P[i] = (urand() - 0.5) * 0.3;
    for (int64_t i = 0; i < nb * 8; ++i) X[i] = urand() * 2.0 - 1.0;
    for (int64_t i = 0; i < nb; ++i) y[i] = (int32_t)(i % 4);
    orc_mlp_forward(P, nb, X, lg);
    for (int step = 1; step <= 3; ++step) {
        CHECK(isfinite(orc_mlp_loss_grad(P, nb, X, y, cw, 2.0, g)));
        orc_adam_step(np_, P, g, m1, m2, step, 1e-3, 0.9, 0.999, 1e-8);
    }

    free(sigma); free(x); free(A); free(L); free(tr); free(B); free(B2); free(Z); free(Y); free(xi); free(S);
    free(fro2); free(amax); free(map); free(Lh); free(ts); free(Oa); free(Ob); free(Od); free(zd); free(raw);
    free(P); free(g); free(m1); free(m2); free(X); free(lg); free(y);
    printf("ok\n");
    return 0;
}
