// Driver of the library's host code under AddressSanitizer and Undefined-
// BehaviorSanitizer (host code only, without UBSan's function-type check;
// the device code is built as usual):
// every call of the C ABI on small problems with ragged last tiles -- maps of
// every rule, factorizations in every arithmetic option, logdet, solve,
// sampling (also without allocation), residuals and estimates, the selector
// (features, inference with verification and fallback, labels), the
// covariance producer, the trainer object and its state, the SHT object --
// and the error paths (bad arguments, calls out of order).  Exits non-zero on
// the first failed check; the sanitizers abort on any host-side invalid
// access or undefined operation.  Built by paper_2408_04440_amd/build.py
// (build_host_sanitize), run by tests/test_gpu_host_sanitize.py.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <vector>
#include "mpchol.h"

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand()
{
    rs = rs * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

#define OK(call)                                                                                          \
    do {                                                                                                  \
        int rc_ = (call);                                                                                 \
        if (rc_ != MPCHOL_OK) {                                                                           \
            fprintf(stderr, "line %d: %s -> %d (%s: %s)\n", __LINE__, #call, rc_, mpchol_strerror(rc_),    \
                    mpchol_last_error());                                                                 \
            return 1;                                                                                     \
        }                                                                                                 \
    } while (0)
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "line %d: check failed: %s\n", __LINE__, #c);  \
            return 1;                                                      \
        }                                                                  \
    } while (0)

// the band-limit-L synthetic covariance inputs: sigma > 0, increasing x
static void workload(int64_t n, std::vector<double> &sigma, std::vector<double> &x)
{
    sigma.resize(n);
    x.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        sigma[i] = 0.5 + urand();
        x[i] = (i ? x[i - 1] : 0.0) + 0.05 + urand();
    }
}

static int run_rules(int64_t n, int32_t tile, int32_t lo16, int32_t lo32, int32_t lo64)
{
    std::vector<double> sigma, x;
    workload(n, sigma, x);
    mpchol_opts o;
    mpchol_default_opts(&o);
    o.lo16 = lo16;
    o.lo32 = lo32;
    o.lo64 = lo64;
    o.profile = 1;
    mpchol_t h = nullptr;
    OK(mpchol_create(&h, n, tile, &o));
    const int64_t nt = (n + tile - 1) / tile;
    std::vector<uint8_t> map(nt * nt), user(nt * nt, 0);
    for (int64_t J = 0; J < nt; ++J)
        for (int64_t I = J + 2; I < nt; ++I) user[I + J * nt] = (uint8_t)((I + 2 * J) % 4);  // beyond the band
    const int32_t rules[4] = {MPCHOL_RULE_FP64, MPCHOL_RULE_NORM, MPCHOL_RULE_BAND, MPCHOL_RULE_USER};
    for (int r = 0; r < 4; ++r) {
        OK(mpchol_set_generator(h, sigma.data(), x.data(), 5.0, 1e-6));
        OK(mpchol_precision_map(h, rules[r], 1e-6, user.data(), map.data()));
        int64_t info = -1;
        OK(mpchol_factor(h, &info));
        CHECK(info == 0);
        double ld = 0, be = 0, est = 0;
        std::vector<double> tr(nt * nt);
        OK(mpchol_logdet(h, &ld));
        CHECK(isfinite(ld));
        OK(mpchol_backward_error(h, &be, tr.data()));
        OK(mpchol_backward_error_estimate(h, 1, 7, &est));
        if (!(be >= 0 && be < 1e-2 && est >= 0)) {
            fprintf(stderr, "rule %d: backward error %g, estimate %g\n", rules[r], be, est);
            return 1;
        }
        mpchol_stats st;
        OK(mpchol_get_stats(h, &st));
        std::vector<int32_t> ts(nt * nt);
        OK(mpchol_get_tile_scales(h, ts.data()));
    }
    OK(mpchol_destroy(h));
    return 0;
}

int main()
{
    // ---- argument and order checks (no device work)
    for (int c = -8; c <= 2; ++c) CHECK(mpchol_strerror(c) != nullptr);
    CHECK(mpchol_destroy(nullptr) == MPCHOL_OK);
    mpchol_opts o;
    mpchol_default_opts(&o);
    mpchol_t h = nullptr;
    CHECK(mpchol_create(&h, 0, 128, &o) == MPCHOL_EINVAL);
    CHECK(mpchol_create(&h, 1000, 100, &o) == MPCHOL_EINVAL);
    CHECK(mpchol_create(nullptr, 1000, 128, &o) == MPCHOL_EINVAL);

    // ---- every rule in each arithmetic option, ragged last tiles
    if (run_rules(1000, 128, MPCHOL_LO16_F16, MPCHOL_LO32_BF16X3, MPCHOL_LO64_FP64)) return 1;
    if (run_rules(1300, 256, MPCHOL_LO16_BF16, MPCHOL_LO32_FP32, MPCHOL_LO64_INT8)) return 1;

    // ---- one handle through the rest of the calls
    const int64_t n = 1100;
    const int32_t tile = 128;
    const int64_t nt = (n + tile - 1) / tile;
    std::vector<double> sigma, x;
    workload(n, sigma, x);
    o.verify = 2;
    o.verify_eps = 1e-9;
    OK(mpchol_create(&h, n, tile, &o));
    double dummy = 0;
    CHECK(mpchol_logdet(h, &dummy) == MPCHOL_EORDER);  // before any factor
    CHECK(mpchol_factor(h, nullptr) == MPCHOL_EORDER);
    OK(mpchol_set_generator(h, sigma.data(), x.data(), 5.0, 1e-8));
    std::vector<float> feats(nt * nt * 8), params(MPCHOL_MLP_NPARAM);
    for (auto &p : params) p = (float)(urand() - 0.5) * 0.2f;
    OK(mpchol_selector_set(h, params.data(), MPCHOL_MLP_NPARAM));
    std::vector<uint8_t> map(nt * nt);
    OK(mpchol_precision_map(h, MPCHOL_RULE_LEARNED, 1e-9, nullptr, map.data()));
    OK(mpchol_selector_features(h, 1e-9, feats.data()));
    int64_t info = -1;
    int rc = mpchol_factor(h, &info);  // random weights: verified, and refactored under a fallback rule if needed
    CHECK(rc == MPCHOL_OK && info == 0);
    double ld = 0;
    OK(mpchol_logdet(h, &ld));
    // solve and sampling on device buffers
    const int nrhs = 3, nd = 5;
    double *B = nullptr;
    float *Y = nullptr, *Z = nullptr;
    uint32_t *raw = nullptr;
    double *Ld = nullptr;
    CHECK(hipMalloc(&B, n * nrhs * sizeof(double)) == hipSuccess);
    CHECK(hipMalloc(&Y, n * nd * sizeof(float)) == hipSuccess);
    CHECK(hipMalloc(&Z, n * nd * sizeof(float)) == hipSuccess);
    CHECK(hipMalloc(&raw, n * nd * sizeof(uint32_t)) == hipSuccess);
    CHECK(hipMalloc(&Ld, n * n * sizeof(double)) == hipSuccess);
    std::vector<double> hb(n * nrhs);
    for (auto &v : hb) v = urand() - 0.5;
    CHECK(hipMemcpy(B, hb.data(), hb.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess);
    OK(mpchol_solve(h, nrhs, B, n));
    OK(mpchol_sample(h, nd, 3, Y, n));
    OK(mpchol_normal_draws(h, n * nd, 3, Z, raw));
    OK(mpchol_sample_z(h, nd, Z, n, Y, n));
    OK(mpchol_sample_noalloc(h, nd, 3, Y, n));
    OK(mpchol_get_factor(h, Ld, n));
    CHECK(hipDeviceSynchronize() == hipSuccess);
    CHECK(mpchol_solve(h, nrhs, nullptr, n) == MPCHOL_EINVAL);
    CHECK(mpchol_sample(h, nd, 3, Y, n - 1) == MPCHOL_EINVAL);
    // a caller matrix: the factor's residual against A = the kept covariance
    std::vector<double> A(n * n);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            A[i + j * n] = sigma[i] * sigma[j] * exp(-fabs(x[i] - x[j]) / 5.0) + (i == j ? 1e-8 : 0.0);
    double bem = 0;
    std::vector<double> tr(nt * nt);
    OK(mpchol_backward_error_matrix(h, A.data(), n, 0, &bem, tr.data()));
    CHECK(bem < 1e-6);
    OK(mpchol_set_verify(h, 1, 1e-9));
    // the covariance producer: Sigma = scale Xi Xi^T + nugget I from host samples
    const int64_t m = 40;
    std::vector<double> xi(n * m);
    for (auto &v : xi) v = urand() - 0.5;
    OK(mpchol_set_samples(h, xi.data(), n, m, 1.0 / m, 1e-2, 0));
    OK(mpchol_precision_map(h, MPCHOL_RULE_NORM, 1e-6, nullptr, nullptr));
    OK(mpchol_factor(h, &info));
    // labels on a set matrix (A = L0 L0^T, small integers: every class exact)
    std::vector<double> L0(n * n, 0.0), A0(n * n, 0.0);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) L0[i + j * n] = (i == j) ? 1.0 + (double)(int)(urand() * 3) : (double)((int)(urand() * 5) - 2);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) {
            double s = 0;
            for (int64_t k = 0; k <= j; ++k) s += L0[i + k * n] * L0[j + k * n];
            A0[i + j * n] = A0[j + i * n] = s;
        }
    OK(mpchol_set_matrix(h, A0.data(), n, 0));
    std::vector<uint8_t> labels(nt * nt);
    double lbe = 0;
    rc = mpchol_selector_labels(h, 1e-9, labels.data(), &lbe, nullptr);
    CHECK(rc == MPCHOL_OK || rc == MPCHOL_EBUDGET);
    OK(mpchol_destroy(h));
    CHECK(hipFree(B) == hipSuccess && hipFree(Y) == hipSuccess && hipFree(Z) == hipSuccess);
    CHECK(hipFree(raw) == hipSuccess && hipFree(Ld) == hipSuccess);

    // ---- the trainer object and its state
    mpchol_mlp_t t = nullptr;
    OK(mpchol_mlp_create(&t, 0, nullptr));
    const int64_t nb = 100;
    std::vector<float> hx(nb * 8);
    std::vector<int32_t> hy(nb);
    for (auto &v : hx) v = (float)(urand() * 2 - 1);
    for (int64_t i = 0; i < nb; ++i) hy[i] = (int32_t)(i % 4);
    float *dx = nullptr;
    int32_t *dy = nullptr, *dc = nullptr;
    CHECK(hipMalloc(&dx, hx.size() * 4) == hipSuccess && hipMalloc(&dy, nb * 4) == hipSuccess &&
          hipMalloc(&dc, nb * 4) == hipSuccess);
    CHECK(hipMemcpy(dx, hx.data(), hx.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
    CHECK(hipMemcpy(dy, hy.data(), nb * 4, hipMemcpyHostToDevice) == hipSuccess);
    const float cw[4] = {1, 1, 1, 1};
    OK(mpchol_mlp_set_params(t, params.data(), MPCHOL_MLP_NPARAM));
    float loss = 0;
    for (int s = 0; s < 3; ++s) OK(mpchol_mlp_train_step(t, dx, dy, nb, cw, 1.0f, 1e-3f, &loss));
    std::vector<float> p2(MPCHOL_MLP_NPARAM), m1(MPCHOL_MLP_NPARAM), m2(MPCHOL_MLP_NPARAM);
    int32_t step = 0;
    OK(mpchol_mlp_get_state(t, p2.data(), m1.data(), m2.data(), &step, MPCHOL_MLP_NPARAM));
    CHECK(step == 3);
    OK(mpchol_mlp_set_state(t, p2.data(), m1.data(), m2.data(), step, MPCHOL_MLP_NPARAM));
    CHECK(mpchol_mlp_set_state(t, p2.data(), m1.data(), m2.data(), -1, MPCHOL_MLP_NPARAM) == MPCHOL_EINVAL);
    OK(mpchol_mlp_predict(t, dx, nb, nullptr, dc));
    OK(mpchol_mlp_destroy(t));
    CHECK(hipFree(dx) == hipSuccess && hipFree(dy) == hipSuccess && hipFree(dc) == hipSuccess);

    // ---- the SHT object
    mpchol_sht_t sh = nullptr;
    OK(mpchol_sht_create(&sh, 16, 17, 32, 4, 0, nullptr));
    OK(mpchol_sht_destroy(sh));

    printf("ok\n");
    return 0;
}
