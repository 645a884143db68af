// Host runtime of libmpchol: handle state, tile storage, the precision-map
// rules, the static per-step schedule of the right-looking tile algorithm
// (Sec. V.A) and the C ABI declared in include/mpchol.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mpchol.h"
#include "common.h"
#include "launch.h"
#include "ozaki_crt.h"

using namespace mpc;

namespace {

enum State { S_CREATED = 0, S_SOURCE = 1, S_LOADED = 2, S_FACTORED = 3, S_FAILED = 4 };

// Panel copy sets, indexed by panel column mod NSET: the two pairs whose
// low-class updates are applied together, and the pair the look-ahead
// stream is factoring.
constexpr int NSET = 6;

double unit_roundoff(int q, int lo16)
{
    switch (q) {
    case P32: return std::ldexp(1.0, -24);
    case P16: return lo16 == LO16_BF16 ? std::ldexp(1.0, -8) : std::ldexp(1.0, -11);
    case P8: return std::ldexp(1.0, -4);
    default: return std::ldexp(1.0, -53);
    }
}

}  // namespace

struct mpchol_handle {
    int dev = 0;
    hipStream_t st = nullptr;
    mpchol_opts o{};
    int64_t n = 0;
    int b = 0, nt = 0;
    int64_t ntile = 0;
    size_t slot_bytes = 0;
    char *slots = nullptr;
    double *orig = nullptr;
    double *d_sigma = nullptr, *d_x = nullptr;
    double rho = 0, nugget = 0;
    int src = 0;  // 0 none, 1 matrix, 2 generator
    bool x_sorted = false;  // generator coordinates nondecreasing
    hipStream_t st2 = nullptr;           // look-ahead stream for the panel of the next step
    hipEvent_t ev_next = nullptr, ev_panel = nullptr;
    // panel copies, four sets (column mod 4: the pair being applied and the pair being factored)
    double *p64 = nullptr;
    float *p32 = nullptr;
    uint16_t *p32s = nullptr;  // three BF16 parts of the FP32 copies (lo32 = BF16x3)
    uint16_t *p16 = nullptr;
    uint8_t *p8 = nullptr;
    uint8_t *p8x = nullptr;      // lo8 MX: E8M0 block scales of the FP8 copies
    unsigned long long *pmax = nullptr;
    int32_t *pscale = nullptr;
    int8_t *poz = nullptr;       // lo64 INT8: residue planes of the FP64 copies, four sets
    int32_t *pexp = nullptr;     // lo64 INT8: their row exponents
    OzakiConst *d_ozc = nullptr; // lo64 INT8: moduli and reconstruction constants (device)
    // per-tile metadata
    uint8_t *d_map = nullptr;
    int32_t *d_tscale = nullptr;
    double *d_fro2 = nullptr, *d_amax = nullptr;
    unsigned long long *d_info = nullptr;
    double *d_scalar = nullptr;
    std::vector<uint8_t> h_map;
    std::vector<double> h_fro2, h_amax;
    double total_fro = 0;
    double last_eps = 1e-9;
    // schedule
    int32_t *d_items = nullptr;
    // (npair * 12 + 1) offsets: pair p (columns 2p, 2p+1), class, part
    // (0: column 2p+1 by column 2p; 1: columns 2p+2, 2p+3 by the pair; 2: the rest by the pair)
    // update classes of the schedule: the four map classes, and FP64-class
    // tiles beyond the band whose products are formed from INT8 products (lo64)
    static constexpr int NQ = 5;
    std::vector<int64_t> item_off;
    std::vector<int32_t> item_syrk;  // per (pair, class, part): how many of its items are SYRK (I == J)
    uint8_t *d_qmask = nullptr;
    int32_t *d_all_items = nullptr;  // every lower tile, for the residual
    double *d_partial = nullptr, *d_tres2 = nullptr;
    // backward-error estimator scratch
    double *d_est = nullptr;
    float *d_zbuf = nullptr;
    // selector
    float *d_params = nullptr, *d_feats = nullptr;
    bool have_params = false;
    int state = S_CREATED;
    int rule_used = MPCHOL_RULE_FP64;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> gev;  // profile mode: start/stop pairs per update launch
    std::vector<int> gev_class;
    std::vector<double> gev_flops;
    mpchol_stats stats{};

    Tiles tiles() const
    {
        Tiles T;
        T.slots = slots;
        T.slot_bytes = (int64_t)slot_bytes;
        T.b = b;
        T.nt = nt;
        T.n = n;
        T.map = d_map;
        T.tscale = d_tscale;
        T.lo16 = o.lo16;
        T.lo32 = o.lo32;
        T.lo8 = o.lo8;
        return T;
    }
    Source source() const
    {
        Source S;
        S.sigma = d_sigma;
        S.x = d_x;
        S.rho = rho;
        S.nugget = nugget;
        S.orig = orig;
        return S;
    }
    Panel panel(int set) const
    {
        const size_t bb = (size_t)b * b;
        Panel P;
        P.p64 = p64 + set * nt * bb;
        P.p32 = p32 + set * nt * bb;
        P.p32s = p32s ? p32s + set * nt * 3 * bb : nullptr;
        P.p16 = p16 + set * nt * bb;
        P.p8 = p8 + set * nt * bb;
        P.pmax = pmax + set * nt;
        P.pscale = pscale + set * nt * 4;
        P.poz = poz ? poz + (size_t)set * nt * OZ_NMOD * bb : nullptr;
        P.pexp = pexp ? pexp + (size_t)set * nt * b : nullptr;
        P.p8x = p8x ? p8x + (size_t)set * nt * bb / 32 : nullptr;
        P.info = d_info;
        return P;
    }
};

// Text of the last failing HIP call on this thread (mpchol_last_error).
static thread_local char g_last_error[512] = "";

static int hip_fail(hipError_t e, const char *expr, int line)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s failed: %s (%d) at mpchol.cpp:%d", expr, hipGetErrorString(e),
             (int)e, line);
    (void)hipGetLastError();
    return MPCHOL_EHIP;
}

// Draw buffer of mpchol_sample_noalloc: one array per device, part of the
// library's code object (so it exists without any allocation call), held
// until the process ends.  Host code never uses this name as an address: the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (noalloc_scratch_setup) and kept in g_scratch.
constexpr int64_t NOALLOC_SCRATCH_FLOATS = (int64_t)1 << 24;  // 64 MiB
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
constexpr int MAX_DEVICES = 64;
static float *g_scratch[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// With `dev` current: the device address of this device's scratch array
// (looked up on the first call for the device).  MPCHOL_EHIP on failure.
static int noalloc_scratch_setup(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        snprintf(g_last_error, sizeof(g_last_error), "device %d beyond the %d devices the draw buffer covers", dev,
                 MAX_DEVICES);
        return MPCHOL_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return MPCHOL_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        snprintf(g_last_error, sizeof(g_last_error), "hipGetSymbolAddress(scratch) failed: %s (%d) on device %d",
                 hipGetErrorString(e), (int)e, dev);
        (void)hipGetLastError();
        return MPCHOL_EHIP;
    }
    g_scratch[dev] = (float *)p;
    return MPCHOL_OK;
}

#define HIPCHK(x)                                                   \
    do {                                                            \
        hipError_t e_ = (x);                                        \
        if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__);    \
    } while (0)

template <typename T>
static int dalloc(T **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return MPCHOL_OK;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        hip_fail(e, "hipMalloc", __LINE__);
        return MPCHOL_ENOMEM;
    }
    return MPCHOL_OK;
}

static void release(mpchol_handle *h)
{
    void *ptrs[] = {h->slots, h->orig, h->d_sigma, h->d_x, h->p64, h->p32, h->p32s, h->p16, h->p8, h->p8x, h->pmax, h->pscale,
                    h->poz, h->pexp, h->d_ozc,
                    h->d_map, h->d_tscale, h->d_fro2, h->d_amax, h->d_info, h->d_scalar, h->d_items, h->d_qmask,
                    h->d_all_items, h->d_partial, h->d_tres2, h->d_params, h->d_feats, h->d_est, h->d_zbuf};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &e : h->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : h->gev) (void)hipEventDestroy(e);
    if (h->ev_next) (void)hipEventDestroy(h->ev_next);
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->st2) (void)hipStreamDestroy(h->st2);
}

extern "C" {

void mpchol_default_opts(mpchol_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->lo16 = MPCHOL_LO16_F16;
    o->band = 1;
    o->allowed = 0xF;
    o->band_variant = MPCHOL_BAND_DP_HP;
    o->verify = 0;
    o->verify_eps = 1e-9;
    o->profile = 0;
    o->lo32 = MPCHOL_LO32_BF16X3;
    o->lo64 = MPCHOL_LO64_FP64;
    o->lo8 = MPCHOL_LO8_TILE;
}

const char *mpchol_last_error(void) { return g_last_error; }

const char *mpchol_strerror(int s)
{
    switch (s) {
    case MPCHOL_OK: return "ok";
    case MPCHOL_NOT_SPD: return "matrix not positive definite (a pivot was not positive)";
    case MPCHOL_EINVAL: return "invalid argument";
    case MPCHOL_ENOMEM: return "device allocation failed";
    case MPCHOL_EHIP: return "HIP runtime error";
    case MPCHOL_EORDER: return "call out of order";
    case MPCHOL_EBUDGET: return "backward-error budget missed after every fallback";
    case MPCHOL_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int mpchol_create(mpchol_t *hp, int64_t n, int32_t tile, const mpchol_opts *o)
{
    if (!hp) return MPCHOL_EINVAL;
    *hp = nullptr;
    if (n <= 0 || tile < 128 || tile > 2048 || tile % 128 != 0) return MPCHOL_EINVAL;
    int64_t nt = (n + tile - 1) / tile;
    if (nt > 32767) return MPCHOL_EINVAL;
    mpchol_opts opt;
    if (o) opt = *o;
    else mpchol_default_opts(&opt);
    if (opt.lo16 != MPCHOL_LO16_F16 && opt.lo16 != MPCHOL_LO16_BF16) return MPCHOL_EINVAL;
    if (opt.lo32 != MPCHOL_LO32_FP32 && opt.lo32 != MPCHOL_LO32_BF16X3) return MPCHOL_EINVAL;
    if (opt.lo64 != MPCHOL_LO64_FP64 && opt.lo64 != MPCHOL_LO64_INT8) return MPCHOL_EINVAL;
    if (opt.lo64 == MPCHOL_LO64_INT8 && tile > OZ_MAX_TILE) return MPCHOL_EUNSUPPORTED;
    if (opt.lo8 != MPCHOL_LO8_TILE && opt.lo8 != MPCHOL_LO8_MX) return MPCHOL_EINVAL;
    if (opt.band < 0) return MPCHOL_EINVAL;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (opt.device < 0 || opt.device >= ndev) {
        snprintf(g_last_error, sizeof(g_last_error), "device %d not present (%d visible)", opt.device, ndev);
        return MPCHOL_EHIP;
    }
    HIPCHK(hipSetDevice(opt.device));
    // look up this device's draw buffer for mpchol_sample_noalloc; a failure
    // is reported by that call only (it leaves g_last_error set here)
    (void)noalloc_scratch_setup(opt.device);

    mpchol_handle *h = new (std::nothrow) mpchol_handle();
    if (!h) return MPCHOL_ENOMEM;
    h->dev = opt.device;
    h->st = (hipStream_t)opt.stream;
    h->o = opt;
    h->n = n;
    h->b = tile;
    h->nt = (int)nt;
    h->ntile = nt * (nt + 1) / 2;
    h->slot_bytes = (size_t)tile * tile * 8;
    const size_t bb = (size_t)tile * tile;
    int rc = MPCHOL_OK;
    auto A = [&](int r) {
        if (rc == MPCHOL_OK && r != MPCHOL_OK) rc = r;
    };
    A(dalloc(&h->slots, h->ntile * h->slot_bytes));
    A(dalloc(&h->p64, NSET * nt * bb * 8));
    A(dalloc(&h->p32, NSET * nt * bb * 4));
    if (h->o.lo32 == MPCHOL_LO32_BF16X3) A(dalloc(&h->p32s, NSET * nt * bb * 3 * 2));
    A(dalloc(&h->p16, NSET * nt * bb * 2));
    A(dalloc(&h->p8, NSET * nt * bb));
    if (h->o.lo8 == MPCHOL_LO8_MX) A(dalloc(&h->p8x, NSET * nt * bb / 32));
    if (h->o.lo64 == MPCHOL_LO64_INT8) {
        A(dalloc(&h->poz, NSET * nt * OZ_NMOD * bb));
        A(dalloc(&h->pexp, NSET * nt * (size_t)tile * 4));
        A(dalloc(&h->d_ozc, sizeof(OzakiConst)));
    }
    A(dalloc(&h->pmax, NSET * nt * 8));
    A(dalloc(&h->pscale, NSET * nt * 4 * 4));
    A(dalloc(&h->d_map, nt * nt));
    A(dalloc(&h->d_tscale, nt * nt * 4));
    A(dalloc(&h->d_fro2, nt * nt * 8));
    A(dalloc(&h->d_amax, nt * nt * 8));
    A(dalloc(&h->d_info, 8));
    A(dalloc(&h->d_scalar, 64));
    A(dalloc(&h->d_qmask, nt * nt));
    A(dalloc(&h->d_all_items, h->ntile * 4));
    A(dalloc(&h->d_partial, h->ntile * (bb / (128 * 128)) * 8));
    A(dalloc(&h->d_tres2, nt * nt * 8));
    A(dalloc(&h->d_params, MPCHOL_MLP_NPARAM * 4));
    A(dalloc(&h->d_feats, nt * nt * 8 * 4));
    auto H = [&](hipError_t e, const char *what) {
        if (rc == MPCHOL_OK && e != hipSuccess) rc = hip_fail(e, what, __LINE__);
    };
    for (auto &e : h->ev)
        if (rc == MPCHOL_OK) H(hipEventCreate(&e), "hipEventCreate");
    if (rc == MPCHOL_OK) H(hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    if (rc == MPCHOL_OK) H(hipEventCreateWithFlags(&h->ev_next, hipEventDisableTiming), "hipEventCreateWithFlags");
    if (rc == MPCHOL_OK) H(hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming), "hipEventCreateWithFlags");
    if (rc == MPCHOL_OK && h->d_ozc) {
        OzakiConst kc;
        ozaki_const_init(&kc);
        H(hipMemcpy(h->d_ozc, &kc, sizeof(kc), hipMemcpyHostToDevice), "hipMemcpy(ozaki constants)");
    }
    if (rc == MPCHOL_OK) {
        std::vector<int32_t> all;
        all.reserve(h->ntile);
        for (int I = 0; I < nt; ++I)
            for (int J = 0; J <= I; ++J) all.push_back((I << 16) | J);
        H(hipMemcpy(h->d_all_items, all.data(), all.size() * 4, hipMemcpyHostToDevice), "hipMemcpy(items)");
        H(hipMemset(h->d_tscale, 0, nt * nt * 4), "hipMemset(tscale)");
        H(hipMemset(h->d_map, 0, nt * nt), "hipMemset(map)");
    }
    if (rc != MPCHOL_OK) {
        release(h);
        delete h;
        return rc;
    }
    h->h_map.assign(nt * nt, 0);
    h->stats.n = n;
    h->stats.tile = tile;
    h->stats.nt = (int)nt;
    *hp = h;
    return MPCHOL_OK;
}

int mpchol_destroy(mpchol_t h)
{
    if (!h) return MPCHOL_OK;
    (void)hipSetDevice(h->dev);
    (void)hipStreamSynchronize(h->st);
    release(h);
    delete h;
    return MPCHOL_OK;
}

int mpchol_set_matrix(mpchol_t h, const double *A, int64_t lda, int32_t on_device)
{
    if (!h || !A || lda < h->n) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    if (!h->orig) {
        int rc = dalloc(&h->orig, h->ntile * h->slot_bytes);
        if (rc) return rc;
    }
    const double *dA = A;
    double *tmp = nullptr;
    if (!on_device) {
        size_t bytes = (size_t)lda * h->n * 8;
        int rc = dalloc(&tmp, bytes);
        if (rc) return rc;
        if (hipMemcpyAsync(tmp, A, bytes, hipMemcpyHostToDevice, h->st) != hipSuccess) {
            (void)hipFree(tmp);
            return MPCHOL_EHIP;
        }
        dA = tmp;
    }
    launch_copy_matrix(h->tiles(), dA, lda, h->orig, h->st);
    hipError_t e = hipStreamSynchronize(h->st);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess || hipGetLastError() != hipSuccess) return MPCHOL_EHIP;
    h->src = 1;
    h->state = S_SOURCE;
    return MPCHOL_OK;
}

int mpchol_set_samples(mpchol_t h, const double *xi, int64_t ldxi, int64_t m, double scale, double nugget,
                       int32_t on_device)
{
    if (!h || !xi || ldxi < h->n || m < 1 || !(scale > 0) || !(nugget >= 0)) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    if (!h->orig) {
        int rc = dalloc(&h->orig, h->ntile * h->slot_bytes);
        if (rc) return rc;
    }
    const int64_t mp = (m + 15) / 16 * 16, ldp = (int64_t)h->nt * h->b;
    double *xp = nullptr, *tmp = nullptr;
    int rc = dalloc(&xp, (size_t)ldp * mp * 8);
    if (rc) return rc;
    const double *dx = xi;
    if (!on_device) {
        const size_t bytes = (size_t)ldxi * (size_t)m * 8;
        rc = dalloc(&tmp, bytes);
        if (rc) {
            (void)hipFree(xp);
            return rc;
        }
        if (hipMemcpyAsync(tmp, xi, bytes, hipMemcpyHostToDevice, h->st) != hipSuccess) {
            (void)hipFree(xp);
            (void)hipFree(tmp);
            return MPCHOL_EHIP;
        }
        dx = tmp;
    }
    hipError_t e = hipEventRecord(h->ev[2], h->st);
    launch_cov_samples(h->tiles(), dx, ldxi, m, scale, nugget, xp, mp, h->orig, h->st);
    if (e == hipSuccess) e = hipEventRecord(h->ev[3], h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e == hipSuccess) e = hipGetLastError();
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev[2], h->ev[3]);
    (void)hipFree(xp);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) {
        hip_fail(e, "set_samples", __LINE__);
        return MPCHOL_EHIP;
    }
    h->stats.t_samples_ms = ms;
    h->src = 1;
    h->state = S_SOURCE;
    return MPCHOL_OK;
}

int mpchol_set_generator(mpchol_t h, const double *sigma, const double *x, double rho, double nugget)
{
    if (!h || !sigma || !x || !(rho > 0) || !(nugget >= 0)) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    if (!h->d_sigma) {
        int rc = dalloc(&h->d_sigma, h->n * 8);
        if (rc) return rc;
        rc = dalloc(&h->d_x, h->n * 8);
        if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(h->d_sigma, sigma, h->n * 8, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(h->d_x, x, h->n * 8, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (h->orig) {
        (void)hipFree(h->orig);
        h->orig = nullptr;
    }
    h->rho = rho;
    h->nugget = nugget;
    h->x_sorted = true;
    for (int64_t i = 1; i < h->n; ++i)
        if (!(x[i] >= x[i - 1])) {
            h->x_sorted = false;
            break;
        }
    h->src = 2;
    h->state = S_SOURCE;
    return MPCHOL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- map rules
static void rule_fp64(mpchol_handle *h, std::vector<uint8_t> &m) { std::fill(m.begin(), m.end(), (uint8_t)P64); }

static void rule_norm(mpchol_handle *h, double eps, std::vector<uint8_t> &m)
{
    const int nt = h->nt;
    const double thr = eps * h->total_fro / nt;
    for (int J = 0; J < nt; ++J)
        for (int I = 0; I < nt; ++I) {
            uint8_t c = P64;
            if (I > J && I - J > h->o.band) {
                double f = std::sqrt(h->h_fro2[I + (size_t)J * nt]);
                for (int cls = P8; cls >= P32; --cls) {
                    if (!(h->o.allowed & (1u << cls))) continue;
                    if (f * unit_roundoff(cls, h->o.lo16) <= thr) {
                        c = (uint8_t)cls;
                        break;
                    }
                }
            }
            m[I + (size_t)J * nt] = (I >= J) ? c : 0;
        }
}

// Highest allowed class at or above (more precise than) `c`.
static uint8_t clamp_allowed(uint32_t allowed, int c)
{
    while (c > P64 && !(allowed & (1u << c))) --c;
    return (uint8_t)c;
}

static void rule_band(mpchol_handle *h, std::vector<uint8_t> &m)
{
    const int nt = h->nt, w = h->o.band;
    int w32 = w;
    if (h->o.band_variant == MPCHOL_BAND_DP_SP_HP) {
        // narrowest band beyond the FP64 band holding >= 5% of the strict-lower tiles
        const double total = (double)nt * (nt - 1) / 2.0;
        double cnt = 0;
        w32 = w;
        while (w32 < nt - 1 && cnt < 0.05 * total) {
            ++w32;
            if (w32 > w) cnt += (double)(nt - w32);
        }
    }
    for (int J = 0; J < nt; ++J)
        for (int I = 0; I < nt; ++I) {
            int c = P64;
            int d = I - J;
            if (I > J && d > w) {
                switch (h->o.band_variant) {
                case MPCHOL_BAND_DP_SP: c = P32; break;
                case MPCHOL_BAND_DP_SP_HP: c = (d <= w32) ? P32 : P16; break;
                default: c = P16; break;
                }
                c = clamp_allowed(h->o.allowed, c);
            }
            m[I + (size_t)J * nt] = (I >= J) ? (uint8_t)c : 0;
        }
}

// Static schedule, by pairs of steps p (panel columns c = 2p and c+1): per
// class q, part 0 the tiles of column c+1 (updated by column c alone, on the
// look-ahead stream inside the pair's panel work), part 1 the tiles of
// columns c+2 and c+3 (which the next pair's panel needs), part 2 the rest
// (J >= c+4); parts 1 and 2 take both columns of the pair (K = 2b).  And, per
// panel tile (I, k), the mask of classes its consumers use.
// Update class of tile (I, J): its map class, except that FP64-class tiles
// beyond the FP64 band form their products from INT8 products when lo64 asks
// for it (class 4); SYRK, the band and the plain FP64 path stay on the FP64
// MFMA.
static int update_class(const mpchol_handle *h, int I, int J, bool int8_ok)
{
    if (I == J) return P64;
    const int cl = h->h_map[I + (size_t)J * h->nt];
    if (cl == P64 && int8_ok && I - J > h->o.band) return 4;
    return cl;
}

static void build_schedule_counts(mpchol_handle *h, std::vector<int32_t> &items, std::vector<uint8_t> &qmask,
                                  bool int8_ok)
{
    const int nt = h->nt, npair = (nt + 1) / 2, NQ = mpchol_handle::NQ;
    h->item_off.assign((size_t)npair * NQ * 3 + 1, 0);
    h->item_syrk.assign((size_t)npair * NQ * 3, 0);
    items.clear();
    for (int p = 0; p < npair; ++p) {
        const int c = 2 * p;
        for (int q = 0; q < NQ; ++q)
            for (int part = 0; part < 3; ++part) {
                const size_t o = ((size_t)p * NQ + q) * 3 + part;
                h->item_off[o] = (int64_t)items.size();
                const int jlo = part == 0 ? c + 1 : part == 1 ? c + 2 : c + 4;
                const int jhi = part == 0 ? c + 1 : part == 1 ? c + 3 : nt - 1;
                for (int J = jlo; J <= jhi && J < nt; ++J)
                    for (int I = J; I < nt; ++I)
                        if (update_class(h, I, J, int8_ok) == q) {
                            items.push_back((I << 16) | J);
                            h->item_syrk[o] += (I == J);
                        }
            }
    }
    h->item_off[(size_t)npair * NQ * 3] = (int64_t)items.size();
    qmask.assign((size_t)nt * nt, 0);
    for (int k = 0; k < nt; ++k)
        for (int I = k + 1; I < nt; ++I) {
            uint8_t msk = 1;  // SYRK(I,I) reads the FP64 copy
            for (int J = k + 1; J < I; ++J) msk |= (uint8_t)(1u << update_class(h, I, J, int8_ok));
            for (int J = I + 1; J < nt; ++J) msk |= (uint8_t)(1u << update_class(h, J, I, int8_ok));
            qmask[I + (size_t)k * nt] = msk;
        }
}

static void fill_flop_stats(mpchol_handle *h)
{
    const int nt = h->nt;
    const double b3 = (double)h->b * h->b * h->b;
    for (int q = 0; q < 4; ++q) {
        h->stats.tiles_per_class[q] = 0;
        h->stats.flops_per_class[q] = 0;
    }
    for (int J = 0; J < nt; ++J) {
        h->stats.flops_per_class[P64] += b3 / 3.0 + (double)(nt - J - 1) * b3;  // POTRF + TRSM below it
        h->stats.flops_per_class[P64] += (double)J * b3;                            // SYRK updates of (J,J)
        for (int I = J + 1; I < nt; ++I) {
            int c = h->h_map[I + (size_t)J * nt];
            h->stats.tiles_per_class[c] += 1;
            h->stats.flops_per_class[c] += 2.0 * b3 * J;  // GEMM updates of (I,J), one per k < J
        }
    }
}

// Host-side map from norms by rule, then upload map + schedule and load.
static int apply_map(mpchol_handle *h, int rule, double eps, const uint8_t *user_map)
{
    const int nt = h->nt;
    std::vector<uint8_t> m((size_t)nt * nt, 0);
    switch (rule) {
    case MPCHOL_RULE_FP64: rule_fp64(h, m); break;
    case MPCHOL_RULE_NORM: rule_norm(h, eps, m); break;
    case MPCHOL_RULE_BAND: rule_band(h, m); break;
    case MPCHOL_RULE_USER:
        for (int J = 0; J < nt; ++J)
            for (int I = 0; I < nt; ++I) {
                uint8_t c = user_map[I + (size_t)J * nt];
                if (c > P8) return MPCHOL_EINVAL;
                m[I + (size_t)J * nt] = (I > J) ? clamp_allowed(h->o.allowed, c) : 0;
            }
        break;
    case MPCHOL_RULE_LEARNED: {
        Tiles T = h->tiles();
        T.map = h->d_map;
        launch_features(T, h->d_fro2, h->d_amax, h->total_fro, eps, h->d_feats, h->st);
        launch_mlp_infer_map(T, h->d_params, h->d_feats, h->o.band, h->o.allowed, h->d_map, h->st);
        HIPCHK(hipMemcpyAsync(m.data(), h->d_map, m.size(), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        break;
    }
    default: return MPCHOL_EINVAL;
    }
    h->h_map = m;
    std::vector<int32_t> items;
    std::vector<uint8_t> qmask;
    // the plain FP64 path (rule FP64) keeps every product on the FP64 MFMA
    build_schedule_counts(h, items, qmask, h->o.lo64 == MPCHOL_LO64_INT8 && rule != MPCHOL_RULE_FP64);
    if (h->d_items) (void)hipFree(h->d_items);
    h->d_items = nullptr;
    if (!items.empty()) {
        int rc = dalloc(&h->d_items, items.size() * 4);
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(h->d_items, items.data(), items.size() * 4, hipMemcpyHostToDevice, h->st));
    }
    HIPCHK(hipMemcpyAsync(h->d_map, m.data(), m.size(), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(h->d_qmask, qmask.data(), qmask.size(), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemsetAsync(h->d_tscale, 0, (size_t)nt * nt * 4, h->st));
    launch_load(h->tiles(), h->source(), h->st);
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipGetLastError());
    h->rule_used = rule;
    fill_flop_stats(h);
    h->state = S_LOADED;
    return MPCHOL_OK;
}

static int compute_norms(mpchol_handle *h)
{
    const int nt = h->nt;
    HIPCHK(hipMemsetAsync(h->d_fro2, 0, (size_t)nt * nt * 8, h->st));
    HIPCHK(hipMemsetAsync(h->d_amax, 0, (size_t)nt * nt * 8, h->st));
    launch_norms(h->tiles(), h->source(), h->d_fro2, h->d_amax, h->st);
    h->h_fro2.assign((size_t)nt * nt, 0.0);
    h->h_amax.assign((size_t)nt * nt, 0.0);
    HIPCHK(hipMemcpyAsync(h->h_fro2.data(), h->d_fro2, (size_t)nt * nt * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipMemcpyAsync(h->h_amax.data(), h->d_amax, (size_t)nt * nt * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipGetLastError());
    double tot = 0.0;
    for (int J = 0; J < nt; ++J)
        for (int I = J; I < nt; ++I) tot += (I == J ? 1.0 : 2.0) * h->h_fro2[I + (size_t)J * nt];
    h->total_fro = std::sqrt(tot);
    h->stats.total_fro = h->total_fro;
    return MPCHOL_OK;
}

static int run_factor(mpchol_handle *h, int64_t *info);
static int residual(mpchol_handle *h, double *berr, double *tile_res2);
static int estimate(mpchol_handle *h, int sets, uint64_t seed, double *ratio);

extern "C" int mpchol_precision_map(mpchol_t h, int32_t rule, double eps, const uint8_t *user_map, uint8_t *map_out)
{
    if (!h) return MPCHOL_EINVAL;
    if (h->state < S_SOURCE) return MPCHOL_EORDER;
    if (rule < MPCHOL_RULE_FP64 || rule > MPCHOL_RULE_LEARNED) return MPCHOL_EINVAL;
    if (rule == MPCHOL_RULE_USER && !user_map) return MPCHOL_EINVAL;
    if (rule == MPCHOL_RULE_LEARNED && !h->have_params) return MPCHOL_EORDER;
    if ((rule == MPCHOL_RULE_NORM || rule == MPCHOL_RULE_LEARNED) && !(eps > 0)) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipEventRecord(h->ev[2], h->st));
    int rc = compute_norms(h);
    if (rc) return rc;
    h->last_eps = eps;
    rc = apply_map(h, rule, eps, user_map);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev[3], h->st));
    HIPCHK(hipEventSynchronize(h->ev[3]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
    h->stats.t_map_ms = ms;
    if (map_out) std::memcpy(map_out, h->h_map.data(), h->h_map.size());
    return MPCHOL_OK;
}

// Panel work of step k on stream st: TRSM of the tiles below the diagonal
// into the FP64 panel (which also takes max |X| per tile), and the
// sender-side conversion.
static int panel_step(mpchol_handle *h, const Tiles &T, const Panel &P, int k, hipStream_t st)
{
    HIPCHK(hipMemsetAsync(P.pmax, 0, (size_t)h->nt * 8, st));
    launch_trsm_panel(T, P, k, st);
    launch_convert(T, P, k, h->d_qmask + (size_t)k * h->nt, st);
    if (h->d_ozc) launch_ozaki_convert(T, P, k, h->d_qmask + (size_t)k * h->nt, h->d_ozc, st);
    return MPCHOL_OK;
}

// Classes whose updates an even pair leaves for the next pair beyond its
// next panel: the FP16/BF16 and FP8 updates, so that each of their FP32 work
// tiles is read and written once per four steps.  Their error comes from the
// 16-bit/8-bit operands, far above the FP32 accumulation over K = 4b; the
// FP32 class, whose error is that accumulation's, keeps K = 2b.
static bool deferred_class(const mpchol_handle *, int q) { return q == P16 || q == P8; }

// The update list (pair p, part) per class on stream st.  P holds the panel
// sets by column mod NSET; c = 2p.  Part 0: column c+1 by column c.  Parts 1
// and 2: the pair's two columns, except for the deferred classes: an even
// pair skips their part 2, and an odd pair applies both pairs (columns c-2
// .. c+1) to its parts 1 and 2 of those classes.
static int update_list(mpchol_handle *h, const Tiles &T, const Panel *P, int p, int part, hipStream_t st)
{
    const double b3 = (double)h->b * h->b * h->b;
    const int c = 2 * p;
    for (int q = 0; q < mpchol_handle::NQ; ++q) {
        const size_t o = ((size_t)p * mpchol_handle::NQ + q) * 3 + part;
        const int64_t off = h->item_off[o];
        const int cnt = (int)(h->item_off[o + 1] - off);
        if (cnt <= 0) continue;
        const Panel *ps[4];
        int npan = 0;
        if (part == 0) {
            ps[npan++] = &P[c % NSET];
        } else if (q < 4 && deferred_class(h, q)) {
            if ((p & 1) == 0 && part == 2) continue;  // left for the next pair
            if (p & 1) {
                ps[npan++] = &P[(c - 2) % NSET];
                ps[npan++] = &P[(c - 1) % NSET];
            }
            ps[npan++] = &P[c % NSET];
            ps[npan++] = &P[(c + 1) % NSET];
        } else {
            ps[npan++] = &P[c % NSET];
            ps[npan++] = &P[(c + 1) % NSET];
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (h->o.profile) {
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            HIPCHK(hipEventRecord(e0, st));
        }
        if (q == 4) launch_ozaki_update(T, *ps[0], npan > 1 ? ps[1] : nullptr, h->d_items + off, cnt, h->d_ozc, st);
        else launch_update(T, ps, npan, q, h->d_items + off, cnt, st, part == 0);
        if (h->o.profile) {
            HIPCHK(hipEventRecord(e1, st));
            h->gev.push_back(e0);
            h->gev.push_back(e1);
            h->gev_class.push_back(q);
            // task flops of the launch: per step GEMM 2b^3, SYRK b^3 (its kernel computes the lower blocks only)
            const int syrk = h->item_syrk[o];
            h->gev_flops.push_back(b3 * (2.0 * (cnt - syrk) + syrk) * npan);
        }
    }
    return MPCHOL_OK;
}

// Panel work of the pair starting at column c on stream st: POTRF(c,c), TRSM
// and conversion of column c, the update of column c+1 by column c, then
// POTRF(c+1,c+1), TRSM and conversion of column c+1.
static int panel_pair(mpchol_handle *h, const Tiles &T, const Panel *P, int c, hipStream_t st)
{
    const int nt = h->nt;
    launch_potrf_tile(T, c, h->d_info, st);
    if (c + 1 >= nt) return MPCHOL_OK;
    int rc = panel_step(h, T, P[c % NSET], c, st);
    if (rc) return rc;
    rc = update_list(h, T, P, c / 2, 0, st);
    if (rc) return rc;
    launch_potrf_tile(T, c + 1, h->d_info, st);
    if (c + 2 < nt) rc = panel_step(h, T, P[(c + 1) % NSET], c + 1, st);
    return rc;
}

// Right-looking tile algorithm taken two steps at a time, with look-ahead:
// the caller's stream A applies pair (c, c+1) to the trailing tiles with
// K = 2b (the deferred classes: K = 4b every other pair); once columns c+2
// and c+3 are updated, a second stream B runs the next pair's panel work
// (into its own two panel sets) while A finishes the rest of the pair's
// update.
static int run_factor(mpchol_handle *h, int64_t *info)
{
    const int nt = h->nt;
    Tiles T = h->tiles();
    Panel P[NSET];
    for (int i = 0; i < NSET; ++i) P[i] = h->panel(i);
    hipStream_t A = h->st, B = h->st2;
    for (auto e : h->gev) (void)hipEventDestroy(e);
    h->gev.clear();
    h->gev_class.clear();
    h->gev_flops.clear();
    HIPCHK(hipMemsetAsync(h->d_info, 0xFF, 8, A));
    HIPCHK(hipEventRecord(h->ev[0], A));
    int rc = panel_pair(h, T, P, 0, A);
    if (rc) return rc;
    for (int c = 0; c + 2 < nt; c += 2) {
        rc = update_list(h, T, P, c / 2, 1, A);
        if (rc) return rc;
        HIPCHK(hipEventRecord(h->ev_next, A));
        HIPCHK(hipStreamWaitEvent(B, h->ev_next, 0));
        rc = panel_pair(h, T, P, c + 2, B);
        if (rc) return rc;
        HIPCHK(hipEventRecord(h->ev_panel, B));
        rc = update_list(h, T, P, c / 2, 2, A);
        if (rc) return rc;
        HIPCHK(hipStreamWaitEvent(A, h->ev_panel, 0));
    }
    HIPCHK(hipEventRecord(h->ev[1], A));
    unsigned long long hinfo = 0;
    HIPCHK(hipMemcpyAsync(&hinfo, h->d_info, 8, hipMemcpyDeviceToHost, A));
    HIPCHK(hipStreamSynchronize(A));
    HIPCHK(hipGetLastError());
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
    h->stats.t_factor_ms = ms;
    for (int q = 0; q < 4; ++q) {
        h->stats.t_gemm_ms[q] = 0;
        h->stats.gemm_launches[q] = 0;
        h->stats.gemm_flops[q] = 0;
    }
    h->stats.t_gemm_int8_ms = 0;
    h->stats.gemm_int8_launches = 0;
    h->stats.gemm_int8_flops = 0;
    for (size_t i = 0; i < h->gev_class.size(); ++i) {
        float g = 0;
        HIPCHK(hipEventElapsedTime(&g, h->gev[2 * i], h->gev[2 * i + 1]));
        int q = h->gev_class[i];
        if (q == 4) {
            h->stats.t_gemm_int8_ms += g;
            h->stats.gemm_int8_launches += 1;
            h->stats.gemm_int8_flops += h->gev_flops[i];
            continue;
        }
        h->stats.t_gemm_ms[q] += g;
        h->stats.gemm_launches[q] += 1;
        h->stats.gemm_flops[q] += h->gev_flops[i];
    }
    h->stats.rule_used = h->rule_used;
    int64_t inf = (hinfo == ~0ull) ? 0 : (int64_t)hinfo;
    if (info) *info = inf;
    if (inf) {
        h->state = S_FAILED;
        return MPCHOL_NOT_SPD;
    }
    h->state = S_FACTORED;
    return MPCHOL_OK;
}

extern "C" int mpchol_factor(mpchol_t h, int64_t *info)
{
    if (!h) return MPCHOL_EINVAL;
    if (info) *info = 0;
    if (h->state != S_LOADED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    h->stats.fallbacks = 0;
    h->stats.verify_first = -1.0;
    int64_t inf = 0;
    int rc = run_factor(h, &inf);
    if (rc < 0) return rc;
    if (h->rule_used == MPCHOL_RULE_LEARNED && h->o.verify) {
        const int fallback_rules[2] = {MPCHOL_RULE_NORM, MPCHOL_RULE_FP64};
        for (int f = 0;; ++f) {
            bool ok = (rc == MPCHOL_OK);
            if (ok) {
                double be = 0;
                if (h->o.verify == 2) {
                    // randomized estimate with one set of probes (64); accept with a
                    // margin of three standard deviations of the estimate, 1 + 3/sqrt(2*64)
                    int r2 = estimate(h, 1, 0x5EEDu + (uint64_t)f, &be);
                    if (r2) return r2;
                    if (f == 0) h->stats.verify_first = be;
                    ok = (be * (1.0 + 3.0 / std::sqrt(2.0 * estimate_probes())) <= h->o.verify_eps);
                } else {
                    int r2 = residual(h, &be, nullptr);
                    if (r2) return r2;
                    if (f == 0) h->stats.verify_first = be;
                    ok = (be <= h->o.verify_eps);
                }
            }
            if (ok) break;
            if (f == 0 && rc != MPCHOL_OK) h->stats.verify_first = INFINITY;  // the map broke down
            if (f >= 2) {
                if (info) *info = inf;
                return rc == MPCHOL_NOT_SPD ? MPCHOL_NOT_SPD : MPCHOL_EBUDGET;
            }
            h->stats.fallbacks += 1;
            int r3 = apply_map(h, fallback_rules[f], h->last_eps, nullptr);
            if (r3) return r3;
            rc = run_factor(h, &inf);
            if (rc < 0) return rc;
        }
    }
    if (info) *info = inf;
    return rc;
}

extern "C" int mpchol_logdet(mpchol_t h, double *out)
{
    if (!h || !out) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    launch_logdet(h->tiles(), h->d_scalar, h->st);
    HIPCHK(hipMemcpyAsync(out, h->d_scalar, 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

extern "C" int mpchol_get_factor(mpchol_t h, double *L, int64_t ldl)
{
    if (!h || !L || ldl < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    launch_get_factor(h->tiles(), L, ldl, h->st);
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

extern "C" int mpchol_get_tile_scales(mpchol_t h, int32_t *t)
{
    if (!h || !t) return MPCHOL_EINVAL;
    if (h->state < S_LOADED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipMemcpyAsync(t, h->d_tscale, (size_t)h->nt * h->nt * 4, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return MPCHOL_OK;
}

static int residual_of(mpchol_handle *h, const Source &S, double total_fro, double *berr, double *tile_res2)
{
    const int nt = h->nt;
    HIPCHK(hipEventRecord(h->ev[2], h->st));
    launch_residual_items(h->tiles(), S, h->d_all_items, (int)h->ntile, h->d_partial, h->d_tres2, h->st);
    std::vector<double> r((size_t)nt * nt, 0.0);
    HIPCHK(hipMemsetAsync(h->d_scalar, 0, 8, h->st));
    HIPCHK(hipMemcpyAsync(r.data(), h->d_tres2, r.size() * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipEventRecord(h->ev[3], h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipGetLastError());
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
    h->stats.t_residual_ms = ms;
    double tot = 0.0;
    for (int J = 0; J < nt; ++J)
        for (int I = J; I < nt; ++I) tot += (I == J ? 1.0 : 2.0) * r[I + (size_t)J * nt];
    if (berr) *berr = std::sqrt(tot) / total_fro;
    if (tile_res2) {
        for (int J = 0; J < nt; ++J)
            for (int I = 0; I < nt; ++I) tile_res2[I + (size_t)J * nt] = (I >= J) ? r[I + (size_t)J * nt] : 0.0;
    }
    return MPCHOL_OK;
}

static int residual(mpchol_handle *h, double *berr, double *tile_res2)
{
    return residual_of(h, h->source(), h->total_fro, berr, tile_res2);
}

static int estimate(mpchol_handle *h, int sets, uint64_t seed, double *ratio)
{
    const int64_t np = (int64_t)h->nt * h->b;
    const int k = estimate_probes();
    if (!h->d_est) {
        int rc = dalloc(&h->d_est, ((size_t)3 * np + 2 * (size_t)estimate_chunks(h->n)) * k * 8);
        if (rc) return rc;
        rc = dalloc(&h->d_zbuf, (size_t)h->n * k * 4);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(h->ev[2], h->st));
    double sum = 0.0;
    for (int p = 0; p < sets; ++p) {
        launch_estimate(h->tiles(), h->source(), h->x_sorted, seed + (uint64_t)p * 0x9E3779B97F4A7C15ull, h->d_est,
                        h->d_zbuf, h->d_scalar + 1, h->st);
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, h->d_scalar + 1, 8, hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        sum += v;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(h->ev[3], h->st));
    HIPCHK(hipEventSynchronize(h->ev[3]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
    h->stats.t_residual_ms = ms;
    *ratio = std::sqrt(sum / ((double)sets * k)) / h->total_fro;
    return MPCHOL_OK;
}

extern "C" int mpchol_backward_error_estimate(mpchol_t h, int32_t sets, uint64_t seed, double *est)
{
    if (!h || !est || sets <= 0) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    return estimate(h, sets, seed, est);
}

extern "C" int mpchol_backward_error(mpchol_t h, double *berr, double *tile_res2)
{
    if (!h || !berr) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    return residual(h, berr, tile_res2);
}

extern "C" int mpchol_backward_error_matrix(mpchol_t h, const double *A, int64_t lda, int32_t on_device, double *berr,
                                            double *tile_res2)
{
    if (!h || !A || !berr || lda < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    const int nt = h->nt;
    double *tmp = nullptr, *fro2 = nullptr, *amax = nullptr;
    auto cleanup = [&]() {
        if (tmp) (void)hipFree(tmp);
        if (fro2) (void)hipFree(fro2);
        if (amax) (void)hipFree(amax);
    };
    Source S{};
    S.dense = A;
    S.ld = lda;
    int rc = dalloc(&fro2, (size_t)nt * nt * 8);
    if (!rc) rc = dalloc(&amax, (size_t)nt * nt * 8);
    if (!rc && !on_device) {
        const size_t bytes = (size_t)lda * (size_t)(h->n - 1) * 8 + (size_t)h->n * 8;
        rc = dalloc(&tmp, bytes);
        if (!rc && hipMemcpyAsync(tmp, A, bytes, hipMemcpyHostToDevice, h->st) != hipSuccess) rc = MPCHOL_EHIP;
        S.dense = tmp;
    }
    if (!rc && hipMemsetAsync(fro2, 0, (size_t)nt * nt * 8, h->st) != hipSuccess) rc = MPCHOL_EHIP;
    std::vector<double> f2((size_t)nt * nt, 0.0);
    if (!rc) {
        launch_norms(h->tiles(), S, fro2, amax, h->st);
        if (hipMemcpyAsync(f2.data(), fro2, f2.size() * 8, hipMemcpyDeviceToHost, h->st) != hipSuccess ||
            hipStreamSynchronize(h->st) != hipSuccess || hipGetLastError() != hipSuccess)
            rc = MPCHOL_EHIP;
    }
    if (!rc) {
        double tot = 0.0;
        for (int J = 0; J < nt; ++J)
            for (int I = J; I < nt; ++I) tot += (I == J ? 1.0 : 2.0) * f2[I + (size_t)J * nt];
        rc = (tot > 0.0) ? residual_of(h, S, std::sqrt(tot), berr, tile_res2) : MPCHOL_EINVAL;
    }
    cleanup();
    return rc;
}

extern "C" int mpchol_set_verify(mpchol_t h, int32_t mode, double eps)
{
    if (!h || mode < 0 || mode > 2 || !(eps > 0)) return MPCHOL_EINVAL;
    h->o.verify = mode;
    h->o.verify_eps = eps;
    return MPCHOL_OK;
}

extern "C" int mpchol_get_stats(mpchol_t h, mpchol_stats *s)
{
    if (!h || !s) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipStreamSynchronize(h->st));
    *s = h->stats;
    return MPCHOL_OK;
}

extern "C" int mpchol_solve(mpchol_t h, int32_t nrhs, double *B, int64_t ldb)
{
    if (!h || !B || nrhs <= 0 || ldb < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipEventRecord(h->ev[2], h->st));
    launch_solve(h->tiles(), B, ldb, nrhs, h->st);
    HIPCHK(hipEventRecord(h->ev[3], h->st));
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

extern "C" int mpchol_sample_z(mpchol_t h, int32_t ndraws, const float *Z, int64_t ldz, float *Y, int64_t ldy)
{
    if (!h || !Z || !Y || ndraws <= 0 || ldz < h->n || ldy < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    launch_lower_apply(h->tiles(), Z, ldz, Y, ldy, ndraws, h->st);
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

extern "C" int mpchol_sample(mpchol_t h, int32_t ndraws, uint64_t seed, float *Y, int64_t ldy)
{
    if (!h || !Y || ndraws <= 0 || ldy < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    float *Z = nullptr;
    int rc = dalloc(&Z, (size_t)h->n * ndraws * 4);
    if (rc) return rc;
    launch_normal_matrix(seed, h->n, ndraws, Z, h->n, h->st);
    launch_lower_apply(h->tiles(), Z, h->n, Y, ldy, ndraws, h->st);
    hipError_t e = hipStreamSynchronize(h->st);
    (void)hipFree(Z);
    if (e != hipSuccess || hipGetLastError() != hipSuccess) return MPCHOL_EHIP;
    return MPCHOL_OK;
}

extern "C" int mpchol_sample_noalloc(mpchol_t h, int32_t ndraws, uint64_t seed, float *Y, int64_t ldy)
{
    if (!h || !Y || ndraws <= 0 || ldy < h->n) return MPCHOL_EINVAL;
    if (h->state != S_FACTORED) return MPCHOL_EORDER;
    if (h->n > NOALLOC_SCRATCH_FLOATS) {
        snprintf(g_last_error, sizeof(g_last_error),
                 "mpchol_sample_noalloc: n = %lld exceeds the draw buffer (%lld values per draw at most)",
                 (long long)h->n, (long long)NOALLOC_SCRATCH_FLOATS);
        return MPCHOL_EINVAL;
    }
    HIPCHK(hipSetDevice(h->dev));
    float *Z = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        Z = (h->dev >= 0 && h->dev < MAX_DEVICES) ? g_scratch[h->dev] : nullptr;
    }
    if (!Z) {
        snprintf(g_last_error, sizeof(g_last_error),
                 "mpchol_sample_noalloc: the draw buffer of device %d could not be looked up", h->dev);
        return MPCHOL_EHIP;
    }
    // draws per pass: as many whole columns as the buffer holds, in multiples
    // of the 128 draws one block of the product covers when possible
    int64_t chunk = NOALLOC_SCRATCH_FLOATS / h->n;
    if (chunk >= 128) chunk -= chunk % 128;
    for (int64_t d0 = 0; d0 < ndraws; d0 += chunk) {
        const int nd = (int)std::min<int64_t>(chunk, ndraws - d0);
        launch_normal_columns(seed, h->n, d0, nd, Z, h->n, h->st);
        launch_lower_apply(h->tiles(), Z, h->n, Y + d0 * ldy, ldy, nd, h->st);
    }
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

extern "C" int mpchol_normal_draws(mpchol_t h, int64_t count, uint64_t seed, float *z, uint32_t *raw)
{
    if (!h || count <= 0 || (!z && !raw)) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    launch_normal_draws(seed, count, z, raw, h->st);
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

// ---------------------------------------------------------------- selector
extern "C" int mpchol_selector_set(mpchol_t h, const float *params, int64_t nparam)
{
    if (!h || !params || nparam != MPCHOL_MLP_NPARAM) return MPCHOL_EINVAL;
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipMemcpyAsync(h->d_params, params, nparam * 4, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    h->have_params = true;
    return MPCHOL_OK;
}

extern "C" int mpchol_selector_features(mpchol_t h, double eps, float *feats)
{
    if (!h || !feats || !(eps > 0)) return MPCHOL_EINVAL;
    if (h->state < S_LOADED) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    launch_features(h->tiles(), h->d_fro2, h->d_amax, h->total_fro, eps, h->d_feats, h->st);
    HIPCHK(hipMemcpyAsync(feats, h->d_feats, (size_t)h->nt * h->nt * 8 * 4, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(hipGetLastError());
    return MPCHOL_OK;
}

// Greedy per-tile lowering under a measured backward-error budget.
extern "C" int mpchol_selector_labels(mpchol_t h, double eps, uint8_t *labels, double *berr_out, const double *rates)
{
    if (!h || !labels || !(eps > 0)) return MPCHOL_EINVAL;
    if (rates)
        for (int q = 0; q < 4; ++q)
            if (!(rates[q] > 0)) return MPCHOL_EINVAL;
    if (h->state < S_SOURCE) return MPCHOL_EORDER;
    HIPCHK(hipSetDevice(h->dev));
    const int nt = h->nt, w = h->o.band;
    int rc = compute_norms(h);
    if (rc) return rc;
    const double budget = 0.5 * (eps * h->total_fro) * (eps * h->total_fro);
    // Per-tile squared residual at each class: factor with every eligible tile
    // at that class; if that breaks down, retry with only the tiles the norm
    // rule puts at that class or lower for targets eps*1e6, eps*1e3, eps (the
    // others FP64).  Residuals are tile-separable, so the other tiles' classes
    // barely matter; a tile never measured at a class is not eligible for it.
    std::vector<std::vector<double>> res(4, std::vector<double>((size_t)nt * nt, INFINITY));
    std::fill(res[P64].begin(), res[P64].end(), 0.0);
    std::vector<uint8_t> um((size_t)nt * nt, 0), nm((size_t)nt * nt, 0);
    for (int q = P32; q <= P8; ++q) {
        if (!(h->o.allowed & (1u << q))) continue;
        const double scales[4] = {0.0, 1e6, 1e3, 1.0};
        for (int trial = 0; trial < 4; ++trial) {
            if (trial > 0) rule_norm(h, eps * scales[trial], nm);
            int cnt = 0;
            for (int J = 0; J < nt; ++J)
                for (int I = J + 1; I < nt; ++I) {
                    size_t t = I + (size_t)J * nt;
                    bool at_q = (I - J > w) && (trial == 0 || nm[t] >= q);
                    um[t] = at_q ? (uint8_t)q : 0;
                    cnt += at_q;
                }
            if (cnt == 0) break;
            rc = apply_map(h, MPCHOL_RULE_USER, eps, um.data());
            if (rc) return rc;
            int64_t inf = 0;
            rc = run_factor(h, &inf);
            if (rc < 0) return rc;
            if (rc == MPCHOL_NOT_SPD) continue;
            std::vector<double> tr((size_t)nt * nt, 0.0);
            double be = 0;
            rc = residual(h, &be, tr.data());
            if (rc) return rc;
            for (size_t t = 0; t < um.size(); ++t)
                if (um[t] == q) res[q][t] = tr[t];
            break;
        }
    }
    // greedy: time weight of tile (I,J) = J updates of 2b^3 flops at the rate
    // of each class's update kernel (TFLOP/s): the caller's, or those the
    // kernels reach inside the factorization at N = 129,600 on MI355X (the
    // 16-bit and FP8 updates are bound by their output traffic, not by their
    // MFMA peaks)
    const double rate_default[4] = {61.0, 168.0, 770.0, 850.0};
    const double *rate = rates ? rates : rate_default;
    std::vector<uint8_t> cur((size_t)nt * nt, 0);
    double used = 0.0;
    struct Move {
        double ratio;
        int I, J, q;
    };
    for (;;) {
        Move best{-1.0, -1, -1, -1};
        for (int J = 0; J < nt; ++J)
            for (int I = J + w + 1; I < nt; ++I) {
                size_t t = I + (size_t)J * nt;
                int c = cur[t];
                for (int q = c + 1; q <= P8; ++q) {
                    if (!(h->o.allowed & (1u << q))) continue;
                    double add = 2.0 * (res[q][t] - (c == 0 ? 0.0 : res[c][t]));
                    if (!std::isfinite(add)) continue;
                    if (used + std::max(add, 0.0) > budget) continue;
                    double saved = (double)J * (1.0 / rate[c] - 1.0 / rate[q]);
                    double ratio = saved / std::max(add, 1e-300);
                    if (ratio > best.ratio) best = Move{ratio, I, J, q};
                }
            }
        if (best.I < 0) break;
        size_t t = best.I + (size_t)best.J * nt;
        int c = cur[t];
        used += 2.0 * (res[best.q][t] - (c == 0 ? 0.0 : res[c][t]));
        cur[t] = (uint8_t)best.q;
    }
    // verify; raise the worst tiles until the measured error fits
    double be = INFINITY;
    bool fits = false;
    for (int it = 0; it < 64; ++it) {
        rc = apply_map(h, MPCHOL_RULE_USER, eps, cur.data());
        if (rc) return rc;
        int64_t inf = 0;
        rc = run_factor(h, &inf);
        if (rc < 0) return rc;
        const bool broke = (rc == MPCHOL_NOT_SPD);
        std::vector<double> tr((size_t)nt * nt, 0.0);
        if (!broke) {
            rc = residual(h, &be, tr.data());
            if (rc) return rc;
            if (be <= eps) {
                fits = true;
                break;
            }
        } else {
            be = INFINITY;
        }
        // raise the 5% of lowered tiles with the largest residual by one level;
        // after a breakdown there is no residual of this map, so the tiles are
        // ranked by the residual measured for their class in the first phase
        std::vector<std::pair<double, size_t>> v;
        for (int J = 0; J < nt; ++J)
            for (int I = J + 1; I < nt; ++I) {
                size_t t = I + (size_t)J * nt;
                if (cur[t] > P64) v.push_back({broke ? res[cur[t]][t] : tr[t], t});
            }
        if (v.empty()) break;
        std::sort(v.begin(), v.end(), [](auto &a, auto &b2) { return a.first > b2.first; });
        size_t nr = std::max<size_t>(1, v.size() / 20);
        for (size_t i = 0; i < nr; ++i) {
            size_t t = v[i].second;
            int c = cur[t] - 1;
            while (c > P64 && !(h->o.allowed & (1u << c))) --c;
            cur[t] = (uint8_t)c;
        }
    }
    std::memcpy(labels, cur.data(), cur.size());
    if (berr_out) *berr_out = be;
    if (!fits) {
        // the map left in labels is the last one tried; it missed the budget or broke down
        snprintf(g_last_error, sizeof(g_last_error),
                 "mpchol_selector_labels: the raised map still misses the budget (backward error %.3e, eps %.3e)",
                 be, eps);
        return MPCHOL_EBUDGET;
    }
    return MPCHOL_OK;
}
