// Learned precision selector: tile features, the MLP 8 -> 64 -> 64 -> 4
// (ReLU, FP32) forward/backward/Adam kernels, the inference kernel that
// writes a precision map, and the trainer object of the C ABI.
#include <cmath>
#include <new>

#include "../../include/mpchol.h"
#include "common.h"
#include "launch.h"

namespace mpc {

constexpr int NF = 8, H1 = 64, H2 = 64, NC = 4;
constexpr int OW1 = 0, OB1 = OW1 + H1 * NF, OW2 = OB1 + H1, OB2 = OW2 + H2 * H1, OW3 = OB2 + H2, OB3 = OW3 + NC * H2;
constexpr int NP = OB3 + NC;
static_assert(NP == MPCHOL_MLP_NPARAM, "parameter layout");

__device__ inline double lg10c(double x) { return x > 0.0 ? fmax(log10(x), -40.0) : -40.0; }
__device__ inline int64_t degree_of(int64_t i)
{
    int64_t l = (int64_t)sqrt((double)i);
    while ((l + 1) * (l + 1) <= i) ++l;
    while (l * l > i) --l;
    return l;
}

__global__ void features_kernel(Tiles T, const double *fro2, const double *amax, double total, double eps, float *f)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = T.nt;
    if (t >= (int64_t)nt * nt) return;
    const int I = (int)(t % nt), J = (int)(t / nt);
    float *o = f + t * NF;
    if (I <= J) {
        for (int q = 0; q < NF; ++q) o[q] = 0.f;
        return;
    }
    const double b = T.b, NT = nt, ref = eps * total;
    const double Lw = (double)(degree_of(T.n - 1) + 1);
    const int64_t i0 = (int64_t)I * T.b, i1 = min((int64_t)(I + 1) * T.b, T.n) - 1;
    const int64_t vj = min((int64_t)T.b, T.n - (int64_t)J * T.b);
    const int64_t jm = (int64_t)J * T.b + vj / 2;
    o[0] = (float)lg10c(sqrt(fro2[t]) * NT / ref);
    o[1] = (float)lg10c(amax[t] * b * NT / ref);
    o[2] = (float)((double)(I - J) / NT);
    o[3] = (float)((double)degree_of(i0) / Lw);
    o[4] = (float)((double)degree_of(i1) / Lw);
    o[5] = (float)((double)degree_of(jm) / Lw);
    o[6] = (float)lg10c(sqrt(fro2[I + (int64_t)I * nt]) / total);
    o[7] = (float)lg10c(sqrt(fro2[J + (int64_t)J * nt]) / total);
}

__device__ inline void mlp_forward1(const float *P, const float *x, float *z)
{
    float h1[H1], h2[H2];
#pragma unroll 4
    for (int o = 0; o < H1; ++o) {
        float s = P[OB1 + o];
#pragma unroll
        for (int i = 0; i < NF; ++i) s += P[OW1 + o * NF + i] * x[i];
        h1[o] = s > 0.f ? s : 0.f;
    }
    for (int o = 0; o < H2; ++o) {
        float s = P[OB2 + o];
#pragma unroll 8
        for (int i = 0; i < H1; ++i) s += P[OW2 + o * H1 + i] * h1[i];
        h2[o] = s > 0.f ? s : 0.f;
    }
    for (int o = 0; o < NC; ++o) {
        float s = P[OB3 + o];
#pragma unroll 8
        for (int i = 0; i < H2; ++i) s += P[OW3 + o * H2 + i] * h2[i];
        z[o] = s;
    }
}

__device__ inline int argmax4(const float *z)
{
    int c = 0;
    for (int q = 1; q < NC; ++q)
        if (z[q] > z[c]) c = q;
    return c;
}

__global__ void infer_map_kernel(Tiles T, const float *P, const float *f, int band, unsigned allowed, uint8_t *map)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = T.nt;
    if (t >= (int64_t)nt * nt) return;
    const int I = (int)(t % nt), J = (int)(t / nt);
    int c = P64;
    if (I > J && I - J > band) {
        float z[NC];
        mlp_forward1(P, f + t * NF, z);
        c = argmax4(z);
        while (c > P64 && !(allowed & (1u << c))) --c;
    }
    map[t] = (uint8_t)((I >= J) ? c : 0);
}

__global__ void forward_kernel(const float *P, const float *X, int64_t nb, float *logits, int32_t *cls)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    float z[NC];
    mlp_forward1(P, X + s * NF, z);
    if (logits)
        for (int q = 0; q < NC; ++q) logits[s * NC + q] = z[q];
    if (cls) cls[s] = argmax4(z);
}

// Forward + backward of 64 samples per block; writes this block's summed
// parameter gradient (scaled by 1/nb) and loss into partials[block][NP + 1].
constexpr int SPB = 64;
__global__ __launch_bounds__(256) void grad_kernel(const float *P, const float *X, const int32_t *y, int64_t nb,
                                                   float cw0, float cw1, float cw2, float cw3, float alpha,
                                                   float *partials)
{
    __shared__ float xs[SPB][NF];
    __shared__ float h1[SPB][H1 + 1], h2[SPB][H2 + 1], g2[SPB][H2 + 1];
    __shared__ float dz[SPB][NC];
    __shared__ float ls[SPB];
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * SPB;
    const float cw[4] = {cw0, cw1, cw2, cw3};
    const float inv = 1.0f / (float)nb;
    for (int e = tid; e < SPB * NF; e += 256) {
        int s = e / NF, i = e % NF;
        xs[s][i] = (s0 + s < nb) ? X[(s0 + s) * NF + i] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < SPB * H1; e += 256) {
        int s = e / H1, o = e % H1;
        float a = P[OB1 + o];
        for (int i = 0; i < NF; ++i) a += P[OW1 + o * NF + i] * xs[s][i];
        h1[s][o] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < SPB * H2; e += 256) {
        int s = e / H2, o = e % H2;
        float a = P[OB2 + o];
        for (int i = 0; i < H1; ++i) a += P[OW2 + o * H1 + i] * h1[s][i];
        h2[s][o] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (tid < SPB) {
        const int s = tid;
        if (s0 + s < nb) {
            float z[NC];
            for (int c = 0; c < NC; ++c) {
                float a = P[OB3 + c];
                for (int i = 0; i < H2; ++i) a += P[OW3 + c * H2 + i] * h2[s][i];
                z[c] = a;
            }
            const int lab = y[s0 + s];
            float zm = z[0];
            for (int c = 1; c < NC; ++c) zm = fmaxf(zm, z[c]);
            float se = 0.f;
            for (int c = 0; c < NC; ++c) se += expf(z[c] - zm);
            float p[NC], pu = 0.f;
            for (int c = 0; c < NC; ++c) {
                p[c] = expf(z[c] - zm) / se;
                if (c > lab) pu += p[c];
            }
            ls[s] = cw[lab] * (-(z[lab] - zm - logf(se))) + alpha * pu;
            for (int c = 0; c < NC; ++c) {
                float g = cw[lab] * (p[c] - (c == lab ? 1.f : 0.f)) + alpha * p[c] * ((c > lab ? 1.f : 0.f) - pu);
                dz[s][c] = g * inv;
            }
        } else {
            ls[s] = 0.f;
            for (int c = 0; c < NC; ++c) dz[s][c] = 0.f;
        }
    }
    __syncthreads();
    for (int e = tid; e < SPB * H2; e += 256) {
        int s = e / H2, i = e % H2;
        float a = 0.f;
        for (int c = 0; c < NC; ++c) a += dz[s][c] * P[OW3 + c * H2 + i];
        g2[s][i] = h2[s][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // g1 overwrites h2's storage once g2 is complete (h2 is still needed for gW3)
    float *out = partials + (int64_t)blockIdx.x * (NP + 1);
    for (int e = tid; e < NC * H2; e += 256) {
        int c = e / H2, i = e % H2;
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += dz[s][c] * h2[s][i];
        out[OW3 + e] = a;
    }
    if (tid < NC) {
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += dz[s][tid];
        out[OB3 + tid] = a;
    }
    for (int e = tid; e < H2 * H1; e += 256) {
        int o = e / H1, i = e % H1;
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += g2[s][o] * h1[s][i];
        out[OW2 + e] = a;
    }
    if (tid < H2) {
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += g2[s][tid];
        out[OB2 + tid] = a;
    }
    __syncthreads();
    for (int e = tid; e < SPB * H1; e += 256) {
        int s = e / H1, i = e % H1;
        float a = 0.f;
        for (int o = 0; o < H2; ++o) a += g2[s][o] * P[OW2 + o * H1 + i];
        h2[s][i] = h1[s][i] > 0.f ? a : 0.f;  // g1
    }
    __syncthreads();
    for (int e = tid; e < H1 * NF; e += 256) {
        int o = e / NF, i = e % NF;
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += h2[s][o] * xs[s][i];
        out[OW1 + e] = a;
    }
    if (tid < H1) {
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += h2[s][tid];
        out[OB1 + tid] = a;
    }
    if (tid == 0) {
        float a = 0.f;
        for (int s = 0; s < SPB; ++s) a += ls[s];
        out[NP] = a * inv;
    }
}

__global__ void reduce_partials_kernel(const float *partials, int nblk, float *grad, float *loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    float a = 0.f;
    for (int k = 0; k < nblk; ++k) a += partials[(int64_t)k * (NP + 1) + p];
    if (p < NP) grad[p] = a;
    else if (loss) *loss = a;
}

__global__ void adam_kernel(float *P, const float *g, float *m, float *v, int64_t np, float lr, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float mi = b1 * m[i] + (1.f - b1) * g[i];
    float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_features(const Tiles &T, const double *fro2, const double *amax, double total, double eps, float *feats,
                     hipStream_t st)
{
    int64_t cnt = (int64_t)T.nt * T.nt;
    features_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(T, fro2, amax, total, eps, feats);
}

void launch_mlp_infer_map(const Tiles &T, const float *params, const float *feats, int band, unsigned allowed,
                          uint8_t *map_out, hipStream_t st)
{
    int64_t cnt = (int64_t)T.nt * T.nt;
    infer_map_kernel<<<(unsigned)((cnt + 127) / 128), 128, 0, st>>>(T, params, feats, band, allowed, map_out);
}

void launch_mlp_forward(const float *params, const float *X, int64_t nb, float *logits, int32_t *cls, hipStream_t st)
{
    forward_kernel<<<(unsigned)((nb + 127) / 128), 128, 0, st>>>(params, X, nb, logits, cls);
}

void launch_mlp_grad(const float *params, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                     float *grad, float *loss, float *partials, hipStream_t st)
{
    int nblk = (int)((nb + SPB - 1) / SPB);
    grad_kernel<<<nblk, 256, 0, st>>>(params, X, y, nb, cw[0], cw[1], cw[2], cw[3], alpha, partials);
    reduce_partials_kernel<<<(NP + 1 + 255) / 256, 256, 0, st>>>(partials, nblk, grad, loss);
}

void launch_adam(float *params, const float *grad, float *m, float *v, int64_t np, int step, float lr, hipStream_t st)
{
    float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
    adam_kernel<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(params, grad, m, v, np, lr, c1, c2);
}

}  // namespace mpc

// ---------------------------------------------------------------- trainer ABI
using namespace mpc;

struct mpchol_mlp {
    int dev = 0;
    hipStream_t st = nullptr;
    float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *loss = nullptr;
    float *partials = nullptr;
    int64_t cap = 0;  // samples the partials buffer holds
    int step = 0;
};

static int mlp_ensure(mpchol_mlp *t, int64_t nb)
{
    if (nb <= t->cap) return MPCHOL_OK;
    if (t->partials) (void)hipFree(t->partials);
    t->partials = nullptr;
    int64_t nblk = (nb + SPB - 1) / SPB;
    if (hipMalloc((void **)&t->partials, (size_t)nblk * (NP + 1) * 4) != hipSuccess) {
        (void)hipGetLastError();
        t->cap = 0;
        return MPCHOL_ENOMEM;
    }
    t->cap = nblk * SPB;
    return MPCHOL_OK;
}

extern "C" {

int mpchol_mlp_create(mpchol_mlp_t *mp, int32_t device, void *stream)
{
    if (!mp) return MPCHOL_EINVAL;
    *mp = nullptr;
    if (hipSetDevice(device) != hipSuccess) return MPCHOL_EHIP;
    mpchol_mlp *t = new (std::nothrow) mpchol_mlp();
    if (!t) return MPCHOL_ENOMEM;
    t->dev = device;
    t->st = (hipStream_t)stream;
    bool ok = hipMalloc((void **)&t->P, NP * 4) == hipSuccess && hipMalloc((void **)&t->m, NP * 4) == hipSuccess &&
              hipMalloc((void **)&t->v, NP * 4) == hipSuccess && hipMalloc((void **)&t->g, NP * 4) == hipSuccess &&
              hipMalloc((void **)&t->loss, 4) == hipSuccess;
    if (ok) ok = hipMemset(t->m, 0, NP * 4) == hipSuccess && hipMemset(t->v, 0, NP * 4) == hipSuccess &&
                 hipMemset(t->P, 0, NP * 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        mpchol_mlp_destroy(t);
        return MPCHOL_ENOMEM;
    }
    *mp = t;
    return MPCHOL_OK;
}

int mpchol_mlp_destroy(mpchol_mlp_t t)
{
    if (!t) return MPCHOL_OK;
    (void)hipSetDevice(t->dev);
    (void)hipStreamSynchronize(t->st);
    float *ps[] = {t->P, t->m, t->v, t->g, t->loss, t->partials};
    for (float *p : ps)
        if (p) (void)hipFree(p);
    delete t;
    return MPCHOL_OK;
}

int mpchol_mlp_set_params(mpchol_mlp_t t, const float *params, int64_t np)
{
    if (!t || !params || np != NP) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(t->P, params, NP * 4, hipMemcpyHostToDevice, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemsetAsync(t->m, 0, NP * 4, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemsetAsync(t->v, 0, NP * 4, t->st) != hipSuccess) return MPCHOL_EHIP;
    t->step = 0;
    return hipStreamSynchronize(t->st) == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_mlp_get_params(mpchol_mlp_t t, float *params, int64_t np)
{
    if (!t || !params || np != NP) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(params, t->P, NP * 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
    return hipStreamSynchronize(t->st) == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_mlp_get_state(mpchol_mlp_t t, float *params, float *m1, float *m2, int32_t *step, int64_t np)
{
    if (!t || !params || !m1 || !m2 || !step || np != NP) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(params, t->P, NP * 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(m1, t->m, NP * 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(m2, t->v, NP * 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipStreamSynchronize(t->st) != hipSuccess) return MPCHOL_EHIP;
    *step = t->step;
    return MPCHOL_OK;
}

int mpchol_mlp_set_state(mpchol_mlp_t t, const float *params, const float *m1, const float *m2, int32_t step,
                         int64_t np)
{
    if (!t || !params || !m1 || !m2 || step < 0 || np != NP) return MPCHOL_EINVAL;
    for (int64_t i = 0; i < NP; ++i)  // Adam's second moment is a running mean of squares
        if (!(m2[i] >= 0.0f)) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(t->P, params, NP * 4, hipMemcpyHostToDevice, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(t->m, m1, NP * 4, hipMemcpyHostToDevice, t->st) != hipSuccess) return MPCHOL_EHIP;
    if (hipMemcpyAsync(t->v, m2, NP * 4, hipMemcpyHostToDevice, t->st) != hipSuccess) return MPCHOL_EHIP;
    t->step = step;
    return hipStreamSynchronize(t->st) == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_mlp_grad(mpchol_mlp_t t, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                    float *grad, float *loss)
{
    if (!t || !X || !y || nb <= 0 || !cw || !grad) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    int rc = mlp_ensure(t, nb);
    if (rc) return rc;
    launch_mlp_grad(t->P, X, y, nb, cw, alpha, grad, t->loss, t->partials, t->st);
    if (loss) {
        if (hipMemcpyAsync(loss, t->loss, 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
        if (hipStreamSynchronize(t->st) != hipSuccess) return MPCHOL_EHIP;
    }
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_mlp_train_step(mpchol_mlp_t t, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                          float lr, float *loss)
{
    if (!t || !X || !y || nb <= 0 || !cw || !(lr > 0)) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    int rc = mlp_ensure(t, nb);
    if (rc) return rc;
    launch_mlp_grad(t->P, X, y, nb, cw, alpha, t->g, t->loss, t->partials, t->st);
    t->step += 1;
    launch_adam(t->P, t->g, t->m, t->v, NP, t->step, lr, t->st);
    if (loss) {
        if (hipMemcpyAsync(loss, t->loss, 4, hipMemcpyDeviceToHost, t->st) != hipSuccess) return MPCHOL_EHIP;
        if (hipStreamSynchronize(t->st) != hipSuccess) return MPCHOL_EHIP;
    }
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

int mpchol_mlp_predict(mpchol_mlp_t t, const float *X, int64_t nb, float *logits, int32_t *cls)
{
    if (!t || !X || nb <= 0 || (!logits && !cls)) return MPCHOL_EINVAL;
    if (hipSetDevice(t->dev) != hipSuccess) return MPCHOL_EHIP;
    launch_mlp_forward(t->P, X, nb, logits, cls, t->st);
    return hipGetLastError() == hipSuccess ? MPCHOL_OK : MPCHOL_EHIP;
}

}  // extern "C"
