// Host-side launchers of the mpchol kernels (all enqueue on `st`, no sync).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

// Where the tiles live (device pointers), passed to kernels by value.
struct Tiles {
    char *slots;          // packed lower tiles, tile_index(I,J) * slot_bytes
    int64_t slot_bytes;   // b*b*8
    int b, nt;
    int64_t n;
    const uint8_t *map;   // nt*nt classes, entry I + J*nt
    int32_t *tscale;      // nt*nt stored scale exponents
    int lo16;
    int lo32;             // FP32-class updates: 0 FP32 MFMA, 1 three-way BF16 split products
    int lo8 = 0;          // FP8-class copies: 0 one scale per tile, 1 E8M0 scale per 32 K elements of a row
};

// Source of Sigma: the generator (sigma, x, rho, nugget), a kept FP64 copy
// in the packed tile layout (orig != nullptr), or a caller's column-major
// matrix whose lower part is read (dense != nullptr, leading dimension ld;
// norms and residuals only).
struct Source {
    const double *sigma, *x;
    double rho, nugget;
    const double *orig;
    const double *dense = nullptr;
    int64_t ld = 0;
};

// Panel copies of the current step: one b*b buffer per panel row tile I.
struct Panel {
    double *p64;      // column-major
    float *p32;       // column-major
    uint16_t *p16;    // row-major (k contiguous)
    uint8_t *p8;      // row-major (k contiguous)
    unsigned long long *pmax;  // nt: max |X| of the TRSM output of tile I (FP64 bits)
    int32_t *pscale;           // nt*4: scale exponent of the class-q copy of tile I
    uint16_t *p32s;            // lo32 split: hi, mid, lo BF16 parts of the FP32 copy, each b*b row-major
    int8_t *poz = nullptr;     // lo64 INT8: per tile 15 residue planes of b*b bytes, row-major
    int32_t *pexp = nullptr;   // lo64 INT8: per tile b row exponents
    uint8_t *p8x = nullptr;    // lo8 MX: per tile b rows x b/32 E8M0 bytes, row-major (block kb of row r at r*b/32 + kb)
    unsigned long long *info = nullptr;  // breakdown column (1-based, atomic minimum): the panel TRSM
                                         // reports the first column where it writes an Inf or NaN
};

// ---- tiles (k_tiles.hip)
void launch_norms(const Tiles &T, const Source &S, double *fro2, double *amax, hipStream_t st);
void launch_load(const Tiles &T, const Source &S, hipStream_t st);
void launch_copy_matrix(const Tiles &T, const double *A, int64_t lda, double *orig, hipStream_t st);
void launch_convert(const Tiles &T, const Panel &P, int k, const uint8_t *qmask, hipStream_t st);
void launch_logdet(const Tiles &T, double *out, hipStream_t st);
void launch_get_factor(const Tiles &T, double *L, int64_t ldl, hipStream_t st);
void launch_zero_upper_diag(const Tiles &T, int k, hipStream_t st);

// ---- factorization (k_factor.hip)
void launch_potrf_tile(const Tiles &T, int k, unsigned long long *info, hipStream_t st);
void launch_trsm_panel(const Tiles &T, const Panel &P, int k, hipStream_t st);
// grouped update A_IJ -= sum_h L_I,k_h L_J,k_h^T of class q over `nitems` packed (I << 16 | J)
// items from the npan panels Ps[0..npan-1] (npan <= 2 for FP64 and FP32-MFMA, <= 4 otherwise);
// small: block shapes that fit beside running update blocks.
void launch_update(const Tiles &T, const Panel *const *Ps, int npan, int q, const int32_t *items, int nitems,
                   hipStream_t st, bool small);

// ---- FP64-class updates from INT8 products (k_ozaki.hip)
struct OzakiConst;
void ozaki_const_init(OzakiConst *k);
// sender side of step k for panel tiles with qmask bit 4: row exponents and residue planes
void launch_ozaki_convert(const Tiles &T, const Panel &P, int k, const uint8_t *qmask, const OzakiConst *K,
                          hipStream_t st);
void launch_ozaki_update(const Tiles &T, const Panel &P, const Panel *P2, const int32_t *items, int nitems,
                         const OzakiConst *K, hipStream_t st);

// ---- residual (k_residual.hip): items = every lower tile as (I << 16 | J);
// partial = scratch of nitems * (b/128)^2 doubles; tile_res2 = nt*nt output
void launch_residual_items(const Tiles &T, const Source &S, const int32_t *items, int nitems, double *partial,
                           double *tile_res2, hipStream_t st);

// ---- backward-error estimate (k_estimate.hip): scratch 3*nt*b*probes doubles,
// zbuf n*probes floats; *out = sum over the probes of ||(Sigma - L L^T) v||^2
void launch_estimate(const Tiles &T, const Source &S, bool sorted, uint64_t seed, double *scratch, float *zbuf,
                     double *out, hipStream_t st);
int estimate_chunks(int64_t n);

// ---- covariance from samples (k_samples.hip)
// xp: (NT*b) x mp scratch (mp = m rounded up to 16); orig: the kept copy.
int launch_cov_samples(const Tiles &T, const double *xi, int64_t ldxi, int64_t m, double scale, double nugget,
                       double *xp, int64_t mp, double *orig, hipStream_t st);
int estimate_probes();

// ---- solve, sample (k_apply.hip)
void launch_solve(const Tiles &T, double *B, int64_t ldb, int nrhs, hipStream_t st);
void launch_normal_draws(uint64_t seed, int64_t count, float *z, uint32_t *raw, hipStream_t st);
void launch_normal_matrix(uint64_t seed, int64_t n, int ndraws, float *Z, int64_t ldz, hipStream_t st);
// draws of columns d0 .. d0+nd-1 of the n x ndraws sequence into Z's columns 0 .. nd-1
void launch_normal_columns(uint64_t seed, int64_t n, int64_t d0, int nd, float *Z, int64_t ldz, hipStream_t st);
void launch_lower_apply(const Tiles &T, const float *Z, int64_t ldz, float *Y, int64_t ldy, int ndraws, hipStream_t st);

// ---- selector (k_mlp.hip)
void launch_features(const Tiles &T, const double *fro2, const double *amax, double total, double eps, float *feats,
                     hipStream_t st);
void launch_mlp_infer_map(const Tiles &T, const float *params, const float *feats, int band, unsigned allowed,
                          uint8_t *map_out, hipStream_t st);
void launch_mlp_forward(const float *params, const float *X, int64_t nb, float *logits, int32_t *cls, hipStream_t st);
void launch_mlp_grad(const float *params, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                     float *grad, float *loss, float *partials, hipStream_t st);
void launch_adam(float *params, const float *grad, float *m, float *v, int64_t np, int step, float lr, hipStream_t st);

}  // namespace mpc
