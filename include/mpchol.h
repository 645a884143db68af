/*
 * mpchol.h -- mixed-precision tile Cholesky of a dense SPD covariance on one
 * AMD Instinct MI355X (gfx950), and the products built on the factor.
 *
 * The operation (paper Sec. III.A.3): factor the covariance of the
 * spherical-harmonic coefficient vectors, U = V V^T with V lower triangular,
 * and use V for the log-determinant, for solves, and for emulation draws
 * xi = V z with z ~ N(0, I) (Sec. III.B).  The factorization is the tile
 * algorithm whose tasks are POTRF, TRSM, SYRK and GEMM (Sec. II.C, Sec. V.A),
 * with a precision chosen per tile (Sec. III.D; precision variants Sec. IV.B)
 * and the conversion of each panel tile done once by its producer for all of
 * its consumers (Sec. V.A).
 *
 * Conventions for every call:
 *   - Return value: MPCHOL_OK (0), MPCHOL_NOT_SPD (1) or a negative error code.
 *     No exception or C++ type crosses this interface.
 *   - Matrices are column-major; "device" pointers are HIP device memory of
 *     the handle's device, "host" pointers are ordinary host memory.
 *   - Pointers need to stay valid only for the duration of the call; the
 *     library copies what it keeps.  The handle owns all tile storage.
 *   - All device work is ordered on the handle's stream.  Calls that return a
 *     host scalar (logdet, backward_error, get_stats, factor's info)
 *     synchronize that stream; the others only enqueue.
 *   - A handle is single-threaded: calls on one handle must not overlap.
 *   - Call order: create -> set_matrix | set_generator -> precision_map ->
 *     factor -> {logdet, solve, sample, backward_error, get_factor}.  A call
 *     made out of order returns MPCHOL_EORDER and changes nothing.
 */
#ifndef MPCHOL_H
#define MPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MPCHOL_OK 0
#define MPCHOL_NOT_SPD 1       /* a diagonal pivot was not positive (or NaN), or the factor took an Inf or NaN */
#define MPCHOL_EINVAL (-1)     /* invalid argument */
#define MPCHOL_ENOMEM (-2)     /* device allocation failed */
#define MPCHOL_EHIP (-3)       /* a HIP runtime call failed */
#define MPCHOL_EORDER (-4)     /* call out of order (see above) */
#define MPCHOL_EBUDGET (-5)    /* backward-error budget missed after every fallback */
#define MPCHOL_EUNSUPPORTED (-6)

/* precision classes of a tile (the codes of a precision map) */
#define MPCHOL_P64 0 /* FP64 storage and FP64 arithmetic */
#define MPCHOL_P32 1 /* FP32 storage, FP32 products and accumulation */
#define MPCHOL_P16 2 /* 16-bit storage (FP16 with a per-tile power-of-two scale, or BF16), FP32 accumulation */
#define MPCHOL_P8 3  /* OCP FP8 E4M3FN with a per-tile power-of-two scale, FP32 accumulation */

/* which 16-bit format the P16 class uses */
#define MPCHOL_LO16_F16 0
#define MPCHOL_LO16_BF16 1
#define MPCHOL_LO32_FP32 0
#define MPCHOL_LO32_BF16X3 1
/* how FP64-class tile products are formed */
#define MPCHOL_LO64_FP64 0 /* on the FP64 MFMA */
#define MPCHOL_LO64_INT8 1 /* exact integer products from INT8 residues (see mpchol_opts.lo64) */
/* how the FP8-class operands are scaled */
#define MPCHOL_LO8_TILE 0 /* one power-of-two scale per panel tile, applied to the accumulated product */
#define MPCHOL_LO8_MX 1   /* one E8M0 scale per 32 consecutive K elements of a row (see mpchol_opts.lo8) */

/* precision-map rules */
#define MPCHOL_RULE_FP64 0    /* every tile FP64 (the plain FP64 path) */
#define MPCHOL_RULE_NORM 1    /* tile-centric norm rule (Sec. III.D "numeric features of the tile") */
#define MPCHOL_RULE_BAND 2    /* band rule (Sec. III.D band-based; variants DP/SP, DP/SP/HP, DP/HP of Sec. IV.B) */
#define MPCHOL_RULE_USER 3    /* caller-supplied map */
#define MPCHOL_RULE_LEARNED 4 /* learned selector (MLP inference kernel) with the norm rule as fallback */

/* band variants for MPCHOL_RULE_BAND (Sec. IV.B) */
#define MPCHOL_BAND_DP_SP 1    /* band in FP64, the rest FP32 */
#define MPCHOL_BAND_DP_SP_HP 2 /* band in FP64, the next band holding >= 5% of the off-diagonal tiles FP32, rest 16-bit */
#define MPCHOL_BAND_DP_HP 3    /* band in FP64, the rest 16-bit */

typedef struct mpchol_handle *mpchol_t;

typedef struct mpchol_opts {
    int32_t device;      /* HIP device ordinal */
    void *stream;        /* hipStream_t to order all work on; NULL = the null stream */
    int32_t lo16;        /* MPCHOL_LO16_F16 or MPCHOL_LO16_BF16 */
    int32_t band;        /* tiles with |I-J| <= band stay FP64 under NORM, BAND and LEARNED (default 1) */
    uint32_t allowed;    /* bit mask of allowed classes (bit p for class p); FP64 is always allowed */
    int32_t band_variant;/* MPCHOL_BAND_* used by MPCHOL_RULE_BAND */
    int32_t verify;      /* LEARNED rule: check the backward error after factor and fall back on violation:
                            0 off, 1 exact FP64 residual, 2 randomized estimate (64 probes, 3-sigma margin) */
    double verify_eps;   /* backward-error budget used by verify */
    int32_t profile;     /* nonzero: time every update-GEMM launch with events (adds event overhead) */
    int32_t lo32;        /* arithmetic of the FP32-class updates: MPCHOL_LO32_FP32 (FP32 MFMA) or
                            MPCHOL_LO32_BF16X3 (each FP32 operand split into three BF16 parts, the six
                            significant part products on the BF16 MFMA, FP32 accumulation); storage,
                            conversion and the map rule are the same for both; default BF16X3 */
    int32_t lo64;        /* arithmetic of the FP64-class GEMM updates of tiles farther than `band` from the
                            diagonal under a mixed rule (NORM, BAND, USER, LEARNED): MPCHOL_LO64_FP64 (FP64
                            MFMA) or MPCHOL_LO64_INT8 -- the Ozaki scheme II (Ozaki, Uchino and Imamura):
                            each row of an FP64 panel copy scaled by 2^e so that its maximum lies in
                            [2^52, 2^53) and rounded to integers (ties to even), the integer product formed
                            exactly from INT8 MFMA products modulo 15 coprime moduli <= 256 and the Chinese
                            remainder theorem, rounded once to FP64 and scaled back; the FP64 work tile
                            accumulates as before.  SYRK, the tiles within `band` and the plain FP64 path
                            (rule FP64) stay on the FP64 MFMA.  Tiles up to 1024 (else MPCHOL_EUNSUPPORTED
                            at create); needs 6 NT tile^2 15 bytes more panel memory (six panel copy
                            sets).  Default FP64. */
    int32_t lo8;         /* scaling of the FP8-class products: MPCHOL_LO8_TILE (the E4M3 copy of a panel
                            tile takes one power-of-two scale from the tile's largest |value|, and the
                            accumulated product is scaled back) or MPCHOL_LO8_MX -- block scaling in the
                            manner of the OCP Microscaling formats: every run of 32 consecutive elements of
                            a row of the copy (the K direction of the products) takes its own power-of-two
                            scale 2^-t, t the largest integer with (block max |value|) 2^t <= 448 (no
                            element saturates; t clamped to [-127, 127]), stored as the E8M0 byte 127 - t
                            and applied inside the block-scaled FP8 MFMA.  Only the FP8 copies of the
                            panel tiles change: stored FP8 tiles keep their per-tile scale, and the map
                            rule prices the class with the same unit roundoff 2^-4.  Needs 6 NT tile^2 / 32
                            bytes more panel memory.  Default TILE. */
} mpchol_opts;

typedef struct mpchol_stats {
    int64_t n;
    int32_t tile, nt;
    int64_t tiles_per_class[4];  /* strict-lower tiles per class */
    double flops_per_class[4];   /* task flops by class: POTRF b^3/3, TRSM b^3, SYRK b^3 in FP64, GEMM 2b^3 in its class */
    double total_fro;            /* ||Sigma||_F of the valid part */
    double t_map_ms;             /* last precision_map: norms, rule, load into work tiles */
    double t_factor_ms;          /* last factor (all of its kernels, conversions included) */
    double t_solve_ms, t_sample_ms, t_residual_ms;
    double t_gemm_ms[4];         /* profile mode: summed update-GEMM kernel time per class in the last factor */
    int64_t gemm_launches[4];    /* profile mode: number of those launches */
    double gemm_flops[4];        /* task flops of those launches: 2b^3 per GEMM and b^3 per SYRK item and step */
    int32_t fallbacks;           /* refactorizations made by verify */
    int32_t rule_used;           /* rule of the map the last factor ran with */
    double verify_first;         /* backward error (exact or estimated) of the first map verify judged;
                                    +inf if that map's factorization broke down; -1 if no map was verified */
    double t_samples_ms;         /* last set_samples: the covariance product (ms) */
    double t_gemm_int8_ms;       /* profile mode: FP64-class update launches formed from INT8 products (lo64) */
    int64_t gemm_int8_launches;
    double gemm_int8_flops;      /* their task flops (2b^3 per item and step) */
} mpchol_stats;

/* Default options: device 0, null stream, FP16, band 1, all classes allowed. */
void mpchol_default_opts(mpchol_opts *o);

/* Create a handle for an n x n matrix in tiles of tile x tile (tile a multiple
 * of 128, 128..2048).  n need not be a multiple of tile: the last tile row and
 * column are padded with an identity block, which changes neither the factor
 * nor the log-determinant.  Allocates the tile storage (about
 * NT(NT+1)/2 * tile^2 * 8 bytes) and the panel buffers on o->device.
 * o may be NULL (defaults).  On error *h is NULL. */
int mpchol_create(mpchol_t *h, int64_t n, int32_t tile, const mpchol_opts *o);

/* Free everything the handle owns.  Accepts NULL. */
int mpchol_destroy(mpchol_t h);

/* Use the caller's matrix A (lower part read, lda >= n).  on_device: A is
 * device memory (else host).  The lower tiles are copied into a device
 * FP64 copy kept for later loads and residuals. */
int mpchol_set_matrix(mpchol_t h, const double *A, int64_t lda, int32_t on_device);

/* Use the synthetic covariance generated on the device on demand,
 *   Sigma_ij = sigma_i sigma_j exp(-|x_i - x_j| / rho) + nugget delta_ij,
 * the exponential kernel over the ordered coefficient index with the
 * diagonal perturbation that keeps it positive definite (Sec. III.A.3).
 * sigma and x: host arrays of n doubles; rho > 0; nugget >= 0. */
int mpchol_set_generator(mpchol_t h, const double *sigma, const double *x, double rho, double nugget);

/* Use the covariance estimated from samples (Sec. III.A.3, "Modeling the Temporal
 * Dependence and Constructing a Covariance Matrix": the average of the outer
 * products of the R(T-P) residual vectors, with a small diagonal perturbation
 * when there are fewer samples than L^2):
 *   Sigma = scale * Xi Xi^T + nugget * I,
 * Xi the n x m samples, column-major with leading dimension ldxi >= n, in
 * host memory (or device memory if on_device); e.g. scale = 1/(R(T-P)).
 * Computed on the GPU by a tall-skinny FP64 MFMA SYRK into the kept FP64
 * copy, which maps, factor and residuals then read as after set_matrix.  The
 * caller keeps ownership of Xi.  Temporary device memory: (NT*b) x
 * roundup(m, 16) doubles, plus n x m for host input.  Synchronizes; the
 * product's time goes to stats.t_samples_ms.  EINVAL for null pointers,
 * ldxi < n, m < 1, scale <= 0 or nugget < 0. */
int mpchol_set_samples(mpchol_t h, const double *xi, int64_t ldxi, int64_t m, double scale, double nugget,
                       int32_t on_device);

/* Choose the precision of every tile and load Sigma into the work tiles.
 * Computes tile norms (FP64 on the device), applies `rule` with accuracy
 * target eps (NORM: the lowest allowed class p with
 * ||Sigma_IJ||_F u_p <= eps ||Sigma||_F / NT; tiles within the band and the
 * diagonal stay FP64), then writes Sigma into FP64 work tiles (FP64 class)
 * or FP32 work tiles (every lower class).
 * user_map: host NT x NT uint8, column-major (entry I + J*NT), lower part
 * read, required for RULE_USER, ignored otherwise (diagonal forced FP64).
 * map_out: optional host NT x NT uint8 receiving the map (strict upper = 0).
 * Synchronizes. */
int mpchol_precision_map(mpchol_t h, int32_t rule, double eps, const uint8_t *user_map, uint8_t *map_out);

/* Factor the loaded matrix in place (right-looking tile algorithm, Sec. V.A).
 * *info = 0 on success, else the smallest 1-based global column of a failing
 * pivot or of an Inf or NaN in an off-diagonal factor tile, as the panel
 * solve writes it -- also where the tile is stored in a format that would
 * saturate it (returns MPCHOL_NOT_SPD).  Under RULE_LEARNED with opts.verify set,
 * a backward error above opts.verify_eps (or a failing pivot) triggers a
 * refactorization under RULE_NORM and then RULE_FP64 (counted in stats);
 * MPCHOL_EBUDGET if all fail.  Synchronizes once at the end. */
int mpchol_factor(mpchol_t h, int64_t *info);

/* log det(Sigma) = 2 sum log diag(L), summed in FP64.  Synchronizes. */
int mpchol_logdet(mpchol_t h, double *out);

/* Overwrite device B (n x nrhs, ldb >= n, FP64) with Sigma^-1 B by forward
 * and backward tile substitution; diagonal blocks in FP64, off-diagonal
 * updates read each tile in its stored precision, exactly widened to FP64. */
int mpchol_solve(mpchol_t h, int32_t nrhs, double *B, int64_t ldb);

/* Emulation draws (Sec. III.B): device Y (n x ndraws, ldy >= n, FP32) =
 * L Z with Z ~ N(0, I) generated on the device by Philox4x32-10 (key =
 * seed) and Box-Muller in FP32; draw e (column-major index of Z) uses counter
 * block e/4, entry e%4.  Tiles are read in their stored precision. */
int mpchol_sample(mpchol_t h, int32_t ndraws, uint64_t seed, float *Y, int64_t ldy);

/* As mpchol_sample with a caller-supplied device Z (n x ndraws, FP32). */
int mpchol_sample_z(mpchol_t h, int32_t ndraws, const float *Z, int64_t ldz, float *Y, int64_t ldy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same draws as
 * mpchol_sample -- Y (device, n x ndraws, ldy >= n, FP32) gets the values
 * mpchol_sample(h, ndraws, seed, Y, ldy) writes, bit for bit -- without any
 * allocation.  Z is generated into a fixed 64 MiB buffer that the library
 * holds per device (16,777,216 FP32 values, kept until the process ends) in
 * passes of as many whole draw columns as fit, each pass multiplied by L
 * before the next is generated.  Only enqueues on the handle's stream (no
 * synchronization).  Every call on one device shares that device's buffer:
 * calls that may overlap on one GPU (other handles, streams or threads)
 * race and must be serialized by the caller.  Errors: MPCHOL_EINVAL for null
 * pointers, ndraws <= 0, ldy < n, or n > 16,777,216 (one draw column must
 * fit the buffer); MPCHOL_EORDER before a successful factor; MPCHOL_EHIP if
 * the buffer's device address could not be looked up. */
int mpchol_sample_noalloc(mpchol_t h, int32_t ndraws, uint64_t seed, float *Y, int64_t ldy);

/* The draw sequence alone: device z (count FP32 normals) and optional device
 * raw (count uint32 Philox outputs), same mapping as mpchol_sample. */
int mpchol_normal_draws(mpchol_t h, int64_t count, uint64_t seed, float *z, uint32_t *raw);

/* Relative backward error ||Sigma - L L^T||_F / ||Sigma||_F with the stored
 * factor exactly widened to FP64 and FP64 accumulation.  Sigma comes from the
 * generator or the kept copy of set_matrix.  tile_res2 (optional host NT x NT
 * doubles, column-major) receives the squared residual norm of each lower
 * tile (strict-lower entries of a diagonal tile counted twice).  Synchronizes. */
int mpchol_backward_error(mpchol_t h, double *berr, double *tile_res2);

/* The same ratio against a caller's matrix A (Sec. III.A.3: the factor of
 * the covariance is judged by ||A - L L^T||_F / ||A||_F):
 * A column-major n x n, lower part read (lda >= n), in device memory if
 * on_device, else host memory (copied to a temporary device buffer).  The
 * stored factor is exactly widened to FP64; FP64 accumulation; ||A||_F is
 * computed from A's lower part.  tile_res2 as in mpchol_backward_error.
 * Temporary device memory: 2 NT^2 doubles, plus the copy of a host A.
 * Synchronizes.  MPCHOL_EINVAL for null pointers, lda < n or A = 0. */
int mpchol_backward_error_matrix(mpchol_t h, const double *A, int64_t lda, int32_t on_device, double *berr,
                                 double *tile_res2);

/* Randomized estimate of the same ratio: with `sets` x 64 probe vectors v
 * (N(0,1) entries from Philox with key derived from `seed`),
 * ||Sigma - L L^T||_F^2 = E ||(Sigma - L L^T) v||^2, and each product costs
 * O(N^2) (L (L^T v) with the stored tiles widened to FP64; Sigma v from the
 * kept copy of set_matrix, or from the generator -- in O(N) per probe by the
 * exponential kernel's two-sided recursion when its coordinates are
 * nondecreasing).  Relative standard deviation of the estimate about
 * 1/sqrt(128 sets).  verify = 2 uses one set.  Synchronizes. */
int mpchol_backward_error_estimate(mpchol_t h, int32_t sets, uint64_t seed, double *est);

/* Copy the factor's represented values into device L (n x n FP64, ldl >= n;
 * the strict upper part is zeroed).  Valid after a successful factor. */
int mpchol_get_factor(mpchol_t h, double *L, int64_t ldl);

/* Host copy of the per-tile stored scale exponents (NT x NT int32,
 * column-major): tile (I,J) represents values code * 2^-t. */
int mpchol_get_tile_scales(mpchol_t h, int32_t *t);

/* Change the verification of learned maps (mode 0 off, 1 exact, 2 estimate;
 * eps the budget) for the following factor calls. */
int mpchol_set_verify(mpchol_t h, int32_t mode, double eps);

/* Fill *s (synchronizes). */
int mpchol_get_stats(mpchol_t h, mpchol_stats *s);

/* Static description of a status code. */
const char *mpchol_strerror(int status);

/* Text of the last HIP failure seen by a call on this thread (the failing
 * runtime call and its error string); empty if none.  Owned by the library,
 * valid until the next call on this thread. */
const char *mpchol_last_error(void);

/* ---- learned precision selector -------------------------------------- */
/* A multilayer perceptron 8 -> 64 -> 64 -> 4 (ReLU, FP32) mapping tile
 * features to the classes {P64, P32, P16, P8}.  Parameter vector (FP32,
 * MPCHOL_MLP_NPARAM values, row-major out x in): W1[64*8] b1[64] W2[64*64]
 * b2[64] W3[4*64] b3[4].
 * Features of tile (I,J) (FP32, computed on the device from FP64 norms):
 *   f0 = log10(||S_IJ||_F NT / (eps ||S||_F))      f1 = log10(max|S_IJ| b NT / (eps ||S||_F))
 *   f2 = (I-J)/NT   f3 = l(first row of I)/Lw   f4 = l(last row of I)/Lw   f5 = l(middle column of J)/Lw
 *   f6 = log10(||S_II||_F/||S||_F)   f7 = log10(||S_JJ||_F/||S||_F)
 * with l(i) = floor(sqrt(i)) the spherical-harmonic degree of index i,
 * Lw = floor(sqrt(n-1)) + 1, and log10 of zero taken as -40. */
#define MPCHOL_MLP_NPARAM 4996

/* Set the selector weights used by RULE_LEARNED (host, nparam floats). */
int mpchol_selector_set(mpchol_t h, const float *params, int64_t nparam);

/* Host copy of the features of every strict-lower tile after a
 * precision_map call: feats (NT*NT x 8, row-major by tile index I + J*NT;
 * entries outside the strict lower part are zero).  eps as in the map. */
int mpchol_selector_features(mpchol_t h, double eps, float *feats);

/* Labels by greedy per-tile lowering under a measured backward-error budget:
 * factor with every off-band tile at each class to measure per-tile
 * residuals, lower tiles greedily by (estimated time saved)/(added squared
 * residual) while the total stays within (eps ||S||_F)^2 / 2, then verify
 * with one factorization and raise the worst tiles until it holds (at most
 * 64 rounds; after a breakdown the tiles are ranked by the residual measured
 * for their class).  The greedy weighs a tile's time by the update rate of
 * each class (FP64, FP32, 16-bit, FP8): rates (optional host double[4],
 * TFLOP/s, all > 0), else those of this library's update kernels inside the
 * factorization at N = 129,600 (61, 168, 770, 850).  labels: host NT x NT
 * uint8 (the resulting map); *berr_out its measured backward error (+inf
 * after a breakdown).  MPCHOL_EBUDGET if no round met the budget (labels
 * then hold the last map tried).  The handle must have a matrix set; its
 * tiles are reloaded and refactored several times. */
int mpchol_selector_labels(mpchol_t h, double eps, uint8_t *labels, double *berr_out, const double *rates);

typedef struct mpchol_mlp *mpchol_mlp_t;

/* Trainer object on the given device/stream (stream may be NULL). */
int mpchol_mlp_create(mpchol_mlp_t *m, int32_t device, void *stream);
int mpchol_mlp_destroy(mpchol_mlp_t m);
/* host params in/out (nparam floats); set also zeroes the Adam moments */
int mpchol_mlp_set_params(mpchol_mlp_t m, const float *params, int64_t nparam);
int mpchol_mlp_get_params(mpchol_mlp_t m, float *params, int64_t nparam);
/* The whole training state, for checkpoints that resume bit for bit: host
 * params, Adam's first and second moments m1, m2 (nparam floats each, caller
 * owned) and the number of Adam steps taken (the bias corrections use it).
 * set_state: EINVAL for null pointers, nparam != MPCHOL_MLP_NPARAM, step < 0
 * or a second moment that is negative or NaN.  Both synchronize. */
int mpchol_mlp_get_state(mpchol_mlp_t m, float *params, float *m1, float *m2, int32_t *step, int64_t nparam);
int mpchol_mlp_set_state(mpchol_mlp_t m, const float *params, const float *m1, const float *m2, int32_t step,
                         int64_t nparam);
/* loss and gradient (device grad, nparam floats) of the batch: device X
 * (nb x 8 row-major), device y (nb int32 labels), host class weights cw[4];
 * per-sample loss w_y (-log p_y) + alpha sum_{c>y} p_c, mean over the batch. */
int mpchol_mlp_grad(mpchol_mlp_t m, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                    float *grad, float *loss);
/* one Adam step (Kingma & Ba) on the batch; *loss (optional) = the batch loss before the step */
int mpchol_mlp_train_step(mpchol_mlp_t m, const float *X, const int32_t *y, int64_t nb, const float *cw, float alpha,
                          float lr, float *loss);
/* logits (device nb x 4 row-major) and/or argmax classes (device nb int32) */
int mpchol_mlp_predict(mpchol_mlp_t m, const float *X, int64_t nb, float *logits, int32_t *cls);

/* ------------------------------------------------------------------ SHT
 * Spherical harmonic transform of real fields and its inverse, batched over
 * time steps, in FP64: the forward transform of Sec. III.A.1 ("Modeling in
 * the Spherical Harmonic Domain": G_m by FFT along longitude, K_{m,m'} by FFT
 * along the colatitude extended to (pi, 2 pi) with G_m(2 pi - theta) =
 * (-1)^m G_m(theta), then the sums with S_{l,m,m''} and I(q), the Wigner-d
 * functions at pi/2 precomputed as in Sec. III.A.2), and the inverse used to
 * turn emulated coefficient vectors into fields (Sec. III.B).
 *   Grid: N_theta colatitudes theta_j = j pi / (N_theta - 1) (both poles) and
 *   N_phi longitudes phi_k = 2 pi k / N_phi.  A field is N_theta x N_phi
 *   doubles, longitude fastest; T fields are contiguous (T x N_theta x N_phi).
 *   Coefficients: z_{l,m} = integral of Z conj(Y_lm) over the sphere, Y_lm
 *   orthonormal with the Condon-Shortley phase, 0 <= l < L.  Each time step
 *   has the real vector f_t of length L^2 (T vectors contiguous, T x L^2):
 *   index l^2 + l holds z_{l,0}; for 0 < m <= l, index l^2 + l + m holds
 *   sqrt(2) Re z_{l,m} and index l^2 + l - m holds sqrt(2) Im z_{l,m} (a real
 *   field has z_{l,-m} = (-1)^m conj z_{l,m}; |f_t| = the L2 norm of the
 *   band-limited part of the field).
 *   The inverse evaluates Z = sum_{l<L} sum_m z_{l,m} Y_lm on the grid (the
 *   longitude synthesis carries the 1/(2 pi) of the inverse Fourier series).
 *   Poles: the extension's symmetry forces G_m = 0 at theta = 0 and pi for
 *   odd m, and those samples are taken as zero (a field single-valued at the
 *   poles, constant along the first and last rows, has them).
 *   For fields band-limited at L the forward transform returns their
 *   coefficients and the inverse reproduces them, up to FP64 rounding
 *   (N_theta > L and N_phi >= 2L - 1 make the paper's FFT steps exact); other
 *   fields go through the same linear map (their higher degrees alias). */
typedef struct mpchol_sht *mpchol_sht_t;

/* Create a transform object on `device`, ordered on `stream` (NULL: the
 * default stream): computes d^l_{k,m}(pi/2) (recursion in the first index)
 * and from it, once, the composition of every step after the longitude FFT
 * (colatitude DFT of the extended G_m and both sums) as one table per order
 * for each direction (about L^2 N_theta / 4 doubles each), and work
 * buffers for up to tmax time steps per call.  Requires 1 <= L <= 1024,
 * N_theta > L, N_phi >= 2L - 1, N_phi a product of 2, 3 and 5 of at most 4096,
 * 1 <= tmax <= 2^20.  Errors: MPCHOL_EINVAL (sizes, with a
 * message from mpchol_sht_last_error), MPCHOL_ENOMEM, MPCHOL_EHIP.
 * Synchronizes the stream once. */
int mpchol_sht_create(mpchol_sht_t *s, int32_t L, int32_t ntheta, int32_t nphi, int32_t tmax, int32_t device,
                      void *stream);
int mpchol_sht_destroy(mpchol_sht_t s);

/* Forward transform: device Z (T x N_theta x N_phi) -> device f (T x L^2),
 * 0 <= T <= tmax (T = 0 does nothing).  Only enqueues.  The object's work
 * buffers are shared by its calls: calls on one object must not overlap. */
int mpchol_sht_forward(mpchol_sht_t s, const double *Z, int64_t T, double *f);

/* Inverse transform: device f (T x L^2) -> device Z (T x N_theta x N_phi).
 * Same rules as the forward call. */
int mpchol_sht_inverse(mpchol_sht_t s, const double *f, int64_t T, double *Z);

/* Device bytes of the tables and of the work buffers, and the FP64 GEMM flops
 * per time step of one transform (unpadded; each argument may be NULL). */
int mpchol_sht_info(mpchol_sht_t s, int64_t *table_bytes, int64_t *work_bytes, int64_t *gemm_flops_per_step);

/* Message of the last failed mpchol_sht_create on this thread. */
const char *mpchol_sht_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
