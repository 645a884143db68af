// FP64-class tile updates from exact integer products on the INT8 MFMA (the
// Ozaki scheme II of Ozaki, Uchino and Imamura): the sender converts each
// FP64 panel tile to row-scaled integers and their residues modulo 15
// coprime moduli (one INT8 plane per modulus); an update forms the INT8
// product of every plane pair, reduces it modulo its modulus, recovers the
// exact integer product by the Chinese remainder theorem, rounds it once to
// FP64 and subtracts it, scaled back, from the FP64 work tile.  The
// arithmetic per element is defined in ozaki_crt.h.
#include "common.h"
#include "gemm_core.h"
#include "launch.h"
#include "ozaki_crt.h"

namespace mpc {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

void ozaki_const_init(OzakiConst *k)
{
    static const uint32_t P[OZ_NMOD] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197};
    typedef unsigned __int128 u128;
    u128 M = 1;
    for (int l = 0; l < OZ_NMOD; ++l) M *= P[l];
    for (int l = 0; l < OZ_NMOD; ++l) {
        const uint32_t p = P[l];
        k->p[l] = p;
        k->pinv[l] = 1.0f / (float)p;
        k->pinvd[l] = 1.0 / (double)p;
        const u128 Ml = M / p;
        const uint32_t y = (uint32_t)(Ml % p);
        uint32_t inv = 0;
        for (uint32_t t = 1; t < p; ++t)
            if ((uint64_t)y * t % p == 1) {
                inv = t;
                break;
            }
        const u128 W = (Ml * inv) % M;  // Ml * inv < M * 256 < 2^128
        for (int i = 0; i < 4; ++i) k->W[l][i] = (uint32_t)(W >> (32 * i));
        for (int i = 0; i < 3; ++i) k->Wd[l][i] = (double)(uint64_t)((W >> (40 * i)) & ((((u128)1) << 40) - 1));
    }
    for (int i = 0; i < 3; ++i) k->Md[i] = (double)(uint64_t)((M >> (40 * i)) & ((((u128)1) << 40) - 1));
    const u128 H = M / 2 + (M & 1);
    for (int i = 0; i < 4; ++i) {
        k->M[i] = (uint32_t)(M >> (32 * i));
        k->H[i] = (uint32_t)(H >> (32 * i));
    }
    k->Minv = 1.0 / ((double)(uint64_t)(M >> 64) * 18446744073709551616.0 + (double)(uint64_t)M);
}

// ---------------------------------------------------------------- sender side
// Row exponents of the FP64 copies of step k's panel tiles that FP64-class
// updates formed from INT8 products consume (qmask bit 4): e_r = 53 - E_r
// with max_c |X_rc| = f 2^E_r, f in [1/2, 1) (0 for a zero row).  One thread
// per row; the column-major copy is read row by row, coalesced over rows.
__global__ __launch_bounds__(256) void ozaki_rowexp_kernel(Tiles T, Panel P, int k, const uint8_t *qmask)
{
    const int I = k + 1 + blockIdx.y, b = T.b;
    if (!(qmask[I] & 16)) return;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= b) return;
    const int64_t bb = (int64_t)b * b;
    const double *x = P.p64 + (int64_t)I * bb + r;
    double mu = 0.0;
    for (int c = 0; c < b; ++c) mu = fmax(mu, fabs(x[(int64_t)c * b]));
    int e = 0;
    if (mu > 0.0) {
        int E;
        frexp(mu, &E);
        e = 53 - E;
    }
    P.pexp[(int64_t)I * b + r] = e;
}

// Residue planes of the same tiles: the integer a = rint(X_rc 2^e_r) (|a| <=
// 2^53, exact in FP64) and, for each modulus p_l, its signed residue as a
// byte in plane l, row-major (K contiguous) for the INT8 MFMA operands.  One
// 64 x 64 sub-tile per block, transposed through LDS; each thread writes 16
// consecutive bytes of one row per plane.
__global__ __launch_bounds__(256) void ozaki_convert_kernel(Tiles T, Panel P, int k, const uint8_t *qmask,
                                                            const OzakiConst *__restrict__ K)
{
    __shared__ double xs[64][65];  // xs[c][r]
    const int I = k + 1 + blockIdx.y, b = T.b, nsub = b / 64;
    if (!(qmask[I] & 16)) return;
    const int sr = blockIdx.x % nsub, sc = blockIdx.x / nsub;
    const int64_t bb = (int64_t)b * b;
    const double *x64 = P.p64 + (int64_t)I * bb;
    for (int e = threadIdx.x; e < 4096; e += 256) {
        const int r = e & 63, c = e >> 6;
        xs[c][r] = x64[(int64_t)(sr * 64 + r) + (int64_t)(sc * 64 + c) * b];
    }
    __syncthreads();
    const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    const int er = P.pexp[(int64_t)I * b + sr * 64 + r];
    double a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = rint(ldexp(xs[c0 + j][r], er));
    uint8_t *dst = (uint8_t *)P.poz + (int64_t)I * OZ_NMOD * bb + (int64_t)(sr * 64 + r) * b + sc * 64 + c0;
    for (int l = 0; l < OZ_NMOD; ++l) {
        const double p = (double)K->p[l], pinv = K->pinvd[l];
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) v |= (uint32_t)(uint8_t)mod_sym(a[4 * q + j], p, pinv) << (8 * j);
            w[q] = v;
        }
        *(u32x4 *)(dst + (int64_t)l * bb) = (u32x4){w[0], w[1], w[2], w[3]};
    }
}

void launch_ozaki_convert(const Tiles &T, const Panel &P, int k, const uint8_t *qmask, const OzakiConst *K,
                          hipStream_t st)
{
    const int np = T.nt - k - 1;
    if (np <= 0) return;
    const int nsub = T.b / 64;
    ozaki_rowexp_kernel<<<dim3((T.b + 255) / 256, np), 256, 0, st>>>(T, P, k, qmask);
    ozaki_convert_kernel<<<dim3(nsub * nsub, np), 256, 0, st>>>(T, P, k, qmask, K);
}

// ---------------------------------------------------------------- update
// A_IJ -= L_Ik L_Jk^T (and, for a pair of steps, then -= L_I,k+1 L_J,k+1^T)
// for FP64-class tiles, each product formed exactly: for every modulus p_l
// the INT8 product of the two residue planes (K = b, |sum| <= 2^24, exact in
// INT32) reduced mod p_l and folded into the residue sum S = sum_l r_l W_l,
// kept exactly in three FP64 parts; S mod M is then the exact integer
// product, rounded once to FP64, scaled by 2^-(e_r + e_s) and subtracted
// from the FP64 work tile.  The K slices of all moduli form one pipelined
// loop (the next slice is fetched while the current one multiplies, across
// modulus boundaries too).  128 x 64 output block (128 rows of I, 64 of J)
// per workgroup of 8 waves, 16 elements per thread; the MFMA operands are
// exchanged (J rows on the instruction's A side) so that each lane owns one
// output row and the column-major stores coalesce.
constexpr int OBM = 128, OBN = 64, OBK = 128, OWM = 2, OWN = 4;
constexpr int ONTH = 64 * OWM * OWN, OLDB = OBK + 16, OCPR = OBK / 16;
constexpr int OCHA = OBN * OCPR, OCHB = OBM * OCPR;  // 16-byte chunks per slice: J side, I side
constexpr int OCA = (OCHA + ONTH - 1) / ONTH, OCB = (OCHB + ONTH - 1) / ONTH;
constexpr int OMB = OBN / OWM / 16, ONB = OBM / OWN / 16;
constexpr size_t OSMEM = (size_t)2 * (OBN + OBM) * OLDB;
static_assert(OCHA % ONTH == 0 && OCHB % ONTH == 0, "load split");

__global__ __launch_bounds__(ONTH) void update_ozaki_kernel(Tiles Tt, const uint8_t *panel0, const int32_t *pexp0,
                                                            const uint8_t *panel1, const int32_t *pexp1,
                                                            const int32_t *items, const OzakiConst *__restrict__ K)
{
    extern __shared__ __align__(16) uint8_t osm[];
    uint8_t *As = osm;                    // [2][OBN][OLDB]  J rows
    uint8_t *Bs = osm + 2 * OBN * OLDB;   // [2][OBM][OLDB]  I rows
    const int b = Tt.b;
    const int tmn = b / OBM, tnn = b / OBN;
    const int64_t lg = xcd_remap(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (tmn * tnn));
    const int rem = (int)(lg % (tmn * tnn));
    const int tm = rem % tmn, tn = rem / tmn;
    const int32_t it = items[item];
    const int I = it >> 16, J = it & 0xFFFF;
    const int64_t bb = (int64_t)b * b;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % OWM, wn = wave / OWM, gi = lane & 15, gg = lane >> 4;
    double *C = (double *)(Tt.slots + tile_index(I, J) * Tt.slot_bytes);
    const int nk = b / OBK, nt_ = OZ_NMOD * nk;
    const int npan = panel1 ? 2 : 1;
#pragma nounroll
    for (int h = 0; h < npan; ++h) {
        const uint8_t *pn = h ? panel1 : panel0;
        const int32_t *pe = h ? pexp1 : pexp0;
        const uint8_t *Abase = pn + (int64_t)J * OZ_NMOD * bb + (int64_t)tn * OBN * b;  // plane 0, J rows
        const uint8_t *Bbase = pn + (int64_t)I * OZ_NMOD * bb + (int64_t)tm * OBM * b;  // plane 0, I rows
        double s[OMB][ONB][4][3];
#pragma unroll
        for (int m = 0; m < OMB; ++m)
#pragma unroll
            for (int n = 0; n < ONB; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) s[m][n][v][0] = s[m][n][v][1] = s[m][n][v][2] = 0.0;
        i32x4 acc[OMB][ONB];
#pragma unroll
        for (int m = 0; m < OMB; ++m)
#pragma unroll
            for (int n = 0; n < ONB; ++n) acc[m][n] = (i32x4){0, 0, 0, 0};
        u32x4 ra[OCA], rb[OCB];
        auto gload = [&](int t) {
            const int l = t / nk, kt = t - l * nk;
            const uint8_t *a = Abase + (int64_t)l * bb + kt * OBK, *bp = Bbase + (int64_t)l * bb + kt * OBK;
#pragma unroll
            for (int c = 0; c < OCA; ++c) {
                const int ch = tid + ONTH * c, row = ch / OCPR, cb = (ch % OCPR) * 16;
                ra[c] = *(const u32x4 *)(a + (int64_t)row * b + cb);
            }
#pragma unroll
            for (int c = 0; c < OCB; ++c) {
                const int ch = tid + ONTH * c, row = ch / OCPR, cb = (ch % OCPR) * 16;
                rb[c] = *(const u32x4 *)(bp + (int64_t)row * b + cb);
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int c = 0; c < OCA; ++c) {
                const int ch = tid + ONTH * c, row = ch / OCPR, cb = (ch % OCPR) * 16;
                *(u32x4 *)(As + (buf * OBN + row) * OLDB + cb) = ra[c];
            }
#pragma unroll
            for (int c = 0; c < OCB; ++c) {
                const int ch = tid + ONTH * c, row = ch / OCPR, cb = (ch % OCPR) * 16;
                *(u32x4 *)(Bs + (buf * OBM + row) * OLDB + cb) = rb[c];
            }
        };
        gload(0);
        sstore(0);
        __syncthreads();
        for (int t = 0; t < nt_; ++t) {
            const int cur = t & 1;
            if (t + 1 < nt_) gload(t + 1);
            const uint8_t *as = As + (cur * OBN + wm * (OBN / OWM) + gi) * OLDB;
            const uint8_t *bs = Bs + (cur * OBM + wn * (OBM / OWN) + gi) * OLDB;
#pragma unroll
            for (int ks = 0; ks < OBK / 64; ++ks) {
                const int kb = ks * 64 + 16 * gg;
                i32x4 fa[OMB], fb[ONB];
#pragma unroll
                for (int m = 0; m < OMB; ++m) fa[m] = *(const i32x4 *)(as + m * 16 * OLDB + kb);
#pragma unroll
                for (int n = 0; n < ONB; ++n) fb[n] = *(const i32x4 *)(bs + n * 16 * OLDB + kb);
#pragma unroll
                for (int m = 0; m < OMB; ++m)
#pragma unroll
                    for (int n = 0; n < ONB; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[m], fb[n], acc[m][n], 0, 0, 0);
            }
            if (t % nk == nk - 1) {  // the last slice of modulus l: fold its residues into S
                const int l = t / nk;
                const uint32_t p = K->p[l];
                const float pinv = K->pinv[l];
                const double w[3] = {K->Wd[l][0], K->Wd[l][1], K->Wd[l][2]};
#pragma unroll
                for (int m = 0; m < OMB; ++m)
#pragma unroll
                    for (int n = 0; n < ONB; ++n) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) crt_fma(s[m][n][v], mod_small(acc[m][n][v], p, pinv), w);
                        acc[m][n] = (i32x4){0, 0, 0, 0};
                    }
            }
            if (t + 1 < nt_) sstore(cur ^ 1);
            __syncthreads();
        }
        // acc[m][n][v] = D[4g + v][i] of the (J rows) x (I rows) product:
        // output row r (of I) = lane's i, output column c (of J) = 4g + v
#pragma unroll
        for (int m = 0; m < OMB; ++m)
#pragma unroll
            for (int n = 0; n < ONB; ++n) {
                const int r = tm * OBM + wn * (OBM / OWN) + n * 16 + gi;
                const int er = pe[(int64_t)I * b + r];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = tn * OBN + wm * (OBN / OWM) + m * 16 + 4 * gg + v;
                    const int ec = pe[(int64_t)J * b + c];
                    uint32_t S[4];
                    crt_parts_to_limbs(s[m][n][v], *K, S);
                    const double d = ldexp(crt_to_double(S, *K), -(er + ec));
                    C[r + (int64_t)c * b] -= d;
                }
            }
    }
}

void launch_ozaki_update(const Tiles &T, const Panel &P, const Panel *P2, const int32_t *items, int nitems,
                         const OzakiConst *K, hipStream_t st)
{
    if (nitems <= 0) return;
    auto k = update_ozaki_kernel;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)OSMEM);
        attr = true;
    }
    const int64_t grid = (int64_t)nitems * (T.b / OBM) * (T.b / OBN);
    k<<<(unsigned)grid, ONTH, OSMEM, st>>>(T, (const uint8_t *)P.poz, P.pexp,
                                                   P2 ? (const uint8_t *)P2->poz : nullptr, P2 ? P2->pexp : nullptr,
                                                   items, K);
}

}  // namespace mpc
