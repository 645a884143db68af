// Residue-number arithmetic of the FP64-class products formed from INT8
// products (the Ozaki scheme II of Ozaki, Uchino and Imamura): an integer
// product P = sum_c a_c b_c with |a|, |b| <= 2^53 and at most 1024 terms
// (|P| <= 2^116) is known from its residues r_l = P mod p_l for 15 pairwise
// coprime moduli p_l <= 256 (product M ~ 2^117.8 > 2 max|P|), and is
// recovered exactly by the Chinese remainder theorem,
//   P = (sum_l r_l W_l) mod M  (mapped to [-M/2, M/2)),
//   W_l = (M / p_l) ((M / p_l)^-1 mod p_l),
// then rounded once to FP64 (nearest, ties to even).  Two exact forms of the
// sum: four 32-bit limbs reduced mod M after every three terms (below 766 M
// < 2^128 in between), or three FP64 parts of at most 40 bits each, exact
// without reductions (crt_fma).  Plain integer and exact floating-point
// arithmetic, usable on the host and the device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

constexpr int OZ_NMOD = 15;      // moduli for tiles up to 1024 (|P| <= 2^116)
constexpr int OZ_MAX_TILE = 1024;

struct OzakiConst {
    double Wd[OZ_NMOD][3];      // W_l = Wd[l][2] 2^80 + Wd[l][1] 2^40 + Wd[l][0], parts < 2^40 (exact doubles)
    double Md[3];               // M in the same three parts
    uint32_t p[OZ_NMOD];        // moduli
    float pinv[OZ_NMOD];        // 1 / p_l (rounded), for quotient estimates of |x| <= 2^24
    double pinvd[OZ_NMOD];      // 1 / p_l (rounded), for quotient estimates of |x| <= 2^53
    uint32_t W[OZ_NMOD][4];     // W_l mod M, little-endian limbs
    uint32_t M[4];              // product of the moduli
    uint32_t H[4];              // ceil(M / 2): residues >= H stand for P - M < 0
    double Minv;                // 1 / M (rounded)
};

// Fill the table (host).  Moduli: 256 and the 14 largest odd values <= 255
// coprime to each other and to 2 (255 = 3 5 17, 253 = 11 23, 247 = 13 19,
// 217 = 7 31, the rest prime).
void ozaki_const_init(OzakiConst *k);

// S += r W (r < 256, W < M), four limbs; the caller keeps S + r W < 2^128.
__host__ __device__ inline void crt_madd(uint32_t (&S)[4], uint32_t r, const uint32_t (&W)[4])
{
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t t = (uint64_t)W[i] * r + S[i] + carry;
        S[i] = (uint32_t)t;
        carry = t >> 32;
    }
}

// a >= b on four limbs
__host__ __device__ inline bool crt_geq(const uint32_t (&a)[4], const uint32_t (&b)[4])
{
#pragma unroll
    for (int i = 3; i >= 0; --i)
        if (a[i] != b[i]) return a[i] > b[i];
    return true;
}

// a -= q b (q < 2^16), assuming the result is >= 0
__host__ __device__ inline void crt_msub(uint32_t (&a)[4], uint32_t q, const uint32_t (&b)[4])
{
    uint64_t carry = 0;   // of q b
    int64_t borrow = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t t = (uint64_t)b[i] * q + carry;
        carry = t >> 32;
        int64_t d = (int64_t)a[i] - (int64_t)(uint32_t)t - borrow;
        borrow = d < 0 ? 1 : 0;
        a[i] = (uint32_t)d;
    }
}

// S mod M for S < 2^128 that is below 2^11 M: subtract (q - 1) M with q an
// estimate of floor(S / M) from the top limbs (off by at most one), then at
// most two more M.
__host__ __device__ inline void crt_reduce(uint32_t (&S)[4], const OzakiConst &k)
{
    const double s = ((double)S[3] * 4294967296.0 + (double)S[2]) * 18446744073709551616.0 + (double)S[1] * 4294967296.0;
    int q = (int)(s * k.Minv) - 1;
    if (q > 0) crt_msub(S, (uint32_t)q, k.M);
    if (crt_geq(S, k.M)) crt_msub(S, 1u, k.M);
    if (crt_geq(S, k.M)) crt_msub(S, 1u, k.M);
}

// x mod p in [0, p) for an integer |x| <= 2^24 (the INT8 products of one
// modulus over at most 1024 terms: |x| <= 1024 * 128 * 128).
__host__ __device__ inline uint32_t mod_small(int32_t x, uint32_t p, float pinv)
{
    int32_t q = (int32_t)floorf((float)x * pinv);
    int32_t r = x - q * (int32_t)p;
    if (r < 0) r += (int32_t)p;
    if (r >= (int32_t)p) r -= (int32_t)p;
    return (uint32_t)r;
}

// Symmetric residue of an integer-valued double |a| <= 2^53 modulo p, as the
// signed byte the INT8 products take: a mod p in [-(p/2), (p-1)/2] (p = 256:
// [-128, 127]).  The fused multiply-add gives a - q p exactly (an integer
// below 2p in magnitude); q may be off by one, corrected after.
__host__ __device__ inline int8_t mod_sym(double a, double p, double pinv)
{
    double q = floor(a * pinv);
    double r = fma(-q, p, a);
    if (r < 0) r += p;
    if (r >= p) r -= p;
    if (r >= 0.5 * (p + 1.0)) r -= p;  // r >= ceil(p / 2)
    return (int8_t)(int)r;
}

// Residue sums in three FP64 parts: S = s[2] 2^80 + s[1] 2^40 + s[0] with
// s[i] += r W_l[i] -- every part an integer below 15 * 255 * 2^40 < 2^52, so
// each fused multiply-add is exact and no reduction is needed on the way.
__host__ __device__ inline void crt_fma(double (&s)[3], uint32_t r, const double (&w)[3])
{
    const double rd = (double)r;
    s[0] = fma(rd, w[0], s[0]);
    s[1] = fma(rd, w[1], s[1]);
    s[2] = fma(rd, w[2], s[2]);
}

// The four-limb value of S mod M for S from crt_fma (S < 15 * 256 * M):
// q = floor(S / M) - 1 or - 2 from the leading parts (q < 2^12, so q M_i <
// 2^52 and each s_i - q M_i is exact), the parts recombined in 128-bit
// integers, and at most two more M subtracted.
__host__ __device__ inline void crt_parts_to_limbs(const double (&s)[3], const OzakiConst &k, uint32_t (&S)[4])
{
    const double approx = s[2] * 1208925819614629174706176.0 + s[1] * 1099511627776.0;  // 2^80, 2^40
    int q = (int)(approx * k.Minv) - 1;
    if (q < 0) q = 0;
    const double qd = (double)q;
    const int64_t t2 = (int64_t)fma(-qd, k.Md[2], s[2]);
    const int64_t t1 = (int64_t)fma(-qd, k.Md[1], s[1]);
    const int64_t t0 = (int64_t)fma(-qd, k.Md[0], s[0]);
    typedef unsigned __int128 u128;
    u128 R = ((u128)(__int128)t2 << 80) + ((u128)(__int128)t1 << 40) + (u128)(__int128)t0;  // in [0, 3M)
    const u128 M = ((u128)k.M[3] << 96) | ((u128)k.M[2] << 64) | ((u128)k.M[1] << 32) | (u128)k.M[0];
    if (R >= M) R -= M;
    if (R >= M) R -= M;
    S[0] = (uint32_t)R;
    S[1] = (uint32_t)(R >> 32);
    S[2] = (uint32_t)(R >> 64);
    S[3] = (uint32_t)(R >> 96);
}

// The residues' integer as a double: S (already reduced, in [0, M)) read as
// S - M when S >= ceil(M/2), rounded to nearest with ties to even.
__host__ __device__ inline double crt_to_double(const uint32_t (&S)[4], const OzakiConst &k)
{
    uint32_t m[4] = {S[0], S[1], S[2], S[3]};
    bool neg = crt_geq(m, k.H);
    if (neg) {  // magnitude M - S
        int64_t borrow = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int64_t d = (int64_t)k.M[i] - (int64_t)m[i] - borrow;
            borrow = d < 0 ? 1 : 0;
            m[i] = (uint32_t)d;
        }
    }
    const uint64_t hi = ((uint64_t)m[3] << 32) | m[2], lo = ((uint64_t)m[1] << 32) | m[0];
    double v;
    if (hi == 0 && (lo >> 53) == 0) {
        v = (double)(uint32_t)(lo >> 32) * 4294967296.0 + (double)(uint32_t)lo;  // exact
    } else {
        const int top = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);  // index of the leading bit
        const int s = top - 52;                                                        // bits dropped, >= 1
        uint64_t mant, rest_hi, rest_lo;  // kept 53 bits; dropped bits as (rest_hi, rest_lo) below bit s
        if (s >= 64) {
            mant = hi >> (s - 64);
            rest_hi = (s - 64) ? (hi & ((1ull << (s - 64)) - 1)) : 0;
            rest_lo = lo;
        } else {
            mant = (hi << (64 - s)) | (lo >> s);
            rest_hi = 0;
            rest_lo = lo & ((1ull << s) - 1);
        }
        // round bit: bit s-1 of the value; sticky: any bit below it
        bool round, sticky;
        if (s - 1 >= 64) {
            const int b = s - 1 - 64;
            round = (rest_hi >> b) & 1ull;
            sticky = (rest_hi & ((1ull << b) - 1)) != 0 || rest_lo != 0;
        } else {
            const int b = s - 1;
            round = (rest_lo >> b) & 1ull;
            sticky = b ? (rest_lo & ((1ull << b) - 1)) != 0 : false;
        }
        if (round && (sticky || (mant & 1ull))) mant += 1;  // may reach 2^53, still exact below
        v = ldexp((double)(uint32_t)(mant >> 32) * 4294967296.0 + (double)(uint32_t)mant, s);
    }
    return neg ? -v : v;
}

}  // namespace mpc
