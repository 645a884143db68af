// Device-side helpers shared by the mpchol kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

enum { P64 = 0, P32 = 1, P16 = 2, P8 = 3 };
enum { LO16_F16 = 0, LO16_BF16 = 1 };

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// index of lower tile (I, J), I >= J, in the packed tile array
__host__ __device__ inline int64_t tile_index(int I, int J) { return (int64_t)I * (I + 1) / 2 + J; }

// ---------------------------------------------------------------- formats
// FP32 -> FP16 bits, round to nearest even (the IEEE conversion).
__device__ inline uint16_t f32_to_f16(float v)
{
    _Float16 h = (_Float16)v;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_to_f32(uint16_t u) { return (float)__builtin_bit_cast(_Float16, u); }

// FP32 -> BF16 bits, round to nearest even on the dropped 16 bits (finite inputs).
__device__ inline uint16_t f32_to_bf16(float v)
{
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// FP32 -> OCP E4M3FN code: round to nearest even, gradual underflow below 2^-6,
// saturation at +-448 (the format has no infinity).  Finite inputs.
__device__ inline uint8_t f32_to_e4m3(float v)
{
    uint32_t sign = (__float_as_uint(v) >> 31) << 7;
    float a = fabsf(v);
    if (a >= 448.0f) return (uint8_t)(sign | 0x7E);
    int e = (int)((__float_as_uint(a) >> 23) & 0xFF) - 127;  // floor(log2 a) for normal a
    uint32_t code;
    if (e < -6) {
        // subnormal spacing 2^-9; 8 units = 2^-6 is the smallest normal (code 8)
        float q = __builtin_rintf(ldexpf(a, 9));
        code = (uint32_t)q;
    } else {
        float q = __builtin_rintf(ldexpf(a, 3 - e));  // in [8, 16]
        uint32_t k = (uint32_t)q;
        if (k == 16) { k = 8; e += 1; }
        code = ((uint32_t)(e + 7) << 3) | (k - 8);
        if (code > 0x7E) code = 0x7E;
    }
    return (uint8_t)(sign | code);
}
__device__ inline float e4m3_to_f32(uint8_t c)
{
    int e = (c >> 3) & 15, m = c & 7;
    float v = (e == 0) ? ldexpf((float)m, -9) : ldexpf((float)(8 + m), e - 10);
    return (c & 0x80) ? -v : v;
}

// Largest integer t with amax * 2^t <= the format's largest finite value for
// the scaled formats (FP16: 65504, E4M3: 448); 0 for FP64, FP32 and BF16
// (BF16 has FP32's exponent range), for amax == 0 and for a maximum that is
// not finite (no t exists; the codes then saturate or carry the NaN).
__host__ __device__ inline bool class_scaled(int q, int lo16) { return q == P8 || (q == P16 && lo16 == LO16_F16); }
__host__ __device__ inline int scale_exp(double amax, int q, int lo16)
{
    if (!class_scaled(q, lo16) || !(amax > 0.0) || !(amax <= 1.7976931348623157e308)) return 0;
    double maxf = (q == P8) ? 448.0 : 65504.0;
    int ea, em;
    frexp(amax, &ea);
    frexp(maxf, &em);
    int t = em - ea;
    while (ldexp(amax, t) > maxf) --t;
    while (ldexp(amax, t + 1) <= maxf) ++t;
    return t;
}

// Round a stored value to class q's copy: FP32 = (float)v; 16-bit / FP8 =
// round_q(round_f32(v * 2^t)).  Returns the bit pattern in the low bits.
__device__ inline uint32_t encode_class(double v, int q, int lo16, int t)
{
    if (q == P32) return __float_as_uint((float)v);
    float s = (float)ldexp(v, t);
    if (q == P16) return lo16 == LO16_BF16 ? f32_to_bf16(s) : f32_to_f16(s);
    return f32_to_e4m3(s);
}

// Represented value of a stored code of class q with scale t.
__device__ inline double decode_class(uint32_t bits, int q, int lo16, int t)
{
    if (q == P32) return (double)__uint_as_float(bits);
    float f;
    if (q == P16) f = lo16 == LO16_BF16 ? bf16_to_f32((uint16_t)bits) : f16_to_f32((uint16_t)bits);
    else f = e4m3_to_f32((uint8_t)bits);
    return ldexp((double)f, -t);
}

// Element (r, c) of a stored tile (column-major, leading dimension b) widened to FP64.
__device__ inline double load_stored(const void *tile, int cls, int lo16, int t, int64_t off)
{
    switch (cls) {
    case P64: return ((const double *)tile)[off];
    case P32: return (double)((const float *)tile)[off];
    case P16: return decode_class(((const uint16_t *)tile)[off], P16, lo16, t);
    default: return decode_class(((const uint8_t *)tile)[off], P8, lo16, t);
    }
}

// Inverse of tile_index: the lower tile (I, J) with I(I+1)/2 + J = t.
__device__ inline void tile_ij(int64_t t, int &I, int &J)
{
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
    while ((int64_t)i * (i + 1) / 2 > t) --i;
    I = i;
    J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// XCD-aware block order: the hardware deals workgroups round-robin over the 8
// XCDs; renumber so that consecutive logical blocks (which share operand rows)
// run on the same XCD and its L2.
__device__ inline int64_t xcd_remap(int64_t wg, int64_t G)
{
    const int64_t X = 8;
    int64_t q = G / X, r = G % X;
    int64_t xcd = wg % X, idx = wg / X;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

}  // namespace mpc
