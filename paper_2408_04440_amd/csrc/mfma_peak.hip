// MFMA throughput on the device: for each matrix-instruction form used by
// (or considered for) the tile updates, every wave of a grid that fills all
// compute units issues long chains of that instruction on register operands,
// and the rate is taken from HIP events.  The result is the attainable dense
// peak per precision that the rooflines compare against, next to the
// datasheet figure.  Register-only: the one memory access per thread is the
// final store of a checksum to `out` (one float per thread, sized by the
// host from the launch shape).
//
// Build: compiled by paper_2408_04440_amd/build.py into
// paper_2408_04440_amd/mfma_peak.  Run: ./paper_2408_04440_amd/mfma_peak
// [milliseconds per form, default 200].
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                                         \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) {                                                                       \
            fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_));        \
            exit(1);                                                                                  \
        }                                                                                             \
    } while (0)

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;  // independent accumulators per wave
constexpr int NTH = 256;   // threads per block (4 waves)

// One instruction form: operand and accumulator types, flops per
// instruction (2*M*N*K per wave), and the instruction itself.
struct F64_16x16x4 {
    typedef double op_t;
    typedef f64x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 4;
    __device__ static op_t op(int t) { return 1.0 + 1e-3 * (t & 7); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
struct F32_16x16x4 {
    typedef float op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 4;
    __device__ static op_t op(int t) { return 1.0f + 1e-3f * (t & 7); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
struct F32_32x32x2 {
    typedef float op_t;
    typedef f32x16 acc_t;
    static constexpr double FLOPS = 2.0 * 32 * 32 * 2;
    __device__ static op_t op(int t) { return 1.0f + 1e-3f * (t & 7); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};
struct F16_16x16x32 {
    typedef f16x8 op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 32;
    __device__ static op_t op(int t)
    {
        op_t v;
        for (int i = 0; i < 8; ++i) v[i] = (_Float16)(1.0f + 0.125f * ((t + i) & 3));
        return v;
    }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
struct F16_32x32x16 {
    typedef f16x8 op_t;
    typedef f32x16 acc_t;
    static constexpr double FLOPS = 2.0 * 32 * 32 * 16;
    __device__ static op_t op(int t) { return F16_16x16x32::op(t); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};
struct BF16_16x16x32 {
    typedef bf16x8 op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 32;
    __device__ static op_t op(int t)
    {
        op_t v;
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)(1.0f + 0.125f * ((t + i) & 3));
        return v;
    }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
// E4M3 codes 0x38..0x3B (1.0 to 1.375): finite, so no special values flow
// through the accumulators.
struct FP8_16x16x32 {
    typedef long op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 32;
    __device__ static op_t op(int t) { return (long)(0x3838383838383838ull + (unsigned long long)(t & 3)); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
};
struct FP8_16x16x128 {
    typedef i32x8 op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 128;
    __device__ static op_t op(int t)
    {
        op_t v;
        for (int i = 0; i < 8; ++i) v[i] = 0x38383838 + ((t + i) & 3);
        return v;
    }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
};
// The same instruction with E8M0 scale operands (byte 127 = 2^0 per lane,
// not a constant zero, which the compiler turns into the unscaled form).
struct FP8_16x16x128_MX {
    typedef i32x8 op_t;
    typedef f32x4 acc_t;
    static constexpr double FLOPS = 2.0 * 16 * 16 * 128;
    __device__ static op_t op(int t) { return FP8_16x16x128::op(t); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c)
    {
        const int s = 127 + (int)(threadIdx.x >> 10);
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, s, 0, s);
    }
};
struct FP8_32x32x64 {
    typedef i32x8 op_t;
    typedef f32x16 acc_t;
    static constexpr double FLOPS = 2.0 * 32 * 32 * 64;
    __device__ static op_t op(int t) { return FP8_16x16x128::op(t); }
    __device__ static acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
};

template <typename Op>
__global__ __launch_bounds__(NTH) void peak_kernel(int iters, float *out)
{
    const int t = threadIdx.x;
    const typename Op::op_t a = Op::op(t), b = Op::op(t + 1);
    typename Op::acc_t acc[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = (typename Op::acc_t)(1e-3f * (c + 1 + (t & 1)));  // distinct chains
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = Op::mma(a, b, acc[c]);
    }
    // Every component of every accumulator feeds the checksum, so that each
    // accumulator stays whole in its registers across the loop.
    constexpr int NV = sizeof(typename Op::acc_t) / sizeof(acc[0][0]);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) s += (float)acc[c][v];
    out[(size_t)blockIdx.x * NTH + t] = s;
}

template <typename Op>
static void run(const char *name, double datasheet_tflops, int cus, float *out, int blocks, double target_ms)
{
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    int iters = 256;
    float ms = 0.f;
    peak_kernel<Op><<<blocks, NTH>>>(iters, out);  // warm-up
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    // Grow the chain length until one launch takes at least target_ms / 4.
    for (;;) {
        CK(hipEventRecord(e0));
        peak_kernel<Op><<<blocks, NTH>>>(iters, out);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (ms >= target_ms / 4 || iters >= (1 << 24)) break;
        iters *= 2;
    }
    const int reps = 4;
    CK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) peak_kernel<Op><<<blocks, NTH>>>(iters, out);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double waves = (double)blocks * (NTH / 64);
    const double flops = waves * iters * CHAINS * Op::FLOPS * reps;
    const double tf = flops / (ms * 1e-3) / 1e12;
    printf("%-34s %10.1f TFLOP/s  datasheet %7.1f  ratio %.3f  (%d CUs, %d blocks x %d threads, %d x %d chains)\n", name,
           tf, datasheet_tflops, tf / datasheet_tflops, cus, blocks, NTH, iters, CHAINS);
    fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
}

int main(int argc, char **argv)
{
    const double target_ms = argc > 1 ? atof(argv[1]) : 200.0;
    hipDeviceProp_t p;
    CK(hipGetDeviceProperties(&p, 0));
    const int cus = p.multiProcessorCount;
    const int blocks = cus * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
    float *out = nullptr;
    CK(hipMalloc(&out, sizeof(float) * (size_t)blocks * NTH));
    printf("device %s, %d CUs, %d MHz\n", p.gcnArchName, cus, p.clockRate / 1000);
    run<F64_16x16x4>("f64 16x16x4", 78.6, cus, out, blocks, target_ms);
    run<F32_16x16x4>("f32 16x16x4", 157.3, cus, out, blocks, target_ms);
    run<F32_32x32x2>("f32 32x32x2", 157.3, cus, out, blocks, target_ms);
    run<F16_16x16x32>("f16 16x16x32", 2500.0, cus, out, blocks, target_ms);
    run<F16_32x32x16>("f16 32x32x16", 2500.0, cus, out, blocks, target_ms);
    run<BF16_16x16x32>("bf16 16x16x32", 2500.0, cus, out, blocks, target_ms);
    run<FP8_16x16x32>("fp8 16x16x32 (fp8_fp8)", 5000.0, cus, out, blocks, target_ms);
    run<FP8_16x16x128>("fp8 16x16x128 (f8f6f4)", 5000.0, cus, out, blocks, target_ms);
    run<FP8_16x16x128_MX>("fp8 16x16x128 (f8f6f4, E8M0 scales)", 5000.0, cus, out, blocks, target_ms);
    run<FP8_32x32x64>("fp8 32x32x64 (f8f6f4)", 5000.0, cus, out, blocks, target_ms);
    CK(hipFree(out));
    return 0;
}
