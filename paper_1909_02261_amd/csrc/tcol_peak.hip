// MFMA throughput measurement: back-to-back matrix instructions on register operands,
// no memory traffic, over every CU, in the instruction forms the contraction uses
// (16x16x128 f8f6f4 with fp4 or fp8 operands, 16x16x32 bf16, 16x16x4 fp32).  It gives
// the achievable peak of this part for each operand type, the denominator beside the
// published one when the contraction's fraction of peak is reported.
#include <hip/hip_runtime.h>

#include "tcol.h"
#include "tcol_internal.h"

namespace tcol {

// keeps the results live (external, so the compiler cannot drop the store): written
// only when a sum equals a value no run produces
__device__ float peak_sink[1];

typedef float pk_f32x4 __attribute__((ext_vector_type(4)));
typedef int pk_i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 pk_bf16x8 __attribute__((ext_vector_type(8)));

static constexpr int kChains = 8;   // independent accumulators per wave
static constexpr int kPeakThreads = 256;   // four waves per block

// (the occupancy attribute keeps each chain's accumulator in place: without it the
// allocator rotated the accumulators through other registers every round)
template <int PREC>
__global__ __launch_bounds__(kPeakThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_mfma_peak(int iters) {
    const int lane = threadIdx.x & 63;
    pk_f32x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = pk_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // operands: small finite values that differ per lane
    pk_i32x8 ai, bi;
    pk_bf16x8 ab, bb;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        ai[e] = 0x22222222 ^ (lane << e);
        bi[e] = 0x24242424 ^ (lane << (7 - e));
        ab[e] = (__bf16)(0.25f * (float)((lane + e) & 7));
        bb[e] = (__bf16)(0.125f * (float)((lane * 3 + e) & 7));
    }
    const float af = 0.5f + 0.001f * lane, bf = 0.25f - 0.001f * lane;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (PREC == kPrecFP4)
                acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(ai, bi, acc[c], 4, 4, 0, 0, 0, 0);
            else if constexpr (PREC == kPrecFP8)
                acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(ai, bi, acc[c], 0, 0, 0, 0, 0, 0);
            else if constexpr (PREC == kPrecBF16)
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, acc[c], 0, 0, 0);
            else
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, acc[c], 0, 0, 0);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == -1.25e-30f) peak_sink[0] = s;
}

static double flops_per_mfma(int prec) {
    if (prec == kPrecFP4 || prec == kPrecFP8) return 2.0 * 16 * 16 * 128;
    if (prec == kPrecBF16) return 2.0 * 16 * 16 * 32;
    return 2.0 * 16 * 16 * 4;
}

}  // namespace tcol

using namespace tcol;

extern "C" tcol_status tcol_mfma_peak(int32_t precision, int32_t iters, double* tflops) {
    if (!tflops || iters < 1 || precision < kPrecFP32 || precision > kPrecFP4) return TCOL_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TCOL_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return TCOL_EHIP;
    const int blocks = cus * 8;     // 32 waves per CU
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tcol_status st = TCOL_EHIP;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        auto launch = [&](int n) {
            switch (precision) {
                case kPrecFP4: hipLaunchKernelGGL(k_mfma_peak<kPrecFP4>, dim3(blocks), dim3(kPeakThreads), 0, s, n); break;
                case kPrecFP8: hipLaunchKernelGGL(k_mfma_peak<kPrecFP8>, dim3(blocks), dim3(kPeakThreads), 0, s, n); break;
                case kPrecBF16: hipLaunchKernelGGL(k_mfma_peak<kPrecBF16>, dim3(blocks), dim3(kPeakThreads), 0, s, n); break;
                default: hipLaunchKernelGGL(k_mfma_peak<kPrecFP32>, dim3(blocks), dim3(kPeakThreads), 0, s, n); break;
            }
        };
        launch(iters < 64 ? iters : 64);    // warm-up
        float ms = 0.0f;
        if (hipGetLastError() == hipSuccess && hipEventRecord(e0, s) == hipSuccess) {
            launch(iters);
            if (hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
                hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
                const double flops = (double)blocks * (kPeakThreads / 64) * (double)iters * kChains * flops_per_mfma(precision);
                *tflops = flops / (ms * 1e-3) / 1e12;
                st = TCOL_OK;
            }
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    return st;
}
