// fr_diag.hip -- microbenchmarks that measure the MI355X ceilings the fused
// kernels are compared with: the v_exp_f32 rate, the FP32 FMA rate, their
// mix in the proportion of one Sinkhorn cell-iteration, and a plain HBM
// copy (also used to calibrate the profiler's byte counters).
#include <hip/hip_runtime.h>

#include "../../include/fairrank_diag.h"
#include "fr_device.h"

namespace fr {
namespace {

constexpr int kChains = 8;   // independent dependency chains per lane

// kind 0: exp only; 1: FMA only; 2: one exp + five FMA per step.
template <int KIND>
__global__ __launch_bounds__(256) void k_alu(float* out, int iters, float seed) {
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = seed * (float)(threadIdx.x + c) * 1e-6f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (KIND == 0) {
                v[c] = ex2(-v[c]);
            } else if constexpr (KIND == 1) {
                v[c] = fmaf(v[c], 0.999f, 1e-7f);
            } else {
                float z = ex2(-v[c]);
                z = fmaf(z, 0.999f, 1e-7f);
                z = fmaf(z, 0.999f, 1e-7f);
                z = fmaf(z, 0.999f, 1e-7f);
                z = fmaf(z, 0.999f, 1e-7f);
                v[c] = fmaf(z, 0.999f, 1e-7f);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    if (s == 12345.678f) out[threadIdx.x] = s;   // keeps the loop live
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              int64_t n4) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace fr

using namespace fr;

extern "C" fr_status fr_diag_alu(int kind, int blocks, int iters, double* ms_out, double* ops_out) {
    if (!ms_out || !ops_out) return FR_E_NULL;
    if (kind < 0 || kind > 2 || blocks < 1 || iters < 1) return FR_E_PARAM;
    float* out = nullptr;
    if (hipMalloc(&out, 256 * sizeof(float)) != hipSuccess) return FR_E_DEVICE;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    auto launch = [&]() {
        if (kind == 0)
            hipLaunchKernelGGL(k_alu<0>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f);
        else if (kind == 1)
            hipLaunchKernelGGL(k_alu<1>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f);
        else
            hipLaunchKernelGGL(k_alu<2>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f);
    };
    launch();  // warm-up
    hipEventRecord(a, 0);
    launch();
    hipEventRecord(b, 0);
    hipEventSynchronize(b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(out);
    if (hipGetLastError() != hipSuccess) return FR_E_DEVICE;
    // lane-operations: kind 0 counts exps, kind 1 FMAs, kind 2 cell-steps
    *ms_out = ms;
    *ops_out = (double)blocks * 256.0 * iters * kChains;
    return FR_OK;
}

extern "C" fr_status fr_diag_copy(const void* src, void* dst, size_t bytes, int reps, double* ms_out,
                                  void* stream) {
    if (!src || !dst || !ms_out) return FR_E_NULL;
    if (bytes % 16 != 0 || reps < 1) return FR_E_PARAM;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n4 = (int64_t)(bytes / 16);
    const int blocks = 256 * 8;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n4);
    hipEventRecord(a, s);
    for (int q = 0; q < reps; ++q)
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst,
                           n4);
    hipEventRecord(b, s);
    hipEventSynchronize(b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return FR_E_DEVICE;
    *ms_out = ms / reps;
    return FR_OK;
}
