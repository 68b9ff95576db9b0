// fr_device.h -- CDNA4 (gfx950) device helpers: hardware transcendentals and
// wave64 cross-lane sums built from DPP row permutes and ds_bpermute.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr {

// v_exp_f32 / v_log_f32 / v_rcp_f32: base-2 exponential and logarithm and the
// reciprocal, each about 1 ulp.
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Padded columns carry this exponent: 2^(kNeg - M) underflows to exactly 0.
constexpr float kNeg = -1.0e30f;

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// DPP controls (GFX9 encoding).
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// Sum of v over lanes l and l ^ 16 (ds_bpermute through the LDS crossbar).
__device__ __forceinline__ float sum_xor16(float v) {
    const int src = ((int)__lane_id() ^ 16) << 2;
    return v + __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src, __builtin_bit_cast(int, v)));
}

// Sum of v over lanes l and l ^ 32.
__device__ __forceinline__ float sum_xor32(float v) {
    const int src = ((int)__lane_id() ^ 32) << 2;
    return v + __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src, __builtin_bit_cast(int, v)));
}

// In-place all-reduce (sum) of MP values over aligned groups of L lanes
// (L a power of two, 1..64, uniform).  Every lane of a group ends with the
// same sums: each step adds a lane's value to its partner's in an order that
// is symmetric in the two operands.
template <int MP>
__device__ __forceinline__ void group_allreduce(float (&v)[MP], int L) {
    if (L > 1) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kQuadXor1>(v[k]);
    }
    if (L > 2) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kQuadXor2>(v[k]);
    }
    if (L > 4) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kRowHalfMirror>(v[k]);
    }
    if (L > 8) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kRowMirror>(v[k]);
    }
    if (L > 16) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] = sum_xor16(v[k]);
    }
    if (L > 32) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] = sum_xor32(v[k]);
    }
}

// Value of lane `k` (compile-time) of v, as a wave-uniform scalar.
template <int K>
__device__ __forceinline__ float lane_value(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), K));
}

// Picks v[lane] for lane < MP (0 elsewhere): turns a uniform array into one
// value per lane.
template <int MP>
__device__ __forceinline__ float pick_lane(const float (&v)[MP], int lane) {
    float out = 0.f;
#pragma unroll
    for (int k = 0; k < MP; ++k) out = (lane == k) ? v[k] : out;
    return out;
}

// Inverse of pick_lane: broadcasts lane k's value into v[k] for every lane.
template <int MP, int K = 0>
__device__ __forceinline__ void spread_lanes(float x, float (&v)[MP]) {
    if constexpr (K < MP) {
        v[K] = lane_value<K>(x);
        spread_lanes<MP, K + 1>(x, v);
    }
}

// float -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t b = __builtin_bit_cast(uint32_t, x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

}  // namespace fr
