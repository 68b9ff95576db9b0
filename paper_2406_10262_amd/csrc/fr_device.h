// fr_device.h -- CDNA4 (gfx950) device helpers: hardware transcendentals and
// wave64 cross-lane sums built from DPP row permutes and the gfx950 row swaps.
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

// Value of a DPP-selected lane.  All patterns used here read lanes of the
// same row, so bound_ctrl never applies; setting it lets the compiler fold
// the move into the consuming add (v_add_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// DPP controls (GFX9 encoding).
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// Row-swap permutes on up to 8 registers per asm statement.
// v_permlane16_swap exchanges the odd 16-lane rows of its first operand with
// the even rows of its second; with both operands holding v, every lane of
// rows 2j and 2j+1 ends up with the values of rows 2j and 2j+1 in its two
// registers (v_permlane32_swap likewise exchanges the 32-lane halves).  The
// instructions are written as inline asm with read-write operands because
// the compiler's builtin folds the instruction's two results into one when
// both are used.  One s_nop on each side covers the VALU-to-permute hazards
// for the whole batch.
#define FR_SWAP_ASM(NAME, OP)                                                                \
    template <int N>                                                                         \
    __device__ __forceinline__ void NAME(unsigned* x, unsigned* y) {                         \
        if constexpr (N == 1) {                                                              \
            asm volatile("s_nop 1\n\t" OP " %0, %1\n\ts_nop 1" : "+v"(x[0]), "+v"(y[0]));    \
        } else if constexpr (N == 2) {                                                       \
            asm volatile("s_nop 1\n\t" OP " %0, %2\n\t" OP " %1, %3\n\ts_nop 1"              \
                         : "+v"(x[0]), "+v"(x[1]), "+v"(y[0]), "+v"(y[1]));                  \
        } else if constexpr (N == 4) {                                                       \
            asm volatile("s_nop 1\n\t" OP " %0, %4\n\t" OP " %1, %5\n\t" OP " %2, %6\n\t" OP  \
                         " %3, %7\n\ts_nop 1"                                                \
                         : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(y[0]),       \
                           "+v"(y[1]), "+v"(y[2]), "+v"(y[3]));                              \
        } else if constexpr (N == 8) {                                                       \
            asm volatile("s_nop 1\n\t" OP " %0, %8\n\t" OP " %1, %9\n\t" OP " %2, %10\n\t" OP \
                         " %3, %11\n\t" OP " %4, %12\n\t" OP " %5, %13\n\t" OP " %6, %14\n\t" \
                         OP " %7, %15\n\ts_nop 1"                                             \
                         : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]),       \
                           "+v"(x[5]), "+v"(x[6]), "+v"(x[7]), "+v"(y[0]), "+v"(y[1]),       \
                           "+v"(y[2]), "+v"(y[3]), "+v"(y[4]), "+v"(y[5]), "+v"(y[6]),       \
                           "+v"(y[7]));                                                      \
        } else {                                                                             \
            constexpr int H = (N > 4) ? 4 : 2;                                               \
            NAME<H>(x, y);                                                                   \
            NAME<N - H>(x + H, y + H);                                                       \
        }                                                                                    \
    }
FR_SWAP_ASM(swap16_batch, "v_permlane16_swap_b32")
FR_SWAP_ASM(swap32_batch, "v_permlane32_swap_b32")
#undef FR_SWAP_ASM

// v[k] <- v[k] (lane l) + v[k] (lane l ^ 16), for every k (or lane l ^ 32
// when XOR32).  Both operands of each sum are the same pair of values, so
// every lane of a pair gets the same rounded result.
template <int MP, bool XOR32, int K0 = 0>
__device__ __forceinline__ void sum_swap(float (&v)[MP]) {
    if constexpr (K0 < MP) {
        constexpr int N = (MP - K0) < 8 ? (MP - K0) : 8;
        unsigned x[N], y[N];
#pragma unroll
        for (int q = 0; q < N; ++q) x[q] = y[q] = __builtin_bit_cast(unsigned, v[K0 + q]);
        if constexpr (XOR32)
            swap32_batch<N>(x, y);
        else
            swap16_batch<N>(x, y);
#pragma unroll
        for (int q = 0; q < N; ++q)
            v[K0 + q] = __builtin_bit_cast(float, x[q]) + __builtin_bit_cast(float, y[q]);
        sum_swap<MP, XOR32, K0 + N>(v);
    }
}

// In-place all-reduce (sum) of MP values over aligned groups of L lanes
// (L a power of two, 1..64, uniform).  Every lane of a group ends with the
// same sums: each step adds a lane's value to its partner's in an order that
// is symmetric in the two operands.  Each step is issued for all MP columns
// before the next one starts (scheduling barriers), so independent columns
// fill the DPP data-hazard slots.
template <int MP>
__device__ __forceinline__ void group_allreduce(float (&v)[MP], int L) {
    __builtin_amdgcn_sched_barrier(0);
    if (L > 1) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kQuadXor1>(v[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (L > 2) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kQuadXor2>(v[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (L > 4) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kRowHalfMirror>(v[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (L > 8) {
#pragma unroll
        for (int k = 0; k < MP; ++k) v[k] += dpp_mov<kRowMirror>(v[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (L > 16) {
        sum_swap<MP, false>(v);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (L > 32) {
        sum_swap<MP, true>(v);
        __builtin_amdgcn_sched_barrier(0);
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

// Pairwise (tree) sum and max of N register values: dependency depth log2 N.
template <int N>
struct Tree {
    static __device__ __forceinline__ float sum(const float* z) {
        return Tree<N / 2>::sum(z) + Tree<N - N / 2>::sum(z + N / 2);
    }
    static __device__ __forceinline__ float max(const float* z) {
        return fmaxf(Tree<N / 2>::max(z), Tree<N - N / 2>::max(z + N / 2));
    }
};
template <>
struct Tree<1> {
    static __device__ __forceinline__ float sum(const float* z) { return z[0]; }
    static __device__ __forceinline__ float max(const float* z) { return z[0]; }
};

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
