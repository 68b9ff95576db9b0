// fr_baselines.hip -- the baseline rankings of the comparison in Section 4.1:
// MaxRele and NSW(Greedy).  Both give deterministic 0/1 plans: sel[u][k] is
// the item consumer u sees at real position k (k < m-1); every other item
// goes to the dummy position.
//
// MaxRele: each consumer's items by descending relevance (equal relevances by
// item index).  One wave per consumer; lane l holds items l + 64 j; m-1
// rounds of a wave argmax.
//
// NSW(Greedy): the paper states only that greedy chooses items by F(X) for
// each position.  Rule fixed here: the real positions are filled in order,
// at each position the consumers choose in index order, and a consumer takes
// the item it has not placed yet whose placement raises F = sum_i log Imp_i
// (Eq. objF) the most.  Placing i at k adds r_ui e_k to Imp_i alone, so the
// gain log(1 + e_k r_ui / Imp_i) is increasing in r_ui / Imp_i: the choice is
// the largest ratio (FP64; Imp_i = 0 counts as +inf), then the larger r_ui,
// then the smaller index.  The U (m-1) decisions form one dependency chain,
// so a single block walks them with the impacts in LDS (FP64, accumulated in
// decision order); the items of a decision are spread over the block, and
// the next decision's relevances and earlier selections are loaded while the
// current one is reduced.
#include <math.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {
namespace {

constexpr int kMaxI = 4096;
constexpr int kGreedyIpt = 4;    // items per thread of the greedy block

// (key, r, i) order of the greedy choice: larger key, larger r, smaller i.
__device__ __forceinline__ bool greedy_better(double k, float r, int i, double bk, float br,
                                              int bi) {
    if (k != bk) return k > bk;
    if (r != br) return r > br;
    return i < bi;
}

__global__ __launch_bounds__(256) void k_maxrele(const float* __restrict__ r, int64_t U, int I,
                                                 int m, int32_t* __restrict__ sel) {
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (u >= U) return;   // the whole wave leaves together
    const float* ru = r + u * I;
    const int J = (I + 63) >> 6;
    uint64_t taken = 0;   // bit j: item lane + 64 j already placed
    for (int k = 0; k < m - 1; ++k) {
        float bv = -INFINITY;
        int bi = 0x7fffffff;
        for (int j = 0; j < J; ++j) {
            const int i = lane + 64 * j;
            if (i < I && !((taken >> j) & 1ull)) {
                float v = ru[i];
                v = (v == v) ? v : -INFINITY;   // a NaN relevance ranks last
                if (v > bv || (v == bv && i < bi)) {
                    bv = v;
                    bi = i;
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        // m - 1 < I, so an untaken item always exists and bi is a valid item
        if (lane == (bi & 63)) taken |= 1ull << (bi >> 6);
        if (lane == 0) sel[u * (m - 1) + k] = bi;
    }
}

__global__ __launch_bounds__(1024) void k_greedy(const float* __restrict__ r,
                                                 const float* __restrict__ e, int64_t U, int I,
                                                 int m, int32_t* sel, double* imp_out) {
    __shared__ double imp[kMaxI];
    __shared__ int mark[kMaxI];       // decision number of the consumer that placed the item
    __shared__ double wk[16];
    __shared__ float wr[16];
    __shared__ int wi[16];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int nw = nt >> 6;
    for (int i = tid; i < I; i += nt) {
        imp[i] = 0.0;
        mark[i] = -1;
    }
    const int64_t D = U * (int64_t)(m - 1);
    // operands of decision d = k U + u: relevances of consumer u, and the
    // items u placed at positions < k (thread t < k holds position t)
    float rcur[kGreedyIpt];
    int scur = -1;
    auto load = [&](int64_t d, float (&rv)[kGreedyIpt], int& s) {
        const int k = (int)(d / U);
        const int64_t u = d - (int64_t)k * U;
#pragma unroll
        for (int q = 0; q < kGreedyIpt; ++q) {
            const int i = tid + q * nt;
            rv[q] = (i < I) ? r[u * I + i] : 0.f;
        }
        s = (tid < k) ? sel[u * (m - 1) + tid] : -1;
    };
    load(0, rcur, scur);
    __syncthreads();
    for (int64_t d = 0; d < D; ++d) {
        const int k = (int)(d / U);
        const int64_t u = d - (int64_t)k * U;
        // prefetch the next decision, except where it reads this one's result
        // (one consumer: position k + 1 needs the item chosen now)
        float rnext[kGreedyIpt];
        int snext = -1;
        const bool pre = d + 1 < D && U > 1;
        if (pre) load(d + 1, rnext, snext);

        if (scur >= 0) mark[scur] = (int)(d & 0x7fffffff);
        __syncthreads();
        double bk = -INFINITY;
        float br = -INFINITY;
        int bi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < kGreedyIpt; ++q) {
            const int i = tid + q * nt;
            if (i >= I || mark[i] == (int)(d & 0x7fffffff)) continue;
            float rv = rcur[q];
            rv = (rv == rv) ? rv : -INFINITY;
            const double key = imp[i] > 0.0 ? (double)rv / imp[i] : INFINITY;
            if (greedy_better(key, rv, i, bk, br, bi)) {
                bk = key;
                br = rv;
                bi = i;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ok = __shfl_xor(bk, off);
            const float orr = __shfl_xor(br, off);
            const int oi = __shfl_xor(bi, off);
            if (greedy_better(ok, orr, oi, bk, br, bi)) {
                bk = ok;
                br = orr;
                bi = oi;
            }
        }
        if (lane == 0) {
            wk[wave] = bk;
            wr[wave] = br;
            wi[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < nw; ++w)
                if (greedy_better(wk[w], wr[w], wi[w], bk, br, bi)) {
                    bk = wk[w];
                    br = wr[w];
                    bi = wi[w];
                }
            // k < m - 1 <= I - 1 earlier placements leave a candidate: bi < I
            sel[u * (m - 1) + k] = bi;
            imp[bi] += (double)r[u * I + bi] * (double)e[k];
        }
        __syncthreads();
        if (pre) {
#pragma unroll
            for (int q = 0; q < kGreedyIpt; ++q) rcur[q] = rnext[q];
            scur = snext;
        } else if (d + 1 < D) {
            load(d + 1, rcur, scur);
        }
    }
    for (int i = tid; i < I; i += nt)
        if (imp_out) imp_out[i] = imp[i];
}

// The 0/1 plan of a selection: one thread per plan row.
__global__ __launch_bounds__(256) void k_plan_from_sel(const int32_t* __restrict__ sel,
                                                       int64_t U, int I, int m, void* X,
                                                       int bf16) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= U * (int64_t)I) return;
    const int64_t u = row / I;
    const int i = (int)(row - u * I);
    int pos = m - 1;
    for (int k = 0; k < m - 1; ++k)
        if (sel[u * (m - 1) + k] == i) pos = k;
    if (bf16) {
        uint16_t* x = (uint16_t*)X + row * m;
        for (int k = 0; k < m; ++k) x[k] = to_bf16(k == pos ? 1.f : 0.f);
    } else {
        float* x = (float*)X + row * m;
        for (int k = 0; k < m; ++k) x[k] = (k == pos) ? 1.f : 0.f;
    }
}

}  // namespace

int greedy_block(int I) {
    int per = (I + kGreedyIpt - 1) / kGreedyIpt;
    int nt = ((per + 63) / 64) * 64;
    return nt < 64 ? 64 : nt;
}

void launch_maxrele(const float* r, int64_t U, int I, int m, int32_t* sel, hipStream_t s) {
    const int64_t blocks = (U + 3) / 4;
    hipLaunchKernelGGL(k_maxrele, dim3((unsigned)blocks), dim3(256), 0, s, r, U, I, m, sel);
}

void launch_greedy(const float* r, const float* e, int64_t U, int I, int m, int32_t* sel,
                   double* imp, hipStream_t s) {
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(greedy_block(I)), 0, s, r, e, U, I, m, sel, imp);
}

void launch_plan_from_sel(const int32_t* sel, int64_t U, int I, int m, void* X, int bf16,
                          hipStream_t s) {
    const int64_t rows = U * (int64_t)I;
    hipLaunchKernelGGL(k_plan_from_sel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                       sel, U, I, m, X, bf16);
}

}  // namespace fr
