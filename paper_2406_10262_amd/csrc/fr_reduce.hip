// fr_reduce.hip -- the only cross-consumer step of the method: item impacts
// Imp_i = sum_u y_ui (Eq. Imp, with y_ui = r_ui sum_{k<m} e_k x_uik formed by
// the producing kernel) and the objective F = sum_i log Imp_i (Eq. objF).
//
// Both sums run in FP64 in a fixed order (consumer chunks, then chunks in
// index order, then a fixed tree over items), so results are bitwise
// reproducible from run to run.  Imp_i <= 0 or a non-finite value raises a
// sticky flag in the workspace header instead of failing the launch.
#include <math.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {
namespace {

constexpr int kChunk = 16;       // consumers per first-stage partial sum
constexpr int kItemLanes = 32;   // lanes summing one item's partials
constexpr int kFinalThreads = 1024;

// Stage 1: partial[ch][i] = sum of y[u][i] over the 16 consumers of chunk ch
// (independent loads, added in consumer order).
__global__ __launch_bounds__(256) void k_imp_partial(const float* __restrict__ y, int64_t U, int I,
                                                     double* __restrict__ partial) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ch = blockIdx.y;
    if (i >= I) return;
    const int64_t u0 = ch * kChunk;
    float v[kChunk];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) v[q] = (u0 + q < U) ? y[(u0 + q) * I + i] : 0.f;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kChunk; ++q) s += (double)v[q];
    partial[ch * I + i] = s;
}

// Stage 2: Imp_i = sum over chunks; 32 lanes per item take chunks c = lane
// mod 32 in order, then a fixed tree combines the lanes.
__global__ __launch_bounds__(256) void k_imp_items(const double* __restrict__ partial, int nchunk,
                                                   int I, double* __restrict__ imp) {
    __shared__ double red[256];
    const int lane = threadIdx.x % kItemLanes;
    const int i = blockIdx.x * (256 / kItemLanes) + threadIdx.x / kItemLanes;
    double s = 0.0;
    if (i < I)
        for (int c = lane; c < nchunk; c += kItemLanes) s += partial[(int64_t)c * I + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kItemLanes / 2; w > 0; w >>= 1) {
        if (lane < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (i < I && lane == 0) imp[i] = red[threadIdx.x];
}

// Stage 3: F = sum_i log Imp_i (fixed tree), device flags, F history, step.
__global__ __launch_bounds__(kFinalThreads) void k_imp_final(const double* __restrict__ imp, int I,
                                                             double* F, double* F_hist,
                                                             int64_t start_step, WsHeader* hdr,
                                                             int advance) {
    __shared__ double red[kFinalThreads];
    double lsum = 0.0;
    uint32_t fl = 0;
    for (int i = threadIdx.x; i < I; i += blockDim.x) {
        const double s = imp[i];
        if (!isfinite(s))
            fl |= FLAG_NONFINITE;
        else if (!(s > 0.0))
            fl |= FLAG_ZERO_IMPACT;
        lsum += log(s);
    }
    if (fl) atomicOr(&hdr->flags, fl);
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double Fv = red[0];
        hdr->F = Fv;
        if (F) *F = Fv;
        const int64_t rep = hdr->rep;
        if (F_hist) F_hist[rep] = Fv;
        if (advance != ADV_NONE) hdr->rep = rep + 1;
        if (advance == ADV_REP_STEP) hdr->step += 1;
    }
}

// y_ui = r_ui sum_{k<m-1} e_k x_uik for an explicit plan (one thread per row).
__global__ __launch_bounds__(256) void k_rows_from_plan(const void* X, int bf16, const float* r,
                                                        const float* e, int64_t rows, int m,
                                                        float* y) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    float s = 0.f;
    if (bf16) {
        const uint16_t* x = (const uint16_t*)X + row * m;
        for (int k = 0; k < m - 1; ++k) s = fmaf(e[k], from_bf16(x[k]), s);
    } else {
        const float* x = (const float*)X + row * m;
        for (int k = 0; k < m - 1; ++k) s = fmaf(e[k], x[k], s);
    }
    y[row] = r[row] * s;
}

// ---- batched forms: blockIdx.x indexes a host-built table of (instance, part)
__global__ __launch_bounds__(256) void k_bimp_partial(const RedDesc* __restrict__ descs,
                                                      const int2* __restrict__ tab) {
    const int2 t = tab[blockIdx.x];
    const RedDesc d = descs[t.x];
    const int64_t u0 = (int64_t)t.y * kChunk;
    for (int i = threadIdx.x; i < d.I; i += blockDim.x) {
        float v[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) v[q] = (u0 + q < d.U) ? d.y[(u0 + q) * d.I + i] : 0.f;
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < kChunk; ++q) sacc += (double)v[q];
        d.partial[(int64_t)t.y * d.I + i] = sacc;
    }
}

__global__ __launch_bounds__(256) void k_bimp_items(const RedDesc* __restrict__ descs,
                                                    const int2* __restrict__ tab) {
    __shared__ double red[256];
    const int2 t = tab[blockIdx.x];
    const RedDesc d = descs[t.x];
    const int lane = threadIdx.x % kItemLanes;
    const int i = t.y * (256 / kItemLanes) + threadIdx.x / kItemLanes;
    double sacc = 0.0;
    if (i < d.I)
        for (int c = lane; c < d.nchunk; c += kItemLanes) sacc += d.partial[(int64_t)c * d.I + i];
    red[threadIdx.x] = sacc;
    __syncthreads();
    for (int w = kItemLanes / 2; w > 0; w >>= 1) {
        if (lane < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (i < d.I && lane == 0) d.imp[i] = red[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_bimp_final(const RedDesc* __restrict__ descs,
                                                    int64_t start_step, WsHeader* hdr) {
    __shared__ double red[256];
    const RedDesc d = descs[blockIdx.x];
    double lsum = 0.0;
    uint32_t fl = 0;
    for (int i = threadIdx.x; i < d.I; i += blockDim.x) {
        const double v = d.imp[i];
        if (!isfinite(v))
            fl |= FLAG_NONFINITE;
        else if (!(v > 0.0))
            fl |= FLAG_ZERO_IMPACT;
        lsum += log(v);
    }
    if (fl) atomicOr(&hdr->flags, fl);
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && d.F_hist) d.F_hist[hdr->step - start_step] = red[0];
}

// Gradient-norm test: FP64 sums of squares over fixed chunks, then one block.
constexpr int kNormPer = 64;   // elements per thread
__global__ __launch_bounds__(256) void k_gnorm_partial(const float* __restrict__ g, int64_t n,
                                                       double* __restrict__ partial,
                                                       const int32_t* stop) {
    __shared__ double red[256];
    if (*stop) return;
    const int64_t base = (int64_t)blockIdx.x * (256 * kNormPer);
    double sq = 0.0;
    for (int q = 0; q < kNormPer; ++q) {
        const int64_t j = base + (int64_t)q * 256 + threadIdx.x;
        if (j < n) {
            const double v = (double)g[j];
            sq += v * v;
        }
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_gnorm_final(const double* __restrict__ partial, int nb,
                                                      double tol, WsHeader* hdr) {
    __shared__ double red[1024];
    if (hdr->stopped) return;
    double sq = 0.0;
    for (int b = threadIdx.x; b < nb; b += 1024) sq += partial[b];
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gn = sqrt(red[0]);
        hdr->gnorm = gn;
        if (gn <= tol)
            hdr->stopped = 1;
        else
            hdr->step += 1;
    }
}

// C += lr g (ascent) or the Adam step on -g (maximisation), unless stopped.
__global__ __launch_bounds__(256) void k_apply(float* __restrict__ C, float* __restrict__ mom,
                                               float* __restrict__ vel, const float* __restrict__ g,
                                               int64_t n, int rule, float lr, float b1, float b2,
                                               float aeps, const WsHeader* hdr) {
    if (hdr->stopped) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (rule == 1) {
        C[j] += lr * g[j];
        return;
    }
    const int64_t st = hdr->step;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)st));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)st));
    const float gl = -g[j];
    const float mo = b1 * mom[j] + (1.f - b1) * gl;
    const float ve = b2 * vel[j] + (1.f - b2) * gl * gl;
    mom[j] = mo;
    vel[j] = ve;
    C[j] -= lr * (mo / bc1) / (sqrtf(ve / bc2) + aeps);
}

}  // namespace

int gnorm_blocks(int64_t n) { return (int)((n + 256 * kNormPer - 1) / (256 * kNormPer)); }

void launch_gnorm_update(const float* g, float* C, float* mom, float* vel, int64_t n, int rule,
                         float lr, float b1, float b2, float aeps, double* partial, double tol,
                         WsHeader* hdr, hipStream_t s) {
    const int nb = gnorm_blocks(n);
    hipLaunchKernelGGL(k_gnorm_partial, dim3(nb), dim3(256), 0, s, g, n, partial, &hdr->stopped);
    hipLaunchKernelGGL(k_gnorm_final, dim3(1), dim3(1024), 0, s, (const double*)partial, nb, tol,
                       hdr);
    hipLaunchKernelGGL(k_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, mom, vel, g,
                       n, rule, lr, b1, b2, aeps, (const WsHeader*)hdr);
}

void launch_impact_batched(const RedDesc* descs, int n_inst, const int2* tab1, int n1,
                           const int2* tab2, int n2, int64_t start_step, WsHeader* hdr,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_bimp_partial, dim3(n1), dim3(256), 0, s, descs, tab1);
    hipLaunchKernelGGL(k_bimp_items, dim3(n2), dim3(256), 0, s, descs, tab2);
    hipLaunchKernelGGL(k_bimp_final, dim3(n_inst), dim3(256), 0, s, descs, start_step, hdr);
}

int impact_item_groups(int I) { return (I + 256 / kItemLanes - 1) / (256 / kItemLanes); }

int impact_chunks(int64_t U, int I) {
    (void)I;
    return (int)((U + kChunk - 1) / kChunk);
}

void launch_impact(const float* y, int64_t U, int I, double* partial, int nchunk, double* imp,
                   double* F, double* F_hist, int64_t start_step, WsHeader* hdr, int advance,
                   hipStream_t s) {
    dim3 g1((I + 255) / 256, nchunk);
    hipLaunchKernelGGL(k_imp_partial, g1, dim3(256), 0, s, y, U, I, partial);
    hipLaunchKernelGGL(k_imp_items, dim3((I + 7) / 8), dim3(256), 0, s, partial, nchunk, I, imp);
    hipLaunchKernelGGL(k_imp_final, dim3(1), dim3(kFinalThreads), 0, s, imp, I, F, F_hist,
                       start_step, hdr, advance);
}

void launch_rows_from_plan(const void* X, int x_bf16, const float* r, const float* e, int64_t U,
                           int I, int m, float* y, hipStream_t s) {
    const int64_t rows = U * I;
    hipLaunchKernelGGL(k_rows_from_plan, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, X,
                       x_bf16, r, e, rows, m, y);
}

}  // namespace fr
