// fr_plain.hip -- the unfused GPU form of Algorithm 1, kept as the
// performance baseline of the fused kernels.
//
// It computes the same T-iterate Sinkhorn map and its reverse-mode gradient
// (Section 3) the way a tensor library would: every half-iteration is its own
// kernel launch that re-reads the cost tensor from HBM, the potentials of
// every iteration are stored in HBM, and the reverse sweep reads them back.
// Each half-step evaluates its log-sum-exp in natural units with the device
// expf/logf:
//   row    f_i = -eps LSE_k((g_k - c_ik)/eps)
//   column g_k =  eps log b_k - eps LSE_i((f_i - c_ik)/eps)
// Reverse of the column half-step (Q_ik = exp((f_i + g_k - c_ik)/eps) / b_k):
//   fbar_i = [t = T] fbar0_i - sum_k Q_ik gbar_k,   cbar_ik += Q_ik gbar_k
// Reverse of the row half-step (P_ik = exp((f_i + g^{t-1}_k - c_ik)/eps)):
//   cbar_ik += P_ik fbar_i,   gbar_k <- -sum_i P_ik fbar_i
#include <hip/hip_runtime.h>
#include <math.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {
namespace {

constexpr int kColsPerBlock = 8;   // columns reduced by one block
constexpr int kLanesPerCol = 32;   // lanes sharing one column's rows

__device__ __forceinline__ float col_mass(int k, int I, int m) {
    return (k == m - 1) ? (float)(I - m + 1) : 1.0f;
}

// Online (max, sum) merge for a log-sum-exp.
__device__ __forceinline__ void lse_merge(float& M, float& S, float M2, float S2) {
    if (M2 > M) {
        S = S * expf(M - M2) + S2;
        M = M2;
    } else if (M2 > -INFINITY) {
        S += S2 * expf(M2 - M);
    }
}

__device__ __forceinline__ void lse_push(float& M, float& S, float z) {
    if (z > M) {
        S = S * expf(M - z) + 1.0f;
        M = z;
    } else {
        S += expf(z - M);
    }
}

// Row half-step: f^t[u][i] from g^{t-1}[u][:].
__global__ __launch_bounds__(256) void k_row(const float* __restrict__ C, const float* __restrict__ gprev,
                                             float* __restrict__ f, int64_t U, int I, int m,
                                             float eps) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= U * I) return;
    const int64_t u = row / I;
    const float* c = C + row * m;
    const float* g = gprev + u * m;
    float M = -INFINITY, S = 0.f;
    for (int k = 0; k < m; ++k) lse_push(M, S, (g[k] - c[k]) / eps);
    f[row] = -eps * (M + logf(S));
}

// Column half-step: g^t[u][k] from f^t[u][:].  Block = 8 columns x 32 lanes.
__global__ __launch_bounds__(256) void k_col(const float* __restrict__ C, const float* __restrict__ f,
                                             float* __restrict__ g, int I, int m, float eps) {
    const int64_t u = blockIdx.x;
    const int k = blockIdx.y * kColsPerBlock + threadIdx.x / kLanesPerCol;
    const int j = threadIdx.x % kLanesPerCol;
    float M = -INFINITY, S = 0.f;
    if (k < m) {
        for (int i = j; i < I; i += kLanesPerCol)
            lse_push(M, S, (f[u * I + i] - C[(u * I + i) * m + k]) / eps);
    }
    for (int d = kLanesPerCol / 2; d > 0; d >>= 1) {
        const float M2 = __shfl_xor(M, d, kLanesPerCol);
        const float S2 = __shfl_xor(S, d, kLanesPerCol);
        lse_merge(M, S, M2, S2);
    }
    if (k < m && j == 0) g[u * m + k] = eps * logf(col_mass(k, I, m)) - eps * (M + logf(S));
}

// Plan from the final potentials, and y_ui = r_ui sum_{k<m-1} e_k x_uik.
__global__ __launch_bounds__(256) void k_plan(const float* __restrict__ C, const float* __restrict__ f,
                                              const float* __restrict__ g, const float* __restrict__ r,
                                              const float* __restrict__ e, float* y, void* X,
                                              int bf16, int64_t U, int I, int m, float eps) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= U * I) return;
    const int64_t u = row / I;
    float s = 0.f;
    for (int k = 0; k < m; ++k) {
        const float x = expf((f[row] + g[u * m + k] - C[row * m + k]) / eps);
        if (k < m - 1) s += e[k] * x;
        if (X) {
            if (bf16)
                ((uint16_t*)X)[row * m + k] = to_bf16(x);
            else
                ((float*)X)[row * m + k] = x;
        }
    }
    y[row] = r[row] * s;
}

// Adjoint of X = exp((f+g-c)/eps) with G = r_i e_k / Imp_i: cbar, fbar0.
__global__ __launch_bounds__(256) void k_adj_init_rows(const float* __restrict__ C, const float* __restrict__ f,
                                                       const float* __restrict__ g, const float* __restrict__ r,
                                                       const float* __restrict__ e, const double* __restrict__ imp,
                                                       float* cbar, float* fbar0, int64_t U, int I, int m,
                                                       float eps) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= U * I) return;
    const int64_t u = row / I;
    const int i = (int)(row - u * I);
    const float gi = (float)((double)r[row] / imp[i]);
    float s = 0.f;
    for (int k = 0; k < m; ++k) {
        const float x = expf((f[row] + g[u * m + k] - C[row * m + k]) / eps);
        const float gx = (k < m - 1) ? gi * e[k] * x / eps : 0.f;
        cbar[row * m + k] = -gx;
        s += gx;
    }
    fbar0[row] = s;
}

// gbar^T_k = sum_i G_ik X_ik / eps (column sums), block = 8 columns x 32 lanes.
__global__ __launch_bounds__(256) void k_adj_init_cols(const float* __restrict__ C, const float* __restrict__ f,
                                                       const float* __restrict__ g, const float* __restrict__ r,
                                                       const float* __restrict__ e, const double* __restrict__ imp,
                                                       float* gbar, int I, int m, float eps) {
    const int64_t u = blockIdx.x;
    const int k = blockIdx.y * kColsPerBlock + threadIdx.x / kLanesPerCol;
    const int j = threadIdx.x % kLanesPerCol;
    float s = 0.f;
    if (k < m - 1) {
        for (int i = j; i < I; i += kLanesPerCol) {
            const int64_t row = u * I + i;
            const float x = expf((f[row] + g[u * m + k] - C[row * m + k]) / eps);
            s += (float)((double)r[row] / imp[i]) * e[k] * x / eps;
        }
    }
    for (int d = kLanesPerCol / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kLanesPerCol);
    if (k < m && j == 0) gbar[u * m + k] = s;
}

// Reverse of the column half-step of iteration t (per row).
__global__ __launch_bounds__(256) void k_rev_col(const float* __restrict__ C, const float* __restrict__ ft,
                                                 const float* __restrict__ gt, const float* __restrict__ gbar,
                                                 const float* __restrict__ fbar0, float* fbar, float* cbar,
                                                 int64_t U, int I, int m, float eps, int first) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= U * I) return;
    const int64_t u = row / I;
    float fb = first ? fbar0[row] : 0.f;
    for (int k = 0; k < m; ++k) {
        const float Q = expf((ft[row] + gt[u * m + k] - C[row * m + k]) / eps) / col_mass(k, I, m);
        fb -= Q * gbar[u * m + k];
        cbar[row * m + k] += Q * gbar[u * m + k];
    }
    fbar[row] = fb;
}

// Reverse of the row half-step of iteration t: cbar += P fbar and
// gbar^{t-1} = -P^T fbar (block = 8 columns x 32 lanes).
__global__ __launch_bounds__(256) void k_rev_row(const float* __restrict__ C, const float* __restrict__ ft,
                                                 const float* __restrict__ gprev, const float* __restrict__ fbar,
                                                 float* cbar, float* gbar, int I, int m, float eps) {
    const int64_t u = blockIdx.x;
    const int k = blockIdx.y * kColsPerBlock + threadIdx.x / kLanesPerCol;
    const int j = threadIdx.x % kLanesPerCol;
    float s = 0.f;
    if (k < m) {
        for (int i = j; i < I; i += kLanesPerCol) {
            const int64_t row = u * I + i;
            const float P = expf((ft[row] + gprev[u * m + k] - C[row * m + k]) / eps);
            cbar[row * m + k] += P * fbar[row];
            s += P * fbar[row];
        }
    }
    for (int d = kLanesPerCol / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kLanesPerCol);
    if (k < m && j == 0) gbar[u * m + k] = -s;
}

__global__ __launch_bounds__(256) void k_update(float* C, float* mom, float* vel, const float* g,
                                                int64_t n, int rule, float lr, float b1, float b2,
                                                float aeps, const int64_t* step_ptr) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (rule == 1) {
        C[j] += lr * g[j];
        return;
    }
    const int64_t st = *step_ptr;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)st));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)st));
    const float gl = -g[j];
    const float mo = b1 * mom[j] + (1.f - b1) * gl;
    const float ve = b2 * vel[j] + (1.f - b2) * gl * gl;
    mom[j] = mo;
    vel[j] = ve;
    C[j] -= lr * (mo / bc1) / (sqrtf(ve / bc2) + aeps);
}

__global__ void k_zero(float* p, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = 0.f;
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void plain_forward(const float* C, const float* r, const float* e, int64_t U, int I, int m,
                   float eps, int T, const PlainBufs& b, void* X, int bf16, hipStream_t s) {
    const int64_t rows = U * I;
    hipLaunchKernelGGL(k_zero, dim3(nblk(U * m)), dim3(256), 0, s, b.gh, U * m);  // g^0 = 0
    const dim3 cgrid((unsigned)U, (unsigned)((m + kColsPerBlock - 1) / kColsPerBlock));
    for (int t = 1; t <= T; ++t) {
        float* ft = b.fh + (int64_t)(t - 1) * rows;
        const float* gp = b.gh + (int64_t)(t - 1) * U * m;
        float* gt = b.gh + (int64_t)t * U * m;
        hipLaunchKernelGGL(k_row, dim3(nblk(rows)), dim3(256), 0, s, C, gp, ft, U, I, m, eps);
        hipLaunchKernelGGL(k_col, cgrid, dim3(256), 0, s, C, ft, gt, I, m, eps);
    }
    hipLaunchKernelGGL(k_plan, dim3(nblk(rows)), dim3(256), 0, s, C,
                       b.fh + (int64_t)(T - 1) * rows, b.gh + (int64_t)T * U * m, r, e, b.y, X,
                       bf16, U, I, m, eps);
}

void plain_backward_update(float* C, const float* r, const float* e, int64_t U, int I, int m,
                           float eps, int T, const PlainBufs& b, float* mom, float* vel, int rule,
                           float lr, float b1, float b2, float aeps, bool apply, hipStream_t s) {
    const int64_t rows = U * I;
    const dim3 cgrid((unsigned)U, (unsigned)((m + kColsPerBlock - 1) / kColsPerBlock));
    const float* fT = b.fh + (int64_t)(T - 1) * rows;
    const float* gT = b.gh + (int64_t)T * U * m;
    hipLaunchKernelGGL(k_adj_init_rows, dim3(nblk(rows)), dim3(256), 0, s, C, fT, gT, r, e, b.imp,
                       b.cbar, b.fbar0, U, I, m, eps);
    hipLaunchKernelGGL(k_adj_init_cols, cgrid, dim3(256), 0, s, C, fT, gT, r, e, b.imp, b.gbar, I,
                       m, eps);
    for (int t = T; t >= 1; --t) {
        const float* ft = b.fh + (int64_t)(t - 1) * rows;
        const float* gt = b.gh + (int64_t)t * U * m;
        const float* gp = b.gh + (int64_t)(t - 1) * U * m;
        hipLaunchKernelGGL(k_rev_col, dim3(nblk(rows)), dim3(256), 0, s, C, ft, gt, b.gbar, b.fbar0,
                           b.fbar, b.cbar, U, I, m, eps, (int)(t == T));
        hipLaunchKernelGGL(k_rev_row, cgrid, dim3(256), 0, s, C, ft, gp, b.fbar, b.cbar, b.gbar, I,
                           m, eps);
    }
    if (apply)
        hipLaunchKernelGGL(k_update, dim3(nblk(rows * m)), dim3(256), 0, s, C, mom, vel, b.cbar,
                           rows * m, rule, lr, b1, b2, aeps, &b.hdr->step);
}

}  // namespace fr
