// fr_metrics.hip -- evaluation metrics of a plan (Section 4.1's list of
// evaluation metrics): user utility, mean max envy, and the fractions of items
// better / worse off than under the uniform ranking policy.
//
// With the exposure matrix W_uj = sum_{k<m-1} e_k x_ujk (FP64, from the FP32 or
// BF16 plan), the impact item i would get with item j's allocation is
//   E_ij = Imp_i(X_j) = sum_u r_ui W_uj,   i.e.  E = R^T W,
// a dense I x I x U contraction: the one step of the method on matrix cores.
// It runs as an FP64 MFMA GEMM (v_mfma_f64_16x16x4f64).  When the I x I tiles
// alone fill the device, each block's epilogue keeps only its rows' maxima
// and the diagonal, so E never reaches HBM; with few tiles (small I) the
// consumers are split over blocks, each writing its partial tile, and a row
// kernel adds the partials in split order and takes the maxima.  E_ii is item
// i's own impact (Eq. Imp), so
//   envy_i = max_j E_ij - E_ii >= 0,   utility = sum_i E_ii / |U|,
// and the uniform policy's impacts are (sum_u r_ui)(sum_{k<m-1} e_k) / I.
#include <math.h>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;     // E tile edge (items i and j)
constexpr int kKc = 16;       // consumers per LDS stage
constexpr int kLdsPad = 2;    // doubles of padding per LDS row
constexpr int kFillBlocks = 2048;        // blocks that keep every SIMD busy
constexpr int kMinSplitUsers = 64;       // consumers per split at least
constexpr double kMaxSplitBytes = 256.0 * 1024 * 1024;   // partial tiles at most

// W_ui = sum_{k<m-1} e_k x_uik in FP64.  A block's ROWS plan rows are one
// contiguous stretch of X: it is staged into LDS with 16-byte loads when X is
// 16-byte aligned (coalesced; every block's stretch then starts aligned, since
// ROWS * sizeof(T) = 512), element by element otherwise; then each thread
// sums its own row.  LDS: ROWS * m * sizeof(T) <= 32 KB.
template <typename T, int ROWS>
__global__ __launch_bounds__(ROWS) void k_expo(const T* __restrict__ X,
                                               const float* __restrict__ e, int64_t rows, int m,
                                               int vec, double* __restrict__ W) {
    extern __shared__ __align__(16) unsigned char expo_lds[];
    T* buf = (T*)expo_lds;
    const int64_t base = (int64_t)blockIdx.x * ROWS;
    const int n = (int)((rows - base) < ROWS ? (rows - base) : ROWS);
    const int64_t total = (int64_t)n * m;               // elements of the stretch
    constexpr int V = 16 / sizeof(T);                     // elements per 16-byte load
    const T* src = X + base * m;
    const int64_t nvec = vec ? total / V : 0;
    for (int64_t q = threadIdx.x; q < nvec; q += ROWS) ((uint4*)buf)[q] = ((const uint4*)src)[q];
    for (int64_t q = nvec * V + threadIdx.x; q < total; q += ROWS) buf[q] = src[q];
    __syncthreads();
    if ((int)threadIdx.x >= n) return;
    const T* x = buf + (int64_t)threadIdx.x * m;
    double s = 0.0;
    for (int k = 0; k < m - 1; ++k) {
        double v;
        if constexpr (sizeof(T) == 2)
            v = (double)from_bf16(x[k]);
        else
            v = (double)x[k];
        s += (double)e[k] * v;
    }
    W[base + threadIdx.x] = s;
}

// One 64 x 64 tile of E = R^T W per block (4 waves, each 32 x 32 as 2 x 2
// MFMA blocks of 16 x 16).  Operand layout of the FP64 16x16x4 MFMA (64
// lanes, checked on the device): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[l / 16 + 4 q][l % 16], q < 4.  Epilogue: the tile goes through LDS; the
// row maxima over the tile's columns go to pmax[i][blockIdx.y], the diagonal
// (tiles with blockIdx.x == blockIdx.y) to diag.
// Consumers [u_lo, u_hi) of split blockIdx.z.  epart == nullptr: the fused
// epilogue (row maxima of the tile into pmax, the diagonal into diag);
// otherwise the partial tile goes to epart[z][i][j].
__global__ __launch_bounds__(256) void k_envy_gemm(const float* __restrict__ r,
                                                   const double* __restrict__ W, int64_t U, int I,
                                                   int nJ, int64_t per_split,
                                                   double* __restrict__ pmax,
                                                   double* __restrict__ diag,
                                                   double* __restrict__ epart) {
    __shared__ double Rs[kKc][kTile + kLdsPad];
    __shared__ double Ws[kKc][kTile + kLdsPad];
    __shared__ double Et[kTile][kTile + 1];
    const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;

    double4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t u_lo = (int64_t)blockIdx.z * per_split;
    const int64_t u_hi = u_lo + per_split < U ? u_lo + per_split : U;
    for (int64_t u0 = u_lo; u0 < u_hi; u0 += kKc) {
#pragma unroll
        for (int q = 0; q < (kKc * kTile) / 256; ++q) {
            const int idx = tid + q * 256;
            const int kk = idx / kTile, c = idx - kk * kTile;
            const int64_t u = u0 + kk;
            const bool uok = u < u_hi;
            Rs[kk][c] = (uok && i0 + c < I) ? (double)r[u * I + i0 + c] : 0.0;
            Ws[kk][c] = (uok && j0 + c < I) ? W[u * I + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kKc; ks += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Rs[ks + lk][wi + 16 * a + lr];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Ws[ks + lk][wj + 16 * b + lr];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }

    if (epart) {   // partial tile of this split, straight from the accumulators
        double* dst = epart + (int64_t)blockIdx.z * I * I;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + wi + 16 * a + lk + 4 * q, j = j0 + wj + 16 * b + lr;
                    if (i < I && j < I) dst[(int64_t)i * I + j] = acc[a][b][q];
                }
        return;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Et[wi + 16 * a + lk + 4 * q][wj + 16 * b + lr] = acc[a][b][q];
    __syncthreads();

    // 4 threads per row, 16 columns each, then a max over the 4
    const int row = tid >> 2, part = tid & 3;
    double mx = -INFINITY;
    for (int c = part * 16; c < part * 16 + 16; ++c)
        if (j0 + c < I) mx = fmax(mx, Et[row][c]);
    mx = fmax(mx, __shfl_xor(mx, 1));
    mx = fmax(mx, __shfl_xor(mx, 2));
    if (part == 0 && i0 + row < I) {
        pmax[(int64_t)(i0 + row) * nJ + blockIdx.y] = mx;
        if (blockIdx.x == blockIdx.y) diag[i0 + row] = Et[row][row];
    }
}

// Row i of E from the split partials (added in split order): its maximum into
// pmax[i] (one column tile) and E_ii into diag[i].
constexpr int kRowThreads = 256;
__global__ __launch_bounds__(kRowThreads) void k_envy_rows(const double* __restrict__ epart,
                                                           int splits, int I,
                                                           double* __restrict__ pmax,
                                                           double* __restrict__ diag) {
    __shared__ double red[kRowThreads];
    const int i = blockIdx.x;
    double mx = -INFINITY;
    for (int j = threadIdx.x; j < I; j += kRowThreads) {
        double e = 0.0;
        for (int sp = 0; sp < splits; ++sp) e += epart[((int64_t)sp * I + i) * I + j];
        mx = fmax(mx, e);
        if (j == i) diag[i] = e;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kRowThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pmax[i] = red[0];
}

// envy_i = max_j E_ij - E_ii; the four metrics (FP64, fixed summation order).
constexpr int kFinal = 512;
__global__ __launch_bounds__(kFinal) void k_metrics_final(const double* __restrict__ pmax,
                                                          const double* __restrict__ diag,
                                                          const double* __restrict__ rsum,
                                                          const float* __restrict__ e, int I, int m,
                                                          int nJ, int64_t U, double* out,
                                                          double* envy, double* imp) {
    __shared__ double red[4][kFinal];
    double esum = 0.0;
    for (int k = 0; k < m - 1; ++k) esum += (double)e[k];
    double s_env = 0.0, s_imp = 0.0, n_better = 0.0, n_worse = 0.0;
    for (int i = threadIdx.x; i < I; i += kFinal) {
        double mx = -INFINITY;
        for (int jb = 0; jb < nJ; ++jb) mx = fmax(mx, pmax[(int64_t)i * nJ + jb]);
        const double own = diag[i];
        const double env = mx - own;
        const double uni = rsum[i] * esum / (double)I;
        s_env += env;
        s_imp += own;
        n_better += (own > 1.1 * uni) ? 1.0 : 0.0;
        n_worse += (own < 0.9 * uni) ? 1.0 : 0.0;
        if (envy) envy[i] = env;
        if (imp) imp[i] = own;
    }
    red[0][threadIdx.x] = s_env;
    red[1][threadIdx.x] = s_imp;
    red[2][threadIdx.x] = n_better;
    red[3][threadIdx.x] = n_worse;
    __syncthreads();
    for (int w = kFinal / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[1][0] / (double)U;
        out[1] = red[0][0] / (double)I;
        out[2] = red[2][0] / (double)I;
        out[3] = red[3][0] / (double)I;
    }
}

}  // namespace

int metrics_tiles(int I) { return (I + kTile - 1) / kTile; }

int metrics_splits(int64_t U, int I) {
    const int nJ = metrics_tiles(I);
    int64_t S = (kFillBlocks + (int64_t)nJ * nJ - 1) / ((int64_t)nJ * nJ);
    const int64_t by_users = (U + kMinSplitUsers - 1) / kMinSplitUsers;
    const int64_t by_bytes = (int64_t)(kMaxSplitBytes / (8.0 * (double)I * (double)I));
    if (S > by_users) S = by_users;
    if (S > by_bytes) S = by_bytes;
    return S < 2 ? 1 : (int)S;
}

void launch_metrics(const void* X, int x_bf16, const float* r, const float* e, int64_t U, int I,
                    int m, const MetricsBufs& b, double* out, double* envy, double* imp,
                    hipStream_t s) {
    const int64_t rows = U * (int64_t)I;
    const int vec = ((uintptr_t)X % 16) == 0;
    if (x_bf16)
        hipLaunchKernelGGL((k_expo<uint16_t, 256>), dim3((unsigned)((rows + 255) / 256)), dim3(256),
                           (size_t)256 * m * sizeof(uint16_t), s, (const uint16_t*)X, e, rows, m,
                           vec, b.W);
    else
        hipLaunchKernelGGL((k_expo<float, 128>), dim3((unsigned)((rows + 127) / 128)), dim3(128),
                           (size_t)128 * m * sizeof(float), s, (const float*)X, e, rows, m, vec,
                           b.W);
    // sum_u r_ui in FP64 with the impact reduction (its header is scratch)
    launch_impact(r, U, I, b.partial, b.nchunk, b.rsum, nullptr, nullptr, 0, b.hdr, 0, s);
    const int nJ = metrics_tiles(I);
    if (b.splits > 1) {
        // per split a multiple of the LDS stage, so only the last split is ragged
        int64_t per = (U + b.splits - 1) / b.splits;
        per = (per + kKc - 1) / kKc * kKc;
        hipLaunchKernelGGL(k_envy_gemm, dim3(nJ, nJ, b.splits), dim3(256), 0, s, r,
                           (const double*)b.W, U, I, nJ, per, b.pmax, b.diag, b.epart);
        hipLaunchKernelGGL(k_envy_rows, dim3(I), dim3(kRowThreads), 0, s, (const double*)b.epart,
                           b.splits, I, b.pmax, b.diag);
        hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(kFinal), 0, s, (const double*)b.pmax,
                           (const double*)b.diag, (const double*)b.rsum, e, I, m, 1, U, out, envy,
                           imp);
    } else {
        hipLaunchKernelGGL(k_envy_gemm, dim3(nJ, nJ, 1), dim3(256), 0, s, r, (const double*)b.W, U,
                           I, nJ, U, b.pmax, b.diag, (double*)nullptr);
        hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(kFinal), 0, s, (const double*)b.pmax,
                           (const double*)b.diag, (const double*)b.rsum, e, I, m, nJ, U, out, envy,
                           imp);
    }
}

}  // namespace fr
