// fr_fused.hip -- fused Sinkhorn forward and adjoint backward for gfx950.
//
// Compiled once per column class with -DFR_MP=<mp>: every kernel here handles
// plans of m <= FR_MP columns (the last real column m-1 is the dummy
// position, Section 2).
//
// Mapping.  A "team" of L lanes owns one consumer u.  Lane l of the team owns
// plan rows i = l + j*L (j < R) and keeps their m costs in registers for the
// whole kernel, so the T Sinkhorn iterations (Section 3, problem otp) never
// touch HBM.  The row half-step (softmax over the m positions of a row) is
// lane-local; the column half-step needs the sum over the team's rows, done
// with DPP/permlane butterflies inside a wave and, for teams of several
// waves, one LDS exchange per half-step.
//
// Arithmetic.  Log-domain, base 2: with gamma_k = g_k / (eps ln 2) and the
// cost exponent z_ik = -c_ik / (eps ln 2) + gamma_k (one FMA), one iteration is
//   P_ik   = 2^(z_ik - M_i) / s_i          (row softmax, M_i the row max)
//   sig_k  = sum_i P_ik
//   gamma_k += log2 b_k - log2 sig_k        (b = 1 ... 1, I-m+1)
// which is the textbook pair of LSE half-steps with a single exponential per
// cell.  The plan is X_ik = 2^(z^T_ik + phi_i), phi_i = -(M_i + log2 s_i) from
// the last row half-step.
//
// Backward (Section 3, "chain rule").  With P^t and the column sums sig^t of
// iteration t, the adjoints of (f, g) and C run backwards as
//   gh_k  = gbar_k / sig^t_k,        sig^t_k = b_k 2^(gamma^{t-1}_k - gamma^t_k)
//   fbar_i = [t = T] fbar0_i - sum_k P_ik gh_k
//   cbar_ik += P_ik (gh_k + fbar_i)
//   gbar_k <- -sum_i P_ik fbar_i
// starting from X, G = dF/dX (G_ik = r_i e_k / Imp_i, Eqs. Imp and objF):
//   cbar = -G X / eps,  fbar0 = (G X) 1 / eps,  gbar = (G X)^T 1 / eps.
// Only the column potentials gamma^t are needed to rebuild P^t, so the forward
// keeps them every K iterations and each segment is recomputed on chip.
#include "fr_device.h"
#include "fr_internal.h"

#ifndef FR_MP
#error "compile with -DFR_MP=<padded column count>"
#endif

namespace fr {
namespace {

struct Team {
    int L;      // lanes per consumer
    int lt;     // lane within the team
    int lw;     // lane within the wave
    int wt;     // wave within the team
    int W;      // waves per team
    int team;   // team within the block
    bool wide;  // the team spans at least one whole wave
    bool multi; // the team spans several waves
};

__device__ __forceinline__ Team make_team(int L) {
    Team t;
    const int tid = threadIdx.x;
    t.L = L;
    t.team = tid / L;
    t.lt = tid - t.team * L;
    t.lw = tid & 63;
    t.wt = t.lt >> 6;
    t.W = (L + 63) >> 6;
    t.wide = L >= 64;
    t.multi = L > 64;
    return t;
}

// Sum acc[k] over the team; every lane ends with the totals.
template <int MP>
__device__ __forceinline__ void team_sum(float (&acc)[MP], const Team& tm, float* red, int par) {
    if (!tm.multi) {
        group_allreduce<MP>(acc, tm.L);
        return;
    }
    group_allreduce<MP>(acc, 64);
    const float mine = pick_lane<MP>(acc, tm.lw);
    float* buf = red + par * (tm.W * MP);
    if (tm.lw < MP) buf[tm.wt * MP + tm.lw] = mine;
    __syncthreads();
    float tot = 0.f;
    if (tm.lw < MP) {
        for (int w = 0; w < tm.W; ++w) tot += buf[w * MP + tm.lw];
    }
    spread_lanes<MP>(tot, acc);
}

// Column half-step: gamma_k += log2 b_k - log2 sum_i P_ik.
template <int MP>
__device__ __forceinline__ void column_step(float (&acc)[MP], float (&gam)[MP], const float (&lb)[MP],
                                            int m, const Team& tm, float* red, int par) {
    if (!tm.wide) {
        group_allreduce<MP>(acc, tm.L);
#pragma unroll
        for (int k = 0; k < MP; ++k) gam[k] = (k < m) ? gam[k] + (lb[k] - lg2(acc[k])) : gam[k];
        return;
    }
    // One logarithm per wave: lane k finishes column k, then spreads it.
    float tot;
    if (!tm.multi) {
        group_allreduce<MP>(acc, 64);
        tot = pick_lane<MP>(acc, tm.lw);
    } else {
        group_allreduce<MP>(acc, 64);
        const float mine = pick_lane<MP>(acc, tm.lw);
        float* buf = red + par * (tm.W * MP);
        if (tm.lw < MP) buf[tm.wt * MP + tm.lw] = mine;
        __syncthreads();
        tot = 0.f;
        if (tm.lw < MP) {
            for (int w = 0; w < tm.W; ++w) tot += buf[w * MP + tm.lw];
        }
    }
    const float gmine = pick_lane<MP>(gam, tm.lw);
    const float lbm = pick_lane<MP>(lb, tm.lw);
    const float gnew = (tm.lw < m) ? gmine + (lbm - lg2(tot)) : gmine;
    spread_lanes<MP>(gnew, gam);
}

// Row half-step for the lane's R rows with column potentials gam.  acc gets
// the lane's share of the column sums sum_i P_ik; M, s the row max and sum.
template <int MP, int R>
__device__ __forceinline__ void row_step(const float (&c)[R][MP], const float (&om)[R],
                                         const float (&gam)[MP], float c2, float (&acc)[MP],
                                         float (&Mo)[R], float (&so)[R]) {
#pragma unroll
    for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float z[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k) z[k] = fmaf(c[j][k], c2, gam[k]);
        const float M = Tree<MP>::max(z);
#pragma unroll
        for (int k = 0; k < MP; ++k) z[k] = ex2(z[k] - M);
        const float s = Tree<MP>::sum(z);
        const float w = om[j] * rcp(s);
#pragma unroll
        for (int k = 0; k < MP; ++k) acc[k] = fmaf(z[k], w, acc[k]);
        Mo[j] = M;
        so[j] = s;
    }
}

template <int MP>
__device__ __forceinline__ void store_gamma(float* dst, const float (&gam)[MP], int m) {
#pragma unroll
    for (int k = 0; k < MP; ++k)
        if (k < m) dst[k] = gam[k];
}

template <int MP, int R>
__device__ __forceinline__ void load_costs(const float* C, int64_t u, bool active, const Team& tm,
                                           int I, int m, float (&c)[R][MP], float (&om)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        const bool valid = active && i < I;
        om[j] = valid ? 1.f : 0.f;
        const float* src = C + (u * I + i) * (int64_t)m;
#pragma unroll
        for (int k = 0; k < MP; ++k) c[j][k] = (valid && k < m) ? src[k] : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Forward for the teams of one block: team q of the block owns consumer
// u_first + q.
template <int MP, int R>
__device__ __forceinline__ void fwd_body(const FwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int64_t u = u_first + tm.team;
    // lanes past the last whole team of the block own no consumer
    const bool active = tm.team < (int)(blockDim.x / a.L) && u < a.U;
    const int I = a.I, m = a.m;
    float* red = smem + tm.team * (2 * tm.W * MP);

    float c[R][MP], om[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, c, om);

    float gam[MP], lb[MP];
    const float lbd = lg2((float)(I - m + 1));
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        gam[k] = (k < m) ? 0.f : kNeg;
        lb[k] = (k == m - 1) ? lbd : 0.f;
    }
    float* hist = (a.hist != nullptr && active) ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    if (hist && tm.lt == 0) store_gamma<MP>(hist, gam, m);

    float Ml[R], sl[R], acc[MP];
    for (int t = 1; t <= a.T; ++t) {
        row_step<MP, R>(c, om, gam, a.c2, acc, Ml, sl);
        column_step<MP>(acc, gam, lb, m, tm, red, t & 1);
        if (hist && tm.lt == 0) {
            if (t % a.K == 0)
                store_gamma<MP>(hist + (int64_t)(t / a.K) * a.hs, gam, m);
            else if (t == a.T)
                store_gamma<MP>(hist + (int64_t)(a.nck - 1) * a.hs, gam, m);
        }
    }

    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < m - 1) ? a.e[k] : 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (!(active && i < I)) continue;
        const float phi = -(Ml[j] + lg2(sl[j]));
        const int64_t row = u * I + i;
        float x[MP];
        float yy = 0.f;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            x[k] = ex2(fmaf(c[j][k], a.c2, gam[k]) + phi);
            yy = fmaf(ek[k], x[k], yy);
        }
        if (a.y) a.y[row] = a.r[row] * yy;
        if (a.X) {
            if (a.x_bf16) {
                uint16_t* dst = (uint16_t*)a.X + row * m;
#pragma unroll
                for (int k = 0; k < MP; ++k)
                    if (k < m) dst[k] = to_bf16(x[k]);
            } else {
                float* dst = (float*)a.X + row * m;
#pragma unroll
                for (int k = 0; k < MP; ++k)
                    if (k < m) dst[k] = x[k];
            }
        }
        if (a.pot) a.pot[u * (int64_t)(I + m) + i] = phi * a.eps_ln2;
    }
    if (a.pot && active && tm.lt == 0) {
#pragma unroll
        for (int k = 0; k < MP; ++k)
            if (k < m) a.pot[u * (int64_t)(I + m) + I + k] = gam[k] * a.eps_ln2;
    }
}

template <int MP, int R, int LB>
__global__ __launch_bounds__(LB) void k_fwd(FwdArgs a) {
    extern __shared__ float smem[];
    fwd_body<MP, R>(a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

// ---------------------------------------------------------------------------
template <int MP, int R>
__device__ __forceinline__ void bwd_body(const BwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int teams = blockDim.x / a.L;
    const int64_t u = u_first + tm.team;
    const bool active = tm.team < teams && u < a.U;
    const int I = a.I, m = a.m;
    const int BL = (a.K == 1) ? kLoadBlock : a.K;
    float* seg = smem + tm.team * ((BL + 1) * MP);
    float* red = smem + teams * ((BL + 1) * MP) + tm.team * (2 * tm.W * MP);

    float c[R][MP], om[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, c, om);

    float rg[R];   // gF r_i / Imp_i, so that G_ik = rg_i e_k
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        rg[j] = (active && i < I) ? (float)(a.gF * (double)a.r[u * I + i] / a.imp[i]) : 0.f;
    }
    float lb[MP];
    const float lbd = lg2((float)(I - m + 1));
    const float invbd = 1.0f / (float)(I - m + 1);
#pragma unroll
    for (int k = 0; k < MP; ++k) lb[k] = (k == m - 1) ? lbd : 0.f;

    const float* hist = active ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    float cb[R][MP], fb0[R], gbar[MP], acc[MP], Ml[R], sl[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        fb0[j] = 0.f;
#pragma unroll
        for (int k = 0; k < MP; ++k) cb[j][k] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < MP; ++k) gbar[k] = 0.f;

    int par = 0;
    const int nblk = (a.K == 1) ? (a.T + BL - 1) / BL : (a.nck - 1);
    for (int s = nblk - 1; s >= 0; --s) {
        const int t0 = s * BL;
        const int t1 = min(t0 + BL, a.T);
        const int n = t1 - t0;
        __syncthreads();  // the previous block's reads of seg are complete
        if (a.K == 1) {
            for (int idx = tm.lt; idx < (n + 1) * MP; idx += tm.L) {
                const int q = idx / MP, k = idx - q * MP;
                seg[idx] = (active && k < m) ? hist[(int64_t)(t0 + q) * a.hs + k] : kNeg;
            }
        } else {
            float gam[MP];
#pragma unroll
            for (int k = 0; k < MP; ++k)
                gam[k] = (active && k < m) ? hist[(int64_t)s * a.hs + k] : kNeg;
            if (tm.lt == 0) {
#pragma unroll
                for (int k = 0; k < MP; ++k) seg[k] = gam[k];
            }
            for (int q = 1; q <= n; ++q) {
                row_step<MP, R>(c, om, gam, a.c2, acc, Ml, sl);
                column_step<MP>(acc, gam, lb, m, tm, red, par);
                par ^= 1;
                if (tm.lt == 0) {
#pragma unroll
                    for (int k = 0; k < MP; ++k) seg[q * MP + k] = gam[k];
                }
            }
        }
        __syncthreads();

        for (int q = n; q >= 1; --q) {
            const int t = t0 + q;
            float gp[MP];
#pragma unroll
            for (int k = 0; k < MP; ++k) gp[k] = seg[(q - 1) * MP + k];

            if (t == a.T) {
                // X = P^T * b / sig^T and the adjoints of X = exp((f+g-c)/eps).
#pragma unroll
                for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    float z[MP];
#pragma unroll
                    for (int k = 0; k < MP; ++k) z[k] = fmaf(c[j][k], a.c2, gp[k]);
                    const float M = Tree<MP>::max(z);
#pragma unroll
                    for (int k = 0; k < MP; ++k) z[k] = ex2(z[k] - M);
                    const float w = om[j] * rcp(Tree<MP>::sum(z));
                    float gsum = 0.f, xe = 0.f;
#pragma unroll
                    for (int k = 0; k < MP; ++k) {
                        const float rho = (k < m) ? ex2(seg[q * MP + k] - gp[k]) : 0.f;
                        const float ekk = (k < m - 1) ? a.e[k] : 0.f;
                        const float x = z[k] * w * rho;
                        const float gx = rg[j] * ekk * x * a.inv_eps;
                        cb[j][k] = -gx;
                        gsum += gx;
                        acc[k] += gx;
                        xe = fmaf(ekk, x, xe);
                    }
                    fb0[j] = gsum;
                    const int i = tm.lt + j * tm.L;
                    if (a.dr && active && i < I)
                        a.dr[u * I + i] = (float)(a.gF / a.imp[i]) * xe;
                }
                team_sum<MP>(acc, tm, red, par);
                par ^= 1;
#pragma unroll
                for (int k = 0; k < MP; ++k) gbar[k] = acc[k];
            }

            // reverse of iteration t
            float gh[MP];
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const float ib = (k == m - 1) ? invbd : 1.0f;
                gh[k] = (k < m) ? gbar[k] * ex2(seg[q * MP + k] - gp[k]) * ib : 0.f;
            }
#pragma unroll
            for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                float z[MP], zg[MP];
#pragma unroll
                for (int k = 0; k < MP; ++k) z[k] = fmaf(c[j][k], a.c2, gp[k]);
                const float M = Tree<MP>::max(z);
#pragma unroll
                for (int k = 0; k < MP; ++k) {
                    z[k] = ex2(z[k] - M);
                    zg[k] = z[k] * gh[k];
                }
                const float w = om[j] * rcp(Tree<MP>::sum(z));
                const float d = Tree<MP>::sum(zg);
                const float fb = (t == a.T ? fb0[j] : 0.f) - w * d;
                const float aa = w * fb;
#pragma unroll
                for (int k = 0; k < MP; ++k) {
                    cb[j][k] = fmaf(z[k], fmaf(w, gh[k], aa), cb[j][k]);
                    acc[k] = fmaf(z[k], aa, acc[k]);
                }
            }
            team_sum<MP>(acc, tm, red, par);
            par ^= 1;
#pragma unroll
            for (int k = 0; k < MP; ++k) gbar[k] = -acc[k];
        }
    }

    // epilogue: write gF * dF/dC, or apply the ascent step to C in place
    if (!active) return;
    float bc1 = 1.f, bc2 = 1.f;
    if (a.Cw && a.rule == 0) {
        const int64_t st = a.step_ptr ? *a.step_ptr : a.step_const;
        bc1 = (float)(1.0 - pow((double)a.b1, (double)st));
        bc2 = (float)(1.0 - pow((double)a.b2, (double)st));
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (i >= I) continue;
        const int64_t base = (u * I + i) * (int64_t)m;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            if (k >= m) continue;
            const float g = cb[j][k];
            if (a.dC) a.dC[base + k] = g;
            if (a.Cw) {
                if (a.rule == 0) {
                    const float gl = -g;
                    const float mo = a.b1 * a.mom[base + k] + (1.f - a.b1) * gl;
                    const float ve = a.b2 * a.vel[base + k] + (1.f - a.b2) * gl * gl;
                    a.mom[base + k] = mo;
                    a.vel[base + k] = ve;
                    a.Cw[base + k] = c[j][k] - a.lr * (mo / bc1) / (sqrtf(ve / bc2) + a.aeps);
                } else {
                    a.Cw[base + k] = c[j][k] + a.lr * g;
                }
            }
        }
    }
}

template <int MP, int R, int LB>
__global__ __launch_bounds__(LB) void k_bwd(BwdArgs a) {
    extern __shared__ float smem[];
    bwd_body<MP, R>(a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

// ---------------------------------------------------------------------------
// Persistent batched kernels: every block repeatedly takes the next work item
// (instance, first consumer) from a global counter and runs the same team
// body on it, until the list is exhausted.  Items are ordered longest first.
template <int MP, int R, int LB>
__global__ __launch_bounds__(LB) void k_bfwd(const FwdArgs* __restrict__ descs,
                                             const BatchItem* __restrict__ items, int n_items,
                                             unsigned* counter) {
    extern __shared__ float smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        const FwdArgs a = descs[bi.inst];
        fwd_body<MP, R>(a, bi.u0, smem);
    }
}

template <int MP, int R, int LB>
__global__ __launch_bounds__(LB) void k_bbwd(const BwdArgs* __restrict__ descs,
                                             const BatchItem* __restrict__ items, int n_items,
                                             unsigned* counter) {
    extern __shared__ float smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        const BwdArgs a = descs[bi.inst];
        bwd_body<MP, R>(a, bi.u0, smem);
    }
}

template <int MP, int R, int LB>
void launch_bfwd(const FwdArgs* d, const BatchItem* it, int n, unsigned* ctr, int grid, int block,
                 size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bfwd<MP, R, LB>), dim3(grid), dim3(block), lds, s, d, it, n, ctr);
}
template <int MP, int R, int LB>
void launch_bbwd(const BwdArgs* d, const BatchItem* it, int n, unsigned* ctr, int grid, int block,
                 size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bbwd<MP, R, LB>), dim3(grid), dim3(block), lds, s, d, it, n, ctr);
}
template <int MP, int R, int LB>
int occupancy_bfwd(int block, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_bfwd<MP, R, LB>, block, lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
template <int MP, int R, int LB>
int occupancy_bbwd(int block, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_bbwd<MP, R, LB>, block, lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int MP, int R, int LB>
void launch_fwd(const FwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd<MP, R, LB>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB>
void launch_bwd(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd<MP, R, LB>), dim3(grid), dim3(block), lds, s, a);
}

template <int R, int LB>
constexpr FusedEntry entry() {
    return FusedEntry{FR_MP,
                      R,
                      LB,
                      &launch_fwd<FR_MP, R, LB>,
                      &launch_bwd<FR_MP, R, LB>,
                      &launch_bfwd<FR_MP, R, LB>,
                      &launch_bbwd<FR_MP, R, LB>,
                      &occupancy_bfwd<FR_MP, R, LB>,
                      &occupancy_bbwd<FR_MP, R, LB>};
}

// Rows per lane instantiated for this column class: the register-resident
// plan share R * MP stays within 128 floats per lane.
#define FR_ROWS_OK(R) ((R) * FR_MP <= 128)

const FusedEntry kEntries[] = {
    entry<1, 256>(),
#if FR_ROWS_OK(2)
    entry<2, 256>(),
#endif
#if FR_ROWS_OK(3)
    entry<3, 256>(),
#endif
#if FR_ROWS_OK(4)
    entry<4, 256>(),
#endif
#if FR_ROWS_OK(6)
    entry<6, 256>(),
#endif
#if FR_ROWS_OK(8)
    entry<8, 256>(),
#endif
    entry<1, 1024>(),
#if FR_ROWS_OK(2)
    entry<2, 1024>(),
#endif
};

}  // namespace

#define FR_CAT2(a, b) a##b
#define FR_CAT(a, b) FR_CAT2(a, b)
const FusedEntry* FR_CAT(fused_entries_, FR_MP)(int* n) {
    *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
    return kEntries;
}

}  // namespace fr
