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
// lane-local; the column half-step needs the sum over the team's rows.
//
// Arithmetic.  Log-domain, base 2: with gamma_k = g_k / (eps ln 2) and the
// scaled cost a_ik = -c_ik / (eps ln 2) - o_i, one iteration is
//   P_ik   = 2^(a_ik + gamma_k) / s_i,  s_i = sum_k 2^(a_ik + gamma_k)   (row softmax)
//   sig_k  = sum_i P_ik
//   gamma_k += log2 b_k - log2 sig_k        (b = 1 ... 1, I-m+1)
// which is the textbook pair of LSE half-steps with a single exponential per
// cell.  The plan is X_ik = 2^(a_ik + gamma^T_k + phi_i), phi_i = -log2 s_i
// from the last row half-step.
//
// Scaling form (k_fwds, k_bwds; see fwds_body and bwds_body).  The same
// iterates on a register-resident kernel 2^(a + gamma_ref + phi_ref) and
// scalings u, v (or, in the reverse sweep, w = 2^(gamma^{t-1} - gamma_ref)):
// multiply-adds per cell, exponentials only when the scalings leave range and
// the kernel is rebuilt from C.
//
// Row centring.  A constant added to a row of the costs leaves every P and X
// unchanged (the row softmax absorbs it), so the registers hold each row of
// scaled costs minus an offset o_i chosen to keep 2^(a + gamma) in range: the
// row maximum at load, and again whenever a row's sum s_i leaves
// [2^-16, 2^16] (or is not finite), when the row is re-centred on its current
// maximum of a + gamma and redone.  The row potential in cost units is then
// (phi_i - o_i) eps ln 2.
//
// Column sums.  Teams narrower than a wave all-reduce every column with DPP
// row butterflies and the gfx950 row swaps.  Teams of whole waves use a
// reduce-scatter instead: v_permlane32_swap and v_permlane16_swap each halve
// the columns a lane carries (columns are taken in chunks of 16), DPP row
// butterflies finish the sums inside 16-lane rows, and then each lane owns at
// most one column.  The owner updates that column's potential and v_readlane
// broadcasts the potentials as wave-uniform (scalar) operands.  Teams of
// several waves add the per-wave totals through LDS.
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
//
// Register budget.  Kernels whose per-lane state (costs, cost adjoints and one
// row of exponentials) would not fit the registers of their launch bound
// recompute the exponentials in a second pass instead of keeping them
// ("recompute" variants): one pass for the row sums, one that produces the
// column partials chunk by chunk.
#include <type_traits>

#include "fr_device.h"
#include "fr_internal.h"

#ifndef FR_MP
#error "compile with -DFR_MP=<padded column count>"
#endif

namespace fr {
namespace {

constexpr float kShiftLo = 1.0f / 65536.0f;
constexpr float kShiftHi = 65536.0f;
// Floor of a column sum before its logarithm: an empty (padded) column keeps
// its potential kNeg, since kNeg + 126 rounds back to kNeg.
constexpr float kTiny = 1.17549435e-38f;

// x, hidden from the optimiser.  Used so that a second pass over a row does
// not reuse (and keep live) the first pass's products, and so that per-column
// conditions after the iteration loop are formed there instead of being kept
// live through it as lane masks.
__device__ __forceinline__ float opaque(float x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ int opaque_u(int x) {
    asm volatile("" : "+s"(x));
    return x;
}

struct Team {
    int L;      // lanes per consumer
    int lt;     // lane within the team
    int lw;     // lane within the wave
    int wt;     // wave within the team
    int W;      // waves per team
    int team;   // team within the block
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
    t.multi = L > 64;
    return t;
}

// ---------------------------------------------------------------------------
// Reduce-scatter layout of a wave.  Chunk ch covers columns [16 ch, 16 ch + n).
// The 32-lane swap leaves columns k0 + [0, H1) in the low half and
// k0 + H1 + [0, n - H1) in the high half; the 16-lane swap splits each half
// at H2, so 16-lane row rho keeps H2 (even rho) or H1 - H2 (odd rho) columns,
// in slots q0 .. q0 + H2 - 1 of the row.
struct ChunkInfo {
    int k0, n, H1, H2, q0;
};

constexpr int n_chunks(int MP) { return (MP + 15) / 16; }

constexpr ChunkInfo chunk_info(int MP, int ch) {
    ChunkInfo c{0, 0, 0, 0, 0};
    int q0 = 0;
    for (int i = 0; i <= ch; ++i) {
        const int k0 = 16 * i;
        const int n = (MP - k0) < 16 ? (MP - k0) : 16;
        const int H1 = (n + 1) / 2;
        const int H2 = (H1 + 1) / 2;
        c = ChunkInfo{k0, n, H1, H2, q0};
        q0 += H2;
    }
    return c;
}

constexpr int n_slots(int MP) {
    return chunk_info(MP, n_chunks(MP) - 1).q0 + chunk_info(MP, n_chunks(MP) - 1).H2;
}
static_assert(n_slots(64) <= 16, "one slot per lane of a 16-lane row");

// Lane of the wave that owns column k after the reduce-scatter.
constexpr int lane_of(int MP, int k) {
    const ChunkInfo c = chunk_info(MP, k / 16);
    const int r = k - c.k0;
    if (r < c.H1) return r < c.H2 ? c.q0 + r : 16 + c.q0 + (r - c.H2);
    const int s = r - c.H1;
    return s < c.H2 ? 32 + c.q0 + s : 48 + c.q0 + (s - c.H2);
}

// Column owned by lane `lane` of a wave (-1 if none); inverse of lane_of.
template <int MP>
__device__ __forceinline__ int owned_col(int lane) {
    const int slot = lane & 15;
    const bool hi = lane >= 32, odd = (lane >> 4) & 1;
    int col = -1;
#pragma unroll
    for (int ch = 0; ch < n_chunks(MP); ++ch) {
        const ChunkInfo c = chunk_info(MP, ch);
        const int j = slot - c.q0;
        if (j >= 0 && j < c.H2) {
            const int r = (hi ? c.H1 : 0) + (odd ? c.H2 : 0) + j;
            const bool ok = (!odd || j < c.H1 - c.H2) && r < c.n;
            col = ok ? c.k0 + r : -1;
        }
    }
    return col;
}

template <int MP, int CH = 0, class F>
__device__ __forceinline__ void for_chunks(F&& f) {
    if constexpr (CH < n_chunks(MP)) {
        f(std::integral_constant<int, CH>{});
        for_chunks<MP, CH + 1>(f);
    }
}

// Reduce-scatter of chunk CH: v holds the lane's partials of the chunk's n
// columns; the two row swaps leave the 4-lane sums in q[q0 .. q0 + H2).
template <int MP, int CH>
__device__ __forceinline__ void scatter_chunk(const float* v, float (&q)[n_slots(MP)]) {
    constexpr ChunkInfo c = chunk_info(MP, CH);
    unsigned x[c.H1], y[c.H1];
#pragma unroll
    for (int j = 0; j < c.H1; ++j) {
        x[j] = __builtin_bit_cast(unsigned, v[j]);
        y[j] = (j + c.H1 < c.n) ? __builtin_bit_cast(unsigned, v[j + c.H1]) : 0u;
    }
    swap32_batch<c.H1>(x, y);
    float h[c.H1];
#pragma unroll
    for (int j = 0; j < c.H1; ++j)
        h[j] = __builtin_bit_cast(float, x[j]) + __builtin_bit_cast(float, y[j]);
    unsigned x2[c.H2], y2[c.H2];
#pragma unroll
    for (int j = 0; j < c.H2; ++j) {
        x2[j] = __builtin_bit_cast(unsigned, h[j]);
        y2[j] = (j + c.H2 < c.H1) ? __builtin_bit_cast(unsigned, h[j + c.H2]) : 0u;
    }
    swap16_batch<c.H2>(x2, y2);
#pragma unroll
    for (int j = 0; j < c.H2; ++j)
        q[c.q0 + j] = __builtin_bit_cast(float, x2[j]) + __builtin_bit_cast(float, y2[j]);
}

template <int MP>
__device__ __forceinline__ void scatter_all(const float (&acc)[MP], float (&q)[n_slots(MP)]) {
    __builtin_amdgcn_sched_barrier(0);
    for_chunks<MP>([&](auto ch) {
        constexpr int CH = decltype(ch)::value;
        scatter_chunk<MP, CH>(acc + 16 * CH, q);
    });
    __builtin_amdgcn_sched_barrier(0);
}

// Team total of the lane's own column from the scattered wave partials q
// (every wave of the team ends with the same value, summed in wave order).
template <int MP>
__device__ __forceinline__ float wide_total(float (&q)[n_slots(MP)], const Team& tm, int col,
                                            float* red, int par) {
    constexpr int Q = n_slots(MP);
    group_allreduce<Q>(q, 16);
    float tot = pick_lane<Q>(q, tm.lw & 15);
    if (tm.multi) {
        float* buf = red + par * (tm.W * MP);
        if (col >= 0) buf[tm.wt * MP + col] = tot;
        __syncthreads();
        tot = 0.f;
        if (col >= 0)
            for (int w = 0; w < tm.W; ++w) tot += buf[w * MP + col];
    }
    return tot;
}

// Broadcast of the owners' values: v[k] = x of lane lane_of(k), as scalars.
template <int MP, int K = 0>
__device__ __forceinline__ void spread_owned(float x, float (&v)[MP]) {
    if constexpr (K < MP) {
        v[K] = lane_value<lane_of(MP, K)>(x);
        spread_owned<MP, K + 1>(x, v);
    }
}

// ---------------------------------------------------------------------------
// Re-centres a row of scaled costs on its current maximum of a + gam if
// `need`; called by the whole wave (rows that do not need it subtract 0), so
// that the rare re-centring stays outside divergent control flow.
template <int MP>
__device__ __forceinline__ void recentre(float (&a)[MP], const float (&gam)[MP], float& off,
                                         bool need) {
    const float one = opaque(1.f);
    float mx[4] = {kNeg, kNeg, kNeg, kNeg};
#pragma unroll
    for (int k = 0; k < MP; ++k) mx[k & 3] = fmaxf(mx[k & 3], fmaf(a[k], one, gam[k]));
    const float M = need ? fmaxf(fmaxf(mx[0], mx[1]), fmaxf(mx[2], mx[3])) : 0.f;
#pragma unroll
    for (int k = 0; k < MP; ++k) a[k] -= M;
    off += M;
}

__device__ __forceinline__ bool in_range(float s) { return s >= kShiftLo && s <= kShiftHi; }

// True on every lane if any lane of the wave has `bad` set.
__device__ __forceinline__ bool wave_any(bool bad) { return __builtin_amdgcn_ballot_w64(bad) != 0; }

// Exponentials of one row: e_k = 2^(a_k + gam_k), s = sum_k e_k; the row is
// re-centred first if the sum leaves range.
template <int MP>
__device__ __forceinline__ void row_exp(float (&a)[MP], const float (&gam)[MP], float (&e)[MP],
                                        float& s, float& off) {
#pragma unroll
    for (int k = 0; k < MP; ++k) e[k] = ex2(a[k] + gam[k]);
    s = Tree<MP>::sum(e);
    const bool bad = !in_range(s);
    if (wave_any(bad)) {
        recentre<MP>(a, gam, off, bad);
        const float one = opaque(1.f);
#pragma unroll
        for (int k = 0; k < MP; ++k) e[k] = ex2(fmaf(a[k], one, gam[k]));
        s = Tree<MP>::sum(e);
    }
}

// s = sum_k e_k and, if GH, d = sum_k e_k gh_k, without keeping the
// exponentials (e_k = 2^(a_k one + gam_k); one is 1, passed opaque so that
// separate passes do not share their products).  Four partial sums shorten
// the dependency chains.
template <int MP, bool GH, bool SHIFT = false>
__device__ __forceinline__ void row_sums(const float (&a)[MP], const float (&gam)[MP],
                                         const float (&gh)[MP], float one, float& s, float& d,
                                         float sh = 0.f) {
    float ps[4] = {0.f, 0.f, 0.f, 0.f}, pd[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const float z = fmaf(a[k], one, gam[k]);
        const float e = ex2(SHIFT ? z - sh : z);
        ps[k & 3] += e;
        if (GH) pd[k & 3] = fmaf(e, gh[k], pd[k & 3]);
    }
    s = (ps[0] + ps[1]) + (ps[2] + ps[3]);
    d = (pd[0] + pd[1]) + (pd[2] + pd[3]);
}

template <int MP, bool GH>
__device__ __forceinline__ void row_stats(float (&a)[MP], const float (&gam)[MP],
                                          const float (&gh)[MP], float& s, float& d, float& off) {
    row_sums<MP, GH>(a, gam, gh, 1.f, s, d);
    const bool bad = !in_range(s);
    if (wave_any(bad)) {
        recentre<MP>(a, gam, off, bad);
        row_sums<MP, GH>(a, gam, gh, opaque(1.f), s, d);
    }
}

// Variant that leaves the costs alone and shifts instead: e_k =
// 2^(a_k + gam_k - sh), with sh kept per row across calls and reset to the
// row's current maximum when the sum leaves range.  Used where the registers
// cannot afford rewriting the costs (the recompute backward).
template <int MP, bool GH>
__device__ __forceinline__ void row_stats_shift(const float (&a)[MP], const float (&gam)[MP],
                                                const float (&gh)[MP], float& s, float& d,
                                                float& sh) {
    row_sums<MP, GH, true>(a, gam, gh, 1.f, s, d, sh);
    const bool bad = !in_range(s);
    if (wave_any(bad)) {
        const float one = opaque(1.f);
        float mx[4] = {kNeg, kNeg, kNeg, kNeg};
#pragma unroll
        for (int k = 0; k < MP; ++k) mx[k & 3] = fmaxf(mx[k & 3], fmaf(a[k], one, gam[k]));
        if (bad) sh = fmaxf(fmaxf(mx[0], mx[1]), fmaxf(mx[2], mx[3]));
        row_sums<MP, GH, true>(a, gam, gh, opaque(1.f), s, d, sh);
    }
}

// ---------------------------------------------------------------------------
// Column state of a team: the potentials gam (registers of every lane for
// narrow teams; wave-uniform scalars for wide ones, with the owner lane's
// copy gd) and the per-column constants.
template <int MP, bool WIDE>
struct Cols;

template <int MP>
struct Cols<MP, false> {
    float lb[MP];    // log2 b_k
    float ib[MP];    // 1 / b_k
    __device__ __forceinline__ void init(const Team&, int m, float lbd, float ibd, float (&gam)[MP]) {
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            gam[k] = (k < m) ? 0.f : kNeg;
            lb[k] = (k == m - 1) ? lbd : 0.f;
            ib[k] = (k == m - 1) ? ibd : 1.f;
        }
    }
};

template <int MP>
struct Cols<MP, true> {
    int col;      // column this lane owns after the reduce-scatter (-1: none)
    bool live;    // col < m
    float lbc;    // log2 b_col
    float ibc;    // 1 / b_col
    float gd;     // gamma_col
    __device__ __forceinline__ void init(const Team& tm, int m, float lbd, float ibd, float (&gam)[MP]) {
        col = owned_col<MP>(tm.lw);
        live = col >= 0 && col < m;
        lbc = (col == m - 1) ? lbd : 0.f;
        ibc = (col == m - 1) ? ibd : 1.f;
        gd = live ? 0.f : kNeg;
        spread_owned<MP>(gd, gam);
    }
};

// Stores the MP column potentials of a team (kNeg on padding) at dst:
// history or LDS segment.
template <int MP, bool WIDE>
__device__ __forceinline__ void put_gamma(float* dst, const float (&gam)[MP],
                                          const Cols<MP, WIDE>& cs, const Team& tm) {
    if constexpr (WIDE) {
        if (tm.wt == 0 && cs.col >= 0) dst[cs.col] = cs.gd;
    } else {
        if (tm.lt == 0) {
#pragma unroll
            for (int k = 0; k < MP; ++k) dst[k] = gam[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Forward row half-step.  Keeps one row of exponentials: acc gets the lane's
// column partials sum_i P_ik; S the rows' log2 s_i.
template <int MP, int R>
__device__ __forceinline__ void row_pass(float (&c)[R][MP], const float (&om)[R],
                                         const float (&gam)[MP], float (&acc)[MP], float (&S)[R],
                                         float (&off)[R]) {
#pragma unroll
    for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float e[MP], s;
        row_exp<MP>(c[j], gam, e, s, off[j]);
        const float w = om[j] * rcp(s);
#pragma unroll
        for (int k = 0; k < MP; ++k) acc[k] = fmaf(e[k], w, acc[k]);
        S[j] = lg2(s);
    }
}

// Recompute variant (wide teams): row sums first, then the column partials
// chunk by chunk, each chunk scattered as soon as it is complete.
// With SHIFT the costs are left alone and sh (per row, kept across calls)
// shifts the exponents instead of re-centring (used inside the recompute
// backward, whose registers cannot afford rewriting the costs).
template <int MP, int R, bool SHIFT = false>
__device__ __forceinline__ void row_pass_recomp(float (&c)[R][MP], const float (&om)[R],
                                                const float (&gam)[MP], float (&q)[n_slots(MP)],
                                                float (&S)[R], float (&off)[R]) {
    float w[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float s, d;
        if constexpr (SHIFT)
            row_stats_shift<MP, false>(c[j], gam, gam, s, d, off[j]);
        else
            row_stats<MP, false>(c[j], gam, gam, s, d, off[j]);
        w[j] = om[j] * rcp(s);
        S[j] = lg2(s);
    }
    __builtin_amdgcn_sched_barrier(0);
    const float one = opaque(1.f);
    for_chunks<MP>([&](auto ch) {
        constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
        float v[ci.n];
#pragma unroll
        for (int kk = 0; kk < ci.n; ++kk) v[kk] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) {
                const int k = ci.k0 + kk;
                const float z = fmaf(c[j][k], one, gam[k]);
                v[kk] = fmaf(ex2(SHIFT ? z - off[j] : z), w[j], v[kk]);
            }
        }
        scatter_chunk<MP, decltype(ch)::value>(v, q);
    });
    __builtin_amdgcn_sched_barrier(0);
}

// Column half-step: gamma_k += log2 b_k - log2 sig_k.  With CHECK, returns
// whether no potential moved by more than tol (the team-uniform convergence
// test of the warm-started form).
template <int MP, bool CHECK>
__device__ __forceinline__ bool col_update(float (&acc)[MP], float (&gam)[MP],
                                           const Cols<MP, false>& cs, const Team& tm, float tol) {
    group_allreduce<MP>(acc, tm.L);
    float dmax = 0.f;
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const float d = cs.lb[k] - lg2(fmaxf(acc[k], kTiny));
        if (CHECK && gam[k] > 0.5f * kNeg) dmax = fmaxf(dmax, fabsf(d));   // real columns
        gam[k] += d;
    }
    return dmax <= tol;
}

template <int MP, bool CHECK>
__device__ __forceinline__ bool col_update_wide(float (&q)[n_slots(MP)], float (&gam)[MP],
                                                Cols<MP, true>& cs, const Team& tm, float* red,
                                                int par, float tol) {
    const float tot = wide_total<MP>(q, tm, cs.col, red, par);
    const float d = cs.lbc - lg2(tot);
    if (cs.live) cs.gd += d;
    spread_owned<MP>(cs.gd, gam);
    return CHECK ? !wave_any(cs.live && fabsf(d) > tol) : true;
}

// One forward Sinkhorn iteration of a team.
template <int MP, int R, bool WIDE, bool RECOMP, bool SHIFT = false, bool CHECK = false>
__device__ __forceinline__ bool fwd_iter(float (&c)[R][MP], const float (&om)[R],
                                         float (&gam)[MP], float (&S)[R], float (&off)[R],
                                         Cols<MP, WIDE>& cs, int m, const Team& tm, float* red,
                                         int par, float tol = 0.f) {
    (void)m;
    if constexpr (!WIDE) {
        float acc[MP];
        row_pass<MP, R>(c, om, gam, acc, S, off);
        return col_update<MP, CHECK>(acc, gam, cs, tm, tol);
    } else {
        float q[n_slots(MP)];
        if constexpr (RECOMP) {
            row_pass_recomp<MP, R, SHIFT>(c, om, gam, q, S, off);
        } else {
            float acc[MP];
            row_pass<MP, R>(c, om, gam, acc, S, off);
            scatter_all<MP>(acc, q);
        }
        return col_update_wide<MP, CHECK>(q, gam, cs, tm, red, par, tol);
    }
}

// Loads the lane's rows of C as centred scaled costs a_ik = c_ik c2 - o_i,
// o_i = max_k c_ik c2 (padded columns repeat the last cost; their potential
// kNeg zeroes them).
template <int MP, int R>
__device__ __forceinline__ void load_costs(const float* C, int64_t u, bool active, const Team& tm,
                                           int I, int m, float c2, float (&c)[R][MP],
                                           float (&om)[R], float (&off)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        const bool valid = active && i < I;
        om[j] = valid ? 1.f : 0.f;
        const float* src = C + (u * I + i) * (int64_t)m;
        float t[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            c[j][k] = valid ? src[k < m ? k : m - 1] : 0.f;
            t[k] = c[j][k] * c2;
        }
        const float M = Tree<MP>::max(t);
#pragma unroll
        for (int k = 0; k < MP; ++k) c[j][k] = fmaf(c[j][k], c2, -M);
        off[j] = M;
    }
}

// ---------------------------------------------------------------------------
// Forward for the teams of one block: team q of the block owns consumer
// u_first + q.
template <int MP, int R, bool WIDE, bool RECOMP, bool CONV = false>
__device__ __forceinline__ void fwd_body(const FwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int64_t u = u_first + tm.team;
    // lanes past the last whole team of the block own no consumer
    const bool active = tm.team < (int)(blockDim.x / a.L) && u < a.U;
    const int I = a.I, m = a.m;
    float* red = smem + tm.team * (2 * tm.W * MP);

    float c[R][MP], om[R], off[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, a.c2, c, om, off);

    float gam[MP];
    Cols<MP, WIDE> cs;
    cs.init(tm, m, lg2((float)(I - m + 1)), 1.0f / (float)(I - m + 1), gam);
    if (CONV && a.gw) {   // warm start from the previous potentials
        const float* gs = a.gw + (active ? u : 0) * (int64_t)a.hs;
        if constexpr (WIDE) {
            cs.gd = (active && cs.col >= 0) ? gs[cs.col] : cs.gd;
            spread_owned<MP>(cs.gd, gam);
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) gam[k] = active ? gs[k] : gam[k];
        }
    }
    float* hist = (a.hist != nullptr && active) ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    if (hist) put_gamma<MP, WIDE>(hist, gam, cs, tm);

    float S[R];
#pragma unroll
    for (int j = 0; j < R; ++j) S[j] = 0.f;
    int used = a.T;
    if constexpr (CONV) {
        // converged-map form: stop once no potential moves by more than tol
        for (int t = 1; t <= a.T; ++t) {
            if (fwd_iter<MP, R, WIDE, RECOMP, false, true>(c, om, gam, S, off, cs, m, tm, red,
                                                           t & 1, a.tol)) {
                used = t;
                break;
            }
        }
    } else {
        for (int t = 1; t <= a.T; ++t) {
            fwd_iter<MP, R, WIDE, RECOMP>(c, om, gam, S, off, cs, m, tm, red, t & 1);
            if (hist) {
                if (t % a.K == 0)
                    put_gamma<MP, WIDE>(hist + (int64_t)(t / a.K) * a.hs, gam, cs, tm);
                else if (t == a.T)
                    put_gamma<MP, WIDE>(hist + (int64_t)(a.nck - 1) * a.hs, gam, cs, tm);
            }
        }
    }
    if (CONV && active) {
        if (a.gw) put_gamma<MP, WIDE>(a.gw + u * (int64_t)a.hs, gam, cs, tm);
        if (a.iters && tm.lt == 0) atomicAdd((unsigned long long*)a.iters, (unsigned long long)used);
    }
    (void)used;

    const int mo = opaque_u(m);
    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < mo - 1) ? a.e[k] : 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (!(active && i < I)) continue;
        const float phi = -S[j];   // row potential of the centred costs
        const int64_t row = u * I + i;
        float yy = 0.f;
        if (a.X && a.x_bf16) {
            uint16_t* dst = (uint16_t*)a.X + row * m;
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const float x = ex2((c[j][k] + gam[k]) + phi);
                yy = fmaf(ek[k], x, yy);
                if (k < mo) dst[k] = to_bf16(x);
            }
        } else if (a.X) {
            float* dst = (float*)a.X + row * m;
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const float x = ex2((c[j][k] + gam[k]) + phi);
                yy = fmaf(ek[k], x, yy);
                if (k < mo) dst[k] = x;
            }
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k)
                yy = fmaf(ek[k], ex2((c[j][k] + gam[k]) + phi), yy);
        }
        if (a.y) a.y[row] = a.r[row] * yy;
        if (a.pot) a.pot[u * (int64_t)(I + m) + i] = (phi - off[j]) * a.eps_ln2;
        if (a.phi) a.phi[row] = phi - off[j];
    }
    if (a.pot && active && tm.lt == 0) {
#pragma unroll
        for (int k = 0; k < MP; ++k)
            if (k < mo) a.pot[u * (int64_t)(I + m) + I + k] = gam[k] * a.eps_ln2;
    }
}

// ---------------------------------------------------------------------------
// Scaling form of the forward: the matrix-scaling iteration of Sinkhorn (the
// form of the algorithm Section 3 cites), stabilised by absorbing the
// scalings into log-domain potentials.  The registers hold the kernel
//   Kt_ik = 2^(a_ik + gam_k + ph_i)
// for absorbed potentials (gam, ph), and an iteration updates scalings only:
//   u_i = 1 / sum_k Kt_ik v_k,      v_k = b_k / sum_i Kt_ik u_i,
// the same iterates as the log-domain form (P^t = Kt diag(v^{t-1}) scaled by
// u^t, gamma^t = gam + log2 v^t) at two multiply-adds per cell and no
// exponential.  When a column scaling leaves [2^-32, 2^32] (or every
// `absorb` iterations, if set), the scalings move into the potentials and Kt
// is rebuilt from the costs in HBM: the log-domain step, one exponential per
// cell.  Padded columns have b = 0, so their scaling stays 0 and they add
// nothing to the row sums.
constexpr float kScaleHi = 4294967296.0f;           // 2^32
constexpr float kScaleLo = 1.0f / 4294967296.0f;    // 2^-32

// Kt of the lane's rows from the costs in HBM: a = c c2 - off (the centring
// offsets of load_costs), Kt = 2^(a + gam + ph).
template <int MP, int R>
__device__ __forceinline__ void build_kernel(const float* C, int64_t u, const Team& tm, int I,
                                             int m, float c2, const float (&om)[R],
                                             const float (&off)[R], const float (&gam)[MP],
                                             const float (&ph)[R], float (&kt)[R][MP]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        const bool valid = om[j] > 0.f;
        const float* src = C + (u * I + (valid ? i : 0)) * (int64_t)m;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const float c = valid ? src[k < m ? k : m - 1] : 0.f;
            kt[j][k] = ex2((fmaf(c, c2, -off[j]) + gam[k]) + ph[j]);
        }
    }
}

// Row half-step of the scaling form: u_j = 1 / sum_k Kt_jk v_k.
template <int MP, int R>
__device__ __forceinline__ void scale_rows(const float (&kt)[R][MP], const float (&v)[MP],
                                           float (&u)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float ps[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MP; ++k) ps[k & 3] = fmaf(kt[j][k], v[k], ps[k & 3]);
        u[j] = rcp((ps[0] + ps[1]) + (ps[2] + ps[3]));
    }
}

template <int MP, int R, bool WIDE>
__device__ __forceinline__ void fwds_body(const FwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int64_t u = u_first + tm.team;
    const bool active = tm.team < (int)(blockDim.x / a.L) && u < a.U;
    const int I = a.I, m = a.m;
    float* red = smem + tm.team * (2 * tm.W * MP);
    const float bd = (float)(I - m + 1);

    float kt[R][MP], om[R], off[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, a.c2, kt, om, off);

    float gam[MP], v[MP], ph[R], us[R];
    Cols<MP, WIDE> cs;
    cs.init(tm, m, lg2(bd), 1.0f / bd, gam);
    [[maybe_unused]] float bk[MP];
    [[maybe_unused]] float vd = 0.f, bc = 0.f;
    if constexpr (WIDE) {
        bc = cs.live ? rcp(cs.ibc) : 0.f;
        vd = cs.live ? 1.f : 0.f;
        spread_owned<MP>(vd, v);
    } else {
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            bk[k] = (k < m) ? ((k == m - 1) ? bd : 1.f) : 0.f;
            v[k] = fminf(bk[k], 1.f);
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        ph[j] = 0.f;
        us[j] = 1.f;
#pragma unroll
        for (int k = 0; k < MP; ++k) kt[j][k] = ex2(kt[j][k] + gam[k]);
    }

    float* hist = (a.hist != nullptr && active) ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    // base-2 column potentials gamma = gam + log2 v (kNeg on padding)
    auto put_hist = [&](float* dst) {
        if constexpr (WIDE) {
            if (tm.wt == 0 && cs.col >= 0) dst[cs.col] = fmaxf(cs.gd + lg2(vd), kNeg);
        } else {
            if (tm.lt == 0) {
#pragma unroll
                for (int k = 0; k < MP; ++k) dst[k] = fmaxf(gam[k] + lg2(v[k]), kNeg);
            }
        }
    };
    if (hist) put_hist(hist);

    for (int t = 1; t <= a.T; ++t) {
        scale_rows<MP, R>(kt, v, us);
        float w[R];
#pragma unroll
        for (int j = 0; j < R; ++j) w[j] = us[j] * om[j];
        bool bad;
        if constexpr (WIDE) {
            float q[n_slots(MP)];
            __builtin_amdgcn_sched_barrier(0);
            for_chunks<MP>([&](auto ch) {
                constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
                float p[ci.n];
#pragma unroll
                for (int kk = 0; kk < ci.n; ++kk) p[kk] = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
#pragma unroll
                    for (int kk = 0; kk < ci.n; ++kk) p[kk] = fmaf(kt[j][ci.k0 + kk], w[j], p[kk]);
                }
                scatter_chunk<MP, decltype(ch)::value>(p, q);
            });
            __builtin_amdgcn_sched_barrier(0);
            const float tot = wide_total<MP>(q, tm, cs.col, red, t & 1);
            vd = bc * rcp(fmaxf(tot, kTiny));
            bad = wave_any(cs.live && !(vd >= kScaleLo && vd <= kScaleHi));
            spread_owned<MP>(vd, v);
        } else {
            float acc[MP];
#pragma unroll
            for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
            for (int j = 0; j < R; ++j) {
#pragma unroll
                for (int k = 0; k < MP; ++k) acc[k] = fmaf(kt[j][k], w[j], acc[k]);
            }
            group_allreduce<MP>(acc, tm.L);
            float hi = 0.f, lo = 1.f;
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                v[k] = bk[k] * rcp(fmaxf(acc[k], kTiny));
                hi = fmaxf(hi, v[k]);
                lo = fminf(lo, v[k] > 0.f ? v[k] : 1.f);
            }
            bad = wave_any(!(hi <= kScaleHi) || lo < kScaleLo);
        }
        if (bad || (a.absorb > 0 && t % a.absorb == 0)) {
            // move the scalings into the potentials and rebuild Kt (log-domain step)
            if constexpr (WIDE) {
                if (cs.live) cs.gd += lg2(vd);
                vd = cs.live ? 1.f : 0.f;
                spread_owned<MP>(cs.gd, gam);
                spread_owned<MP>(vd, v);
            } else {
#pragma unroll
                for (int k = 0; k < MP; ++k) {
                    gam[k] = (v[k] > 0.f) ? gam[k] + lg2(v[k]) : gam[k];
                    v[k] = fminf(bk[k], 1.f);
                }
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                ph[j] += lg2(us[j]);
                us[j] = 1.f;
            }
            build_kernel<MP, R>(a.C, active ? u : 0, tm, I, m, a.c2, om, off, gam, ph, kt);
        }
        if (hist) {
            if (t % a.K == 0)
                put_hist(hist + (int64_t)(t / a.K) * a.hs);
            else if (t == a.T)
                put_hist(hist + (int64_t)(a.nck - 1) * a.hs);
        }
    }

    const int mo = opaque_u(m);
    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < mo - 1) ? a.e[k] : 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (!(active && i < I)) continue;
        const int64_t row = u * I + i;
        float yy = 0.f;
        if (a.X && a.x_bf16) {
            uint16_t* dst = (uint16_t*)a.X + row * m;
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const float x = (kt[j][k] * v[k]) * us[j];
                yy = fmaf(ek[k], x, yy);
                if (k < mo) dst[k] = to_bf16(x);
            }
        } else if (a.X) {
            float* dst = (float*)a.X + row * m;
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                const float x = (kt[j][k] * v[k]) * us[j];
                yy = fmaf(ek[k], x, yy);
                if (k < mo) dst[k] = x;
            }
        } else {
            // the same products as with X, so the impacts do not depend on it
#pragma unroll
            for (int k = 0; k < MP; ++k) yy = fmaf(ek[k], (kt[j][k] * v[k]) * us[j], yy);
        }
        if (a.y) a.y[row] = a.r[row] * yy;
        const float phi = ph[j] + lg2(us[j]) - off[j];
        if (a.pot) a.pot[u * (int64_t)(I + m) + i] = phi * a.eps_ln2;
        if (a.phi) a.phi[row] = phi;
    }
    if (a.pot && active) {
        if constexpr (WIDE) {
            if (tm.wt == 0 && cs.live) a.pot[u * (int64_t)(I + m) + I + cs.col] = (cs.gd + lg2(vd)) * a.eps_ln2;
        } else if (tm.lt == 0) {
#pragma unroll
            for (int k = 0; k < MP; ++k)
                if (k < mo) a.pot[u * (int64_t)(I + m) + I + k] = (gam[k] + lg2(v[k])) * a.eps_ln2;
        }
    }
}

// ---------------------------------------------------------------------------
// Cost adjoints of a lane's R rows: rows j < R - NL in registers, the last NL
// in LDS, column-major over the team's lanes ((j' MP + k) L + lane), so that
// the 64 lanes of a wave touch consecutive words.  Every lane owns its slots:
// no synchronisation is needed.  NL > 0 is for the wide recompute kernels,
// whose registers cannot hold costs, cost adjoints and a pass's temporaries.
template <int MP, int R, int NL>
struct CostAdj {
    static constexpr int RR = R - NL;
    float reg[RR > 0 ? RR : 1][MP];
    float* lds = nullptr;
    int L = 0, lt = 0;
    __device__ __forceinline__ float& operator()(int j, int k) {
        if (j < RR) return reg[j][k];
        return lds[((j - RR) * MP + k) * L + lt];
    }
};

// The same access to a plain register array of cost adjoints.
template <int MP, int R>
struct ArrAdj {
    float (&a)[R][MP];
    __device__ __forceinline__ float& operator()(int j, int k) { return a[j][k]; }
};

// ---------------------------------------------------------------------------
// Backward pieces.  Reverse of iteration t for the lane's rows: gp = gamma^{t-1},
// gh_k = gbar_k / sig^t_k; cb += P (gh + fbar); the lane's share of
// sum_i P_ik fbar_i goes to acc (or, recompute variant, to the scattered q).
template <int MP, int R, class CB>
__device__ __forceinline__ void rev_pass(float (&c)[R][MP], const float (&om)[R],
                                         const float (&gp)[MP], const float (&gh)[MP],
                                         const float (&fb0)[R], bool first, CB& cb,
                                         float (&acc)[MP], float (&off)[R]) {
#pragma unroll
    for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float e[MP], s;
        row_exp<MP>(c[j], gp, e, s, off[j]);
        float pd[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MP; ++k) pd[k & 3] = fmaf(e[k], gh[k], pd[k & 3]);
        const float d = (pd[0] + pd[1]) + (pd[2] + pd[3]);
        const float w = om[j] * rcp(s);
        const float fb = (first ? fb0[j] : 0.f) - w * d;
        const float aa = w * fb;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            cb(j, k) = fmaf(e[k], fmaf(w, gh[k], aa), cb(j, k));
            acc[k] = fmaf(e[k], aa, acc[k]);
        }
    }
}

// Owner broadcast of the columns [K0, K0 + N): out[kk] = x of the lane that
// owns column K0 + kk, as scalars.
template <int MP, int K0, int N, int KK = 0>
__device__ __forceinline__ void spread_range(float x, float (&out)[N]) {
    if constexpr (KK < N) {
        out[KK] = lane_value<lane_of(MP, K0 + KK)>(x);
        spread_range<MP, K0, N, KK + 1>(x, out);
    }
}

// Reverse of iteration t for the wide recompute variant (registers too few
// for a row of exponentials, so every pass recomputes them under a per-row
// shift sh, as row_stats_shift does).  It never holds a whole row of
// column values: gamma^{t-1} and gh arrive as the owner lanes' values gpd and
// ghd and are broadcast chunk by chunk, once per pass (each broadcast from a
// fresh opaque copy, so that passes do not share them), which leaves only the
// costs and cost adjoints live across the iteration.
template <int MP, int R, class CB>
__device__ __forceinline__ void rev_pass_owned(const float (&c)[R][MP], const float (&om)[R],
                                               float gpd, float ghd, const float (&fb0)[R],
                                               bool first, CB& cb,
                                               float (&q)[n_slots(MP)], float (&sh)[R]) {
    float s[R], d[R];
    auto sums = [&](float one) {
        float ps[R][4], pd[R][4];
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) ps[j][p] = pd[j][p] = 0.f;
        const float gpo = opaque(gpd), gho = opaque(ghd);
        for_chunks<MP>([&](auto ch) {
            constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
            float g[ci.n], h[ci.n];
            spread_range<MP, ci.k0, ci.n>(gpo, g);
            spread_range<MP, ci.k0, ci.n>(gho, h);
#pragma unroll
            for (int j = 0; j < R; ++j) {
#pragma unroll
                for (int kk = 0; kk < ci.n; ++kk) {
                    const int k = ci.k0 + kk;
                    const float e = ex2(fmaf(c[j][k], one, g[kk]) - sh[j]);
                    ps[j][k & 3] += e;
                    pd[j][k & 3] = fmaf(e, h[kk], pd[j][k & 3]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        });
#pragma unroll
        for (int j = 0; j < R; ++j) {
            s[j] = (ps[j][0] + ps[j][1]) + (ps[j][2] + ps[j][3]);
            d[j] = (pd[j][0] + pd[j][1]) + (pd[j][2] + pd[j][3]);
        }
    };
    sums(1.f);
    bool bad[R], anybad = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        bad[j] = !in_range(s[j]);
        anybad |= bad[j];
    }
    if (wave_any(anybad)) {
        // rare: rows whose sum left range shift to their current maximum
        const float one = opaque(1.f);
        float mx[R][4];
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int p = 0; p < 4; ++p) mx[j][p] = kNeg;
        const float gpo = opaque(gpd);
        for_chunks<MP>([&](auto ch) {
            constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
            float g[ci.n];
            spread_range<MP, ci.k0, ci.n>(gpo, g);
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int kk = 0; kk < ci.n; ++kk) {
                    const int k = ci.k0 + kk;
                    mx[j][k & 3] = fmaxf(mx[j][k & 3], fmaf(c[j][k], one, g[kk]));
                }
        });
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (bad[j]) sh[j] = fmaxf(fmaxf(mx[j][0], mx[j][1]), fmaxf(mx[j][2], mx[j][3]));
        sums(opaque(1.f));
    }
    float w[R], aa[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        w[j] = om[j] * rcp(s[j]);
        const float fb = (first ? fb0[j] : 0.f) - w[j] * d[j];
        aa[j] = w[j] * fb;
    }
    __builtin_amdgcn_sched_barrier(0);
    const float one = opaque(1.f);
    const float gpo = opaque(gpd), gho = opaque(ghd);
    for_chunks<MP>([&](auto ch) {
        constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
        float g[ci.n], h[ci.n], v[ci.n];
        spread_range<MP, ci.k0, ci.n>(gpo, g);
        spread_range<MP, ci.k0, ci.n>(gho, h);
#pragma unroll
        for (int kk = 0; kk < ci.n; ++kk) v[kk] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) {
                const int k = ci.k0 + kk;
                const float e = ex2(fmaf(c[j][k], one, g[kk]) - sh[j]);
                cb(j, k) = fmaf(e, fmaf(w[j], h[kk], aa[j]), cb(j, k));
                v[kk] = fmaf(e, aa[j], v[kk]);
            }
        }
        scatter_chunk<MP, decltype(ch)::value>(v, q);
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Start of the reverse sweep (t = T): X = P^T diag(rho), rho_k = b_k / sig^T_k,
// and the adjoints of X = exp((f + g - c)/eps): cb = -G X / eps,
// fb0 = (G X) 1 / eps, acc (or q) = the lane's share of (G X)^T 1 / eps;
// also dr = gF e.X / Imp.  Rows are processed chunk by chunk with the
// exponentials recomputed, so no row of them is kept.
template <int MP, int R, bool WIDE, class CB>
__device__ __forceinline__ void rev_init(const BwdArgs& a, const float (&c)[R][MP],
                                         const float (&om)[R], const float (&gp)[MP],
                                         const float (&rho)[MP], const float (&rg)[R],
                                         float (&fb0)[R], CB& cb,
                                         float (&acc)[WIDE ? 1 : MP], float (&q)[n_slots(MP)],
                                         float (&sh)[R], int64_t u, bool active, const Team& tm) {
    const int m = opaque_u(a.m);
    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < m - 1) ? a.e[k] : 0.f;
    float w[R], xe[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float s, d;
        row_stats_shift<MP, false>(c[j], gp, gp, s, d, sh[j]);
        w[j] = om[j] * rcp(s) * a.inv_eps;
        fb0[j] = 0.f;
        xe[j] = 0.f;
    }
    const float one = opaque(1.f);
    for_chunks<MP>([&](auto ch) {
        constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
        float v[ci.n];
#pragma unroll
        for (int kk = 0; kk < ci.n; ++kk) v[kk] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) {
                const int k = ci.k0 + kk;
                // xs = x / eps, gx = G x / eps
                const float xs = ex2(fmaf(c[j][k], one, gp[k]) - sh[j]) * w[j] * rho[k];
                const float gx = rg[j] * ek[k] * xs;
                cb(j, k) = -gx;
                fb0[j] += gx;
                v[kk] += gx;
                xe[j] = fmaf(ek[k], xs, xe[j]);
            }
        }
        if constexpr (WIDE) {
            scatter_chunk<MP, decltype(ch)::value>(v, q);
        } else {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) acc[ci.k0 + kk] = v[kk];
        }
    });
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (a.dr && active && i < a.I)
            a.dr[u * a.I + i] = (float)(a.gF / a.imp[i]) * (xe[j] / a.inv_eps);
    }
}

// Backward epilogue for the lane's rows: writes gF * dF/dC, or applies Adam /
// ascent to C in place (re-reading C from HBM: the registers hold transformed
// costs).
template <int MP, int R, class CB>
__device__ __forceinline__ void bwd_epilogue(const BwdArgs& a, CB& cb, int64_t u, const Team& tm) {
    const int I = a.I, m = a.m;
    const int mo = opaque_u(m);
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
            if (k >= mo) continue;
            const float g = cb(j, k);
            if (a.dC) a.dC[base + k] = g;
            if (a.Cw) {
                const float craw = a.C[base + k];   // the registers do not hold raw costs
                if (a.rule == 0) {
                    const float gl = -g;
                    const float mo = a.b1 * a.mom[base + k] + (1.f - a.b1) * gl;
                    const float ve = a.b2 * a.vel[base + k] + (1.f - a.b2) * gl * gl;
                    a.mom[base + k] = mo;
                    a.vel[base + k] = ve;
                    a.Cw[base + k] = craw - a.lr * (mo / bc1) / (sqrtf(ve / bc2) + a.aeps);
                } else {
                    a.Cw[base + k] = craw + a.lr * g;
                }
            }
        }
    }
}

// NL: rows of cost adjoints per lane kept in LDS (after the block's segment
// and reduction buffers, NL * MP * L floats per team).
template <int MP, int R, bool WIDE, bool RECOMP, int NL = 0>
__device__ __forceinline__ void bwd_body(const BwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int teams = blockDim.x / a.L;
    const int64_t u = u_first + tm.team;
    const bool active = tm.team < teams && u < a.U;
    const int I = a.I, m = a.m;
    const int BL = (a.K == 1) ? kLoadBlock : a.K;
    float* seg = smem + tm.team * ((BL + 1) * MP);
    float* red = smem + teams * ((BL + 1) * MP) + tm.team * (2 * tm.W * MP);

    float c[R][MP], om[R], off[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, a.c2, c, om, off);

    float rg[R];   // gF r_i / Imp_i, so that G_ik = rg_i e_k
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        rg[j] = (active && i < I) ? (float)(a.gF * (double)a.r[u * I + i] / a.imp[i]) : 0.f;
    }
    float gam[MP];   // recomputed potentials (K > 1 segments)
    Cols<MP, WIDE> cs;
    cs.init(tm, m, lg2((float)(I - m + 1)), 1.0f / (float)(I - m + 1), gam);

    const float* hist = active ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    CostAdj<MP, R, NL> cb;
    if constexpr (NL > 0) {
        cb.lds = smem + teams * ((BL + 1) * MP + 2 * tm.W * MP) + tm.team * (NL * MP * tm.L);
        cb.L = tm.L;
        cb.lt = tm.lt;
    }
    float fb0[R], Sf[R], sh[R], shf[R];
    float gbar[WIDE ? 1 : MP];   // narrow: every column; wide: the owned column
#pragma unroll
    for (int k = 0; k < (WIDE ? 1 : MP); ++k) gbar[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        fb0[j] = 0.f;
        Sf[j] = 0.f;
        sh[j] = 0.f;   // costs are centred at load: start unshifted
        shf[j] = 0.f;
    }

    int par = 0;
    const int nblk = (a.K == 1) ? (a.T + BL - 1) / BL : (a.nck - 1);
    for (int s = nblk - 1; s >= 0; --s) {
        const int t0 = s * BL;
        const int t1 = min(t0 + BL, a.T);
        const int n = t1 - t0;
        __syncthreads();  // the previous block's reads of seg are complete
        if (a.K == 1) {
            for (int idx = tm.lt; idx < (n + 1) * MP; idx += tm.L) {
                const int qq = idx / MP, k = idx - qq * MP;
                seg[idx] = active ? hist[(int64_t)(t0 + qq) * a.hs + k] : 0.f;
            }
        } else {
            // rebuild gamma^{t0} .. gamma^{t1} from the checkpoint
            if constexpr (WIDE) {
                cs.gd = (active && cs.col >= 0) ? hist[(int64_t)s * a.hs + cs.col] : kNeg;
                spread_owned<MP>(cs.gd, gam);
            } else {
#pragma unroll
                for (int k = 0; k < MP; ++k) gam[k] = active ? hist[(int64_t)s * a.hs + k] : kNeg;
            }
            put_gamma<MP, WIDE>(seg, gam, cs, tm);
            for (int qq = 1; qq <= n; ++qq) {
                fwd_iter<MP, R, WIDE, RECOMP, RECOMP>(c, om, gam, Sf, RECOMP ? shf : off, cs, m, tm,
                                                      red, par);
                par ^= 1;
                put_gamma<MP, WIDE>(seg + qq * MP, gam, cs, tm);
            }
        }
        __syncthreads();

        for (int qq = n; qq >= 1; --qq) {
            const int t = t0 + qq;
            const float* sq = seg + qq * MP;        // gamma^t
            const float* sp = seg + (qq - 1) * MP;  // gamma^{t-1}
            if constexpr (WIDE && RECOMP) {
                // column values stay with their owner lanes (rev_pass_owned)
                const float gpd = (cs.col >= 0) ? sp[cs.col] : kNeg;
                if (t == a.T) {
                    float gp[MP], rho[MP];
                    spread_owned<MP>(gpd, gp);
#pragma unroll
                    for (int k = 0; k < MP; ++k) rho[k] = ex2(sq[k] - gp[k]);   // 1 on padding
                    float acc[1];
                    float q[n_slots(MP)];
                    rev_init<MP, R, WIDE>(a, c, om, gp, rho, rg, fb0, cb, acc, q, sh, u, active, tm);
                    gbar[0] = wide_total<MP>(q, tm, cs.col, red, par);
                    par ^= 1;
                }
                const float ghd = cs.live ? gbar[0] * ex2(sq[cs.col] - sp[cs.col]) * cs.ibc : 0.f;
                float q[n_slots(MP)];
                rev_pass_owned<MP, R>(c, om, gpd, ghd, fb0, t == a.T, cb, q, sh);
                gbar[0] = -wide_total<MP>(q, tm, cs.col, red, par);
                par ^= 1;
                continue;
            }
            float gp[MP], gh[MP];
            if constexpr (WIDE) {
                spread_owned<MP>((cs.col >= 0) ? sp[cs.col] : kNeg, gp);
            } else {
#pragma unroll
                for (int k = 0; k < MP; ++k) gp[k] = sp[k];
            }

            if (t == a.T) {
                float rho[MP];
#pragma unroll
                for (int k = 0; k < MP; ++k) rho[k] = ex2(sq[k] - gp[k]);   // 1 on padding
                float acc[WIDE ? 1 : MP];
                float q[n_slots(MP)];
                rev_init<MP, R, WIDE>(a, c, om, gp, rho, rg, fb0, cb, acc, q, sh, u, active, tm);
                if constexpr (WIDE) {
                    gbar[0] = wide_total<MP>(q, tm, cs.col, red, par);
                } else {
                    group_allreduce<MP>(acc, tm.L);
#pragma unroll
                    for (int k = 0; k < MP; ++k) gbar[k] = acc[k];
                }
                par ^= 1;
            }

            // gh_k = gbar_k / sig^t_k
            if constexpr (WIDE) {
                const float ghd = cs.live ? gbar[0] * ex2(sq[cs.col] - sp[cs.col]) * cs.ibc : 0.f;
                spread_owned<MP>(ghd, gh);
            } else {
#pragma unroll
                for (int k = 0; k < MP; ++k) gh[k] = gbar[k] * ex2(sq[k] - gp[k]) * cs.ib[k];
            }

            // reverse of iteration t
            if constexpr (WIDE) {
                float q[n_slots(MP)];
                float acc[MP];
                rev_pass<MP, R>(c, om, gp, gh, fb0, t == a.T, cb, acc, off);
                scatter_all<MP>(acc, q);
                gbar[0] = -wide_total<MP>(q, tm, cs.col, red, par);
            } else {
                float acc[MP];
                rev_pass<MP, R>(c, om, gp, gh, fb0, t == a.T, cb, acc, off);
                group_allreduce<MP>(acc, tm.L);
#pragma unroll
                for (int k = 0; k < MP; ++k) gbar[k] = -acc[k];
            }
            par ^= 1;
        }
    }

    // epilogue: write gF * dF/dC, or apply the ascent step to C in place
    if (active) bwd_epilogue<MP, R>(a, cb, u, tm);

}

// ---------------------------------------------------------------------------
// Implicit-function gradient at a converged plan (the converged-map form of
// Algorithm 1).  With the plan X, G_ik = gF r_i e_k / Imp_i (0 on the dummy),
// the row and column sums rX, cX of X and h_i = sum_k X_ik G_ik, the gradient
// of the balanced plan is
//   dF/dc_ik = -(1/eps) X_ik (G_ik - lam_i - mu_k),
// where mu (mu_{m-1} = 0) solves the Schur system of the optimality
// conditions,
//   S mu = t,  S = diag(cX) - X^T diag(rX)^-1 X,  t_k = sum_i X_ik (G_ik - h_i / rX_i),
// and lam_i = (h_i - sum_k X_ik mu_k) / rX_i.  On mu_{m-1} = 0, S is symmetric
// positive definite (v^T S v is a sum of per-row variances of v), so mu comes
// from conjugate gradients preconditioned by diag(S): one product S p per
// iteration is two FMAs per plan cell and one column reduction.

// Column vectors of the solver: every lane holds all of them in a narrow
// team; in a wide team each lane holds the component of the column it owns.
template <int MP, bool WIDE>
struct CVec;
template <int MP>
struct CVec<MP, false> {
    float v[MP];
};
template <int MP>
struct CVec<MP, true> {
    float v;
};

template <int MP, bool WIDE>
struct Solver {
    const Team& tm;
    Cols<MP, WIDE>& cs;
    float* red;
    int par = 0;
    CVec<MP, WIDE> msk;   // 1 on the real positions k < m - 1, else 0

    __device__ Solver(const Team& t, Cols<MP, WIDE>& c, float* r, int m) : tm(t), cs(c), red(r) {
        if constexpr (WIDE) {
            msk.v = (cs.col >= 0 && cs.col < m - 1) ? 1.f : 0.f;
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) msk.v[k] = (k < m - 1) ? 1.f : 0.f;
        }
    }
    // team sums of the lanes' column partials
    __device__ CVec<MP, WIDE> reduce(float (&acc)[MP]) {
        CVec<MP, WIDE> out;
        if constexpr (WIDE) {
            float q[n_slots(MP)];
            scatter_all<MP>(acc, q);
            out.v = wide_total<MP>(q, tm, cs.col, red, par);
            par ^= 1;
        } else {
            group_allreduce<MP>(acc, tm.L);
#pragma unroll
            for (int k = 0; k < MP; ++k) out.v[k] = acc[k];
        }
        return out;
    }
    __device__ float dot(const CVec<MP, WIDE>& x, const CVec<MP, WIDE>& y) {
        if constexpr (WIDE) {
            float t[1] = {x.v * y.v * msk.v};
            group_allreduce<1>(t, 64);
            return t[0];
        } else {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < MP; ++k) s = fmaf(x.v[k] * msk.v[k], y.v[k], s);
            return s;
        }
    }
    // the vector as a uniform array (scalars in a wide team)
    __device__ void spread(const CVec<MP, WIDE>& x, float (&out)[MP]) {
        if constexpr (WIDE) {
            spread_owned<MP>(x.v * msk.v, out);
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) out[k] = x.v[k] * msk.v[k];
        }
    }
};

template <int MP, bool WIDE, class F>
__device__ __forceinline__ void cv_apply(CVec<MP, WIDE>& out, F&& f) {
    if constexpr (WIDE) {
        out.v = f(out.v, 0);
    } else {
#pragma unroll
        for (int k = 0; k < MP; ++k) out.v[k] = f(out.v[k], k);
    }
}

template <int MP, int R, bool WIDE>
__device__ __forceinline__ void ibwd_body(const BwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int teams = blockDim.x / a.L;
    const int64_t u = u_first + tm.team;
    const bool active = tm.team < teams && u < a.U;
    const int I = a.I, m = a.m;
    float* red = smem + tm.team * (2 * tm.W * MP);

    float x[R][MP], om[R], off[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, a.c2, x, om, off);
    float gam[MP];
    Cols<MP, WIDE> cs;
    cs.init(tm, m, 0.f, 1.f, gam);
    const float* gs = a.gw + (active ? u : 0) * (int64_t)a.hs;
    if constexpr (WIDE) {
        cs.gd = (active && cs.col >= 0) ? gs[cs.col] : kNeg;
        spread_owned<MP>(cs.gd, gam);
    } else {
#pragma unroll
        for (int k = 0; k < MP; ++k) gam[k] = active ? gs[k] : kNeg;
    }

    // the plan, its row sums, h_i and the column partials of cX, t and diag S
    const int mo = opaque_u(m);
    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < mo - 1) ? a.e[k] : 0.f;
    float rX[R], h[R], rg[R];
    float ac[MP], at[MP], ad[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ac[k] = at[k] = ad[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        const bool valid = active && i < I;
        const float ph = valid ? a.phi[u * I + i] + off[j] : 0.f;
        rg[j] = valid ? (float)(a.gF * (double)a.r[u * I + i] / a.imp[i]) : 0.f;
        float s = 0.f, hh = 0.f;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const float xv = valid ? ex2((x[j][k] + gam[k]) + ph) : 0.f;
            x[j][k] = xv;
            s += xv;
            hh = fmaf(ek[k], xv, hh);
        }
        rX[j] = valid ? s : 1.f;
        h[j] = rg[j] * hh;
        const float ir = 1.f / rX[j];
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            ac[k] += x[j][k];
            at[k] = fmaf(x[j][k], rg[j] * ek[k] - h[j] * ir, at[k]);
            ad[k] = fmaf(x[j][k] * x[j][k], ir, ad[k]);
        }
    }
    Solver<MP, WIDE> sv(tm, cs, red, m);
    const CVec<MP, WIDE> cX = sv.reduce(ac);
    const CVec<MP, WIDE> tv = sv.reduce(at);
    CVec<MP, WIDE> dg = sv.reduce(ad);
    cv_apply<MP, WIDE>(dg, [&](float d, int k) {
        float cxk;
        if constexpr (WIDE) cxk = cX.v; else cxk = cX.v[k];
        const float v = cxk - d;
        return v > 0.f ? v : 1.f;
    });

    // preconditioned conjugate gradients for mu
    CVec<MP, WIDE> xs, rr = tv, z, p, Sp;
    cv_apply<MP, WIDE>(xs, [](float, int) { return 0.f; });
    auto precond = [&](const CVec<MP, WIDE>& r) {
        CVec<MP, WIDE> o;
        if constexpr (WIDE) {
            o.v = r.v / dg.v;
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) o.v[k] = r.v[k] / dg.v[k];
        }
        return o;
    };
    z = precond(rr);
    p = z;
    float rz = sv.dot(rr, z);
    const float tn = sqrtf(sv.dot(tv, tv));
    for (int it = 0; it < a.cg_max && tn > 0.f; ++it) {
        float pa[MP];
        sv.spread(p, pa);
        float acc[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < MP; ++k) s = fmaf(x[j][k], pa[k], s);
            const float w = s / rX[j];
#pragma unroll
            for (int k = 0; k < MP; ++k) acc[k] = fmaf(x[j][k], w, acc[k]);
        }
        const CVec<MP, WIDE> tot = sv.reduce(acc);
        if constexpr (WIDE) {
            Sp.v = cX.v * p.v - tot.v;
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) Sp.v[k] = cX.v[k] * p.v[k] - tot.v[k];
        }
        const float pSp = sv.dot(p, Sp);
        if (!(pSp > 0.f)) break;
        const float al = rz / pSp;
        if constexpr (WIDE) {
            xs.v = fmaf(al, p.v, xs.v);
            rr.v = fmaf(-al, Sp.v, rr.v);
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) {
                xs.v[k] = fmaf(al, p.v[k], xs.v[k]);
                rr.v[k] = fmaf(-al, Sp.v[k], rr.v[k]);
            }
        }
        if (sqrtf(sv.dot(rr, rr)) <= a.cg_tol * tn) break;
        z = precond(rr);
        const float rzn = sv.dot(rr, z);
        const float be = rzn / rz;
        rz = rzn;
        if constexpr (WIDE) {
            p.v = fmaf(be, p.v, z.v);
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) p.v[k] = fmaf(be, p.v[k], z.v[k]);
        }
    }
    float mu[MP];
    sv.spread(xs, mu);

    // lam, the gradient, and the update (or dF/dC)
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
        float xm = 0.f, xe = 0.f;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            xm = fmaf(x[j][k], mu[k], xm);
            xe = fmaf(ek[k], x[j][k], xe);
        }
        const float lam = (h[j] - xm) / rX[j];
        if (a.dr) a.dr[u * I + i] = (float)(a.gF / a.imp[i]) * xe;
        const int64_t base = (u * I + i) * (int64_t)m;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            if (k >= mo) continue;
            const float g = -a.inv_eps * x[j][k] * (rg[j] * ek[k] - lam - mu[k]);
            if (a.dC) a.dC[base + k] = g;
            if (a.Cw) {
                const float craw = a.C[base + k];
                if (a.rule == 0) {
                    const float gl = -g;
                    const float mo1 = a.b1 * a.mom[base + k] + (1.f - a.b1) * gl;
                    const float ve = a.b2 * a.vel[base + k] + (1.f - a.b2) * gl * gl;
                    a.mom[base + k] = mo1;
                    a.vel[base + k] = ve;
                    a.Cw[base + k] = craw - a.lr * (mo1 / bc1) / (sqrtf(ve / bc2) + a.aeps);
                } else {
                    a.Cw[base + k] = craw + a.lr * g;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Reverse sweep in the scaling form (every iterate stored, K = 1).  The
// registers hold Kt_ik = 2^(a_ik + rf_k + ph_i) for reference column
// potentials rf and a row offset ph that puts each row's largest entry at 1,
// so that P^t_ik = Kt_ik w_k / s_i with w_k = 2^(gamma^{t-1}_k - rf_k) (one
// exponential per column and iteration) and s_i = sum_k Kt_ik w_k: the
// reverse recursion of the log-domain sweep runs on multiplies and
// multiply-adds only.  When a live column's w leaves [2^-32, 2^32] (or every
// `absorb` iterations, if set) the reference moves to gamma^{t-1} and Kt is
// rebuilt from the costs in HBM, one exponential per cell; entries that
// underflow at a rebuild stay below 2^-94 of their row until the next one.

// Kt of the lane's rows for reference rf: from the centred costs held in kt
// (FROM_REGS, at the start) or re-read from C -- then in two passes over the
// row (its maximum, then the exponentials), so that no row of temporaries is
// live beside Kt and the cost adjoints.
template <int MP, int R, bool FROM_REGS>
__device__ __forceinline__ void rebase_rows(const float* C, int64_t u, const Team& tm, int I, int m,
                                            float c2, const float (&om)[R], const float (&off)[R],
                                            const float (&rf)[MP], float (&kt)[R][MP]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        const bool valid = om[j] > 0.f;
        const float* src = C + (u * I + (valid ? i : 0)) * (int64_t)m;
        auto z = [&](int k) {
            if constexpr (FROM_REGS)
                return kt[j][k] + rf[k];
            else
                return (valid ? fmaf(src[k < m ? k : m - 1], c2, -off[j]) : 0.f) + rf[k];
        };
        float mx[4] = {kNeg, kNeg, kNeg, kNeg};
#pragma unroll
        for (int k = 0; k < MP; ++k) mx[k & 3] = fmaxf(mx[k & 3], z(k));
        const float M = fmaxf(fmaxf(mx[0], mx[1]), fmaxf(mx[2], mx[3]));
#pragma unroll
        for (int k = 0; k < MP; ++k) kt[j][k] = ex2(z(k) - M);
    }
}

// Start of the reverse sweep in the scaling form (see rev_init).
template <int MP, int R, bool WIDE>
__device__ __forceinline__ void rev_init_s(const BwdArgs& a, const float (&kt)[R][MP],
                                           const float (&om)[R], const float (&wv)[MP],
                                           const float (&rho)[MP], const float (&rg)[R],
                                           float (&fb0)[R], float (&cb)[R][MP],
                                           float (&acc)[WIDE ? 1 : MP], float (&q)[n_slots(MP)],
                                           int64_t u, bool active, const Team& tm) {
    const int m = opaque_u(a.m);
    float ek[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) ek[k] = (k < m - 1) ? a.e[k] : 0.f;
    float w[R], xe[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float ps[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MP; ++k) ps[k & 3] = fmaf(kt[j][k], wv[k], ps[k & 3]);
        w[j] = om[j] * rcp((ps[0] + ps[1]) + (ps[2] + ps[3])) * a.inv_eps;
        fb0[j] = 0.f;
        xe[j] = 0.f;
    }
    for_chunks<MP>([&](auto ch) {
        constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
        float v[ci.n];
#pragma unroll
        for (int kk = 0; kk < ci.n; ++kk) v[kk] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) {
                const int k = ci.k0 + kk;
                const float xs = fmaf(kt[j][k], wv[k], 0.f) * w[j] * rho[k];   // x / eps
                const float gx = rg[j] * ek[k] * xs;                            // G x / eps
                cb[j][k] = -gx;
                fb0[j] += gx;
                v[kk] += gx;
                xe[j] = fmaf(ek[k], xs, xe[j]);
            }
        }
        if constexpr (WIDE) {
            scatter_chunk<MP, decltype(ch)::value>(v, q);
        } else {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) acc[ci.k0 + kk] = v[kk];
        }
    });
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        if (a.dr && active && i < a.I)
            a.dr[u * a.I + i] = (float)(a.gF / a.imp[i]) * (xe[j] / a.inv_eps);
    }
}

// Reverse of iteration t in the scaling form, one row of e = Kt w kept at a
// time (see rev_pass).
template <int MP, int R>
__device__ __forceinline__ void rev_pass_s(const float (&kt)[R][MP], const float (&om)[R],
                                           const float (&wv)[MP], const float (&gh)[MP],
                                           const float (&fb0)[R], bool first, float (&cb)[R][MP],
                                           float (&acc)[MP]) {
#pragma unroll
    for (int k = 0; k < MP; ++k) acc[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float e[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k) e[k] = kt[j][k] * wv[k];
        const float s = Tree<MP>::sum(e);
        float pd[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MP; ++k) pd[k & 3] = fmaf(e[k], gh[k], pd[k & 3]);
        const float d = (pd[0] + pd[1]) + (pd[2] + pd[3]);
        const float w = om[j] * rcp(s);
        const float fb = (first ? fb0[j] : 0.f) - w * d;
        const float aa = w * fb;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            cb[j][k] = fmaf(e[k], fmaf(w, gh[k], aa), cb[j][k]);
            acc[k] = fmaf(e[k], aa, acc[k]);
        }
    }
}

// Two-pass variant (wide teams whose registers cannot keep a row of e): row
// totals first, then the cost adjoint and the column partials chunk by chunk.
// The second pass forms e as an FMA with 0 so that the first pass's products
// are not kept live for it.
template <int MP, int R>
__device__ __forceinline__ void rev_pass_s_recomp(const float (&kt)[R][MP], const float (&om)[R],
                                                  const float (&wv)[MP], const float (&gh)[MP],
                                                  const float (&fb0)[R], bool first,
                                                  float (&cb)[R][MP], float (&q)[n_slots(MP)]) {
    float w[R], aa[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        float ps[4] = {0.f, 0.f, 0.f, 0.f}, pd[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < MP; ++k) {
            const float e = kt[j][k] * wv[k];
            ps[k & 3] += e;
            pd[k & 3] = fmaf(e, gh[k], pd[k & 3]);
        }
        const float s = (ps[0] + ps[1]) + (ps[2] + ps[3]);
        const float d = (pd[0] + pd[1]) + (pd[2] + pd[3]);
        w[j] = om[j] * rcp(s);
        const float fb = (first ? fb0[j] : 0.f) - w[j] * d;
        aa[j] = w[j] * fb;
    }
    __builtin_amdgcn_sched_barrier(0);
    for_chunks<MP>([&](auto ch) {
        constexpr ChunkInfo ci = chunk_info(MP, decltype(ch)::value);
        float v[ci.n];
#pragma unroll
        for (int kk = 0; kk < ci.n; ++kk) v[kk] = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int kk = 0; kk < ci.n; ++kk) {
                const int k = ci.k0 + kk;
                const float e = fmaf(kt[j][k], wv[k], 0.f);
                cb[j][k] = fmaf(e, fmaf(w[j], gh[k], aa[j]), cb[j][k]);
                v[kk] = fmaf(e, aa[j], v[kk]);
            }
        }
        scatter_chunk<MP, decltype(ch)::value>(v, q);
    });
    __builtin_amdgcn_sched_barrier(0);
}

template <int MP, int R, bool WIDE, bool RECOMP>
__device__ __forceinline__ void bwds_body(const BwdArgs& a, int64_t u_first, float* smem) {
    const Team tm = make_team(a.L);
    const int teams = blockDim.x / a.L;
    const int64_t u = u_first + tm.team;
    const bool active = tm.team < teams && u < a.U;
    const int I = a.I, m = a.m;
    constexpr int BL = kLoadBlock;
    float* seg = smem + tm.team * ((BL + 1) * MP);
    float* red = smem + teams * ((BL + 1) * MP) + tm.team * (2 * tm.W * MP);

    float kt[R][MP], om[R], off[R];
    load_costs<MP, R>(a.C, u, active, tm, I, m, a.c2, kt, om, off);   // centred costs until the first rebase

    float rg[R];   // gF r_i / Imp_i, so that G_ik = rg_i e_k
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tm.lt + j * tm.L;
        rg[j] = (active && i < I) ? (float)(a.gF * (double)a.r[u * I + i] / a.imp[i]) : 0.f;
    }
    float gdum[MP];
    Cols<MP, WIDE> cs;
    cs.init(tm, m, lg2((float)(I - m + 1)), 1.0f / (float)(I - m + 1), gdum);

    const float* hist = active ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    float cb[R][MP], fb0[R];
    float gbar[WIDE ? 1 : MP];
#pragma unroll
    for (int k = 0; k < (WIDE ? 1 : MP); ++k) gbar[k] = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) fb0[j] = 0.f;
    float rf[MP];                 // reference potentials (wide: wave-uniform copies)
#pragma unroll
    for (int k = 0; k < MP; ++k) rf[k] = 0.f;   // set at t = T, before any use
    [[maybe_unused]] float rfd = 0.f;   // wide: the owned column's reference

    // first reference: gamma^{T-1}, from the centred costs in the registers
    {
        const float* last = active ? hist + (int64_t)(a.T - 1) * a.hs : nullptr;
        if constexpr (WIDE) {
            rfd = (active && cs.col >= 0) ? last[cs.col] : 0.f;
            spread_owned<MP>(rfd, rf);
        } else {
#pragma unroll
            for (int k = 0; k < MP; ++k) rf[k] = active ? last[k] : 0.f;
        }
        rebase_rows<MP, R, true>(a.C, active ? u : 0, tm, I, m, a.c2, om, off, rf, kt);
    }

    int par = 0;
    const int nblk = (a.T + BL - 1) / BL;
    for (int s = nblk - 1; s >= 0; --s) {
        const int t0 = s * BL;
        const int t1 = min(t0 + BL, a.T);
        const int n = t1 - t0;
        __syncthreads();  // the previous block's reads of seg are complete
        for (int idx = tm.lt; idx < (n + 1) * MP; idx += tm.L) {
            const int qq = idx / MP, k = idx - qq * MP;
            seg[idx] = active ? hist[(int64_t)(t0 + qq) * a.hs + k] : 0.f;
        }
        __syncthreads();

        for (int qq = n; qq >= 1; --qq) {
            const int t = t0 + qq;
            const float* sq = seg + qq * MP;        // gamma^t
            const float* sp = seg + (qq - 1) * MP;  // gamma^{t-1}
            const bool force = t < a.T && a.absorb > 0 && (a.T - t) % a.absorb == 0;

            // scalings of gamma^{t-1} against the reference; rebase when out of range
            float wv[MP];
            if constexpr (WIDE) {
                const float gpd = (cs.col >= 0) ? sp[cs.col] : kNeg;
                float wd = cs.live ? ex2(gpd - rfd) : 0.f;
                const bool bad = wave_any(cs.live && !(wd >= kScaleLo && wd <= kScaleHi));
                if (force || bad) {
                    rfd = gpd;
                    wd = cs.live ? 1.f : 0.f;
                    spread_owned<MP>(rfd, rf);
                    rebase_rows<MP, R, false>(a.C, active ? u : 0, tm, I, m, a.c2, om, off, rf, kt);
                }
                spread_owned<MP>(wd, wv);
            } else {
                bool bad = false;
#pragma unroll
                for (int k = 0; k < MP; ++k) {
                    wv[k] = ex2(sp[k] - rf[k]);   // padding: kNeg - kNeg = 0, w = 1 on a zero Kt
                    bad = bad || !(wv[k] >= kScaleLo && wv[k] <= kScaleHi);
                }
                if (force || wave_any(bad)) {
#pragma unroll
                    for (int k = 0; k < MP; ++k) {
                        rf[k] = sp[k];
                        wv[k] = 1.f;
                    }
                    rebase_rows<MP, R, false>(a.C, active ? u : 0, tm, I, m, a.c2, om, off, rf, kt);
                }
            }

            if (t == a.T) {
                float rho[MP];
                float gp[MP];
                if constexpr (WIDE) {
                    spread_owned<MP>((cs.col >= 0) ? sp[cs.col] : kNeg, gp);
                } else {
#pragma unroll
                    for (int k = 0; k < MP; ++k) gp[k] = sp[k];
                }
#pragma unroll
                for (int k = 0; k < MP; ++k) rho[k] = ex2(sq[k] - gp[k]);   // 1 on padding
                float acc[WIDE ? 1 : MP];
                float q[n_slots(MP)];
                rev_init_s<MP, R, WIDE>(a, kt, om, wv, rho, rg, fb0, cb, acc, q, u, active, tm);
                if constexpr (WIDE) {
                    gbar[0] = wide_total<MP>(q, tm, cs.col, red, par);
                } else {
                    group_allreduce<MP>(acc, tm.L);
#pragma unroll
                    for (int k = 0; k < MP; ++k) gbar[k] = acc[k];
                }
                par ^= 1;
            }

            // gh_k = gbar_k / sig^t_k
            float gh[MP];
            if constexpr (WIDE) {
                const float ghd = cs.live ? gbar[0] * ex2(sq[cs.col] - sp[cs.col]) * cs.ibc : 0.f;
                spread_owned<MP>(ghd, gh);
            } else {
#pragma unroll
                for (int k = 0; k < MP; ++k) gh[k] = gbar[k] * ex2(sq[k] - sp[k]) * cs.ib[k];
            }

            // reverse of iteration t
            if constexpr (WIDE) {
                float q[n_slots(MP)];
                if constexpr (RECOMP) {
                    rev_pass_s_recomp<MP, R>(kt, om, wv, gh, fb0, t == a.T, cb, q);
                } else {
                    float acc[MP];
                    rev_pass_s<MP, R>(kt, om, wv, gh, fb0, t == a.T, cb, acc);
                    scatter_all<MP>(acc, q);
                }
                gbar[0] = -wide_total<MP>(q, tm, cs.col, red, par);
            } else {
                float acc[MP];
                rev_pass_s<MP, R>(kt, om, wv, gh, fb0, t == a.T, cb, acc);
                group_allreduce<MP>(acc, tm.L);
#pragma unroll
                for (int k = 0; k < MP; ++k) gbar[k] = -acc[k];
            }
            par ^= 1;
        }
    }
    if (active) {
        ArrAdj<MP, R> cba{cb};
        bwd_epilogue<MP, R>(a, cba, u, tm);
    }
}

// ---------------------------------------------------------------------------
// Per-lane registers available at launch bound LB (512 per SIMD lane shared
// by LB / 256 waves, at most 256 architectural VGPRs), minus a reserve for
// addresses and temporaries.
constexpr int reg_budget(int LB) { return (131072 / LB < 256 ? 131072 / LB : 256) - 32; }
template <int R, int LB, bool WIDE>
constexpr bool recomp_fwd() { return WIDE && (R * FR_MP + 2 * FR_MP > reg_budget(LB)); }
template <int R, int LB, bool WIDE>
constexpr bool recomp_bwd() { return WIDE && (2 * R * FR_MP + 2 * FR_MP > reg_budget(LB)); }

template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_fwd(FwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    fwd_body<MP, R, WIDE, recomp_fwd<R, LB, WIDE>()>(a, (int64_t)blockIdx.x * (blockDim.x / a.L),
                                                     smem);
}

// Scaling-form reverse sweep (K = 1; same gradient as k_bwd).  Its register
// need is the log-domain kernel's, so it recomputes under the same rule.
template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_bwds(BwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    bwds_body<MP, R, WIDE, recomp_bwd<R, LB, WIDE>()>(a, (int64_t)blockIdx.x * (blockDim.x / a.L),
                                                      smem);
}

// Scaling-form forward (same iterates as k_fwd).
template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_fwds(FwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    fwds_body<MP, R, WIDE>(a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

// Converged-map forward: warm start from a.gw, stop at tolerance a.tol.
template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_fwdc(FwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;
    fwd_body<MP, R, WIDE, recomp_fwd<R, LB, WIDE>(), true>(
        a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_bwd(BwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    bwd_body<MP, R, WIDE, recomp_bwd<R, LB, WIDE>()>(a, (int64_t)blockIdx.x * (blockDim.x / a.L),
                                                     smem);
}

// Rows of cost adjoints per lane that the wide recompute reverse sweep keeps
// in LDS at launch bound LB (512 or 1024: one team per block): as many as fit,
// with the segment and reduction buffers of K = 1, in 144 KB of the 160 KB of
// LDS, all but one row at most.
template <int R, int LB, bool WIDE>
constexpr int cb_lds_rows() {
    if (!(WIDE && LB >= 512 && recomp_bwd<R, LB, WIDE>())) return 0;
    for (int n = R - 1; n >= 1; --n)
        if ((n * LB + (kLoadBlock + 1) + 2 * (LB / 64)) * FR_MP * 4 <= 144 * 1024) return n;
    return 0;
}

// k_bwd with cb_lds_rows() rows of cost adjoints in LDS.
template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_bwdl(BwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    if constexpr (cb_lds_rows<R, LB, WIDE>() > 0)
        bwd_body<MP, R, WIDE, recomp_bwd<R, LB, WIDE>(), cb_lds_rows<R, LB, WIDE>()>(
            a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

template <int MP, int R, int LB, bool WIDE>
__global__ __launch_bounds__(LB) void k_ibwd(BwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    ibwd_body<MP, R, WIDE>(a, (int64_t)blockIdx.x * (blockDim.x / a.L), smem);
}

// ---------------------------------------------------------------------------
// Persistent batched kernels: every block repeatedly takes the next work item
// (instance, first consumer) from a global counter and runs the same team
// body on it, until the list is exhausted.  Items are ordered longest first.
// Blocks of LB threads: 256 (several teams of up to 256 lanes) or 512 (one
// team of 512 lanes).
template <int MP, int R, int LB, bool WIDE, bool SCALE>
__global__ __launch_bounds__(LB) void k_bfwd(const FwdArgs* __restrict__ descs,
                                              const BatchItem* __restrict__ items, int n_items,
                                              unsigned* counter) {
    extern __shared__ float smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        const FwdArgs a = descs[bi.inst];
        if constexpr (SCALE)
            fwds_body<MP, R, WIDE>(a, bi.u0, smem);
        else
            fwd_body<MP, R, WIDE, recomp_fwd<R, LB, WIDE>()>(a, bi.u0, smem);
    }
}

template <int MP, int R, int LB, bool WIDE, bool SCALE>
__global__ __launch_bounds__(LB) void k_bbwd(const BwdArgs* __restrict__ descs,
                                              const BatchItem* __restrict__ items, int n_items,
                                              unsigned* counter) {
    extern __shared__ float smem[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const BatchItem bi = items[it];
        const BwdArgs a = descs[bi.inst];
        if constexpr (SCALE)
            bwds_body<MP, R, WIDE, recomp_bwd<R, LB, WIDE>()>(a, bi.u0, smem);
        else
            bwd_body<MP, R, WIDE, recomp_bwd<R, LB, WIDE>()>(a, bi.u0, smem);
    }
}

template <int MP, int R, int LB, bool WIDE, bool SCALE>
void launch_bfwd(const FwdArgs* d, const BatchItem* it, int n, unsigned* ctr, int grid, int block,
                 size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bfwd<MP, R, LB, WIDE, SCALE>), dim3(grid), dim3(block), lds, s, d, it, n,
                       ctr);
}
template <int MP, int R, int LB, bool WIDE, bool SCALE>
void launch_bbwd(const BwdArgs* d, const BatchItem* it, int n, unsigned* ctr, int grid, int block,
                 size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bbwd<MP, R, LB, WIDE, SCALE>), dim3(grid), dim3(block), lds, s, d, it, n,
                       ctr);
}
template <int MP, int R, int LB, bool WIDE, bool SCALE>
int occupancy_bfwd(int block, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_bfwd<MP, R, LB, WIDE, SCALE>, block,
                                                     lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
template <int MP, int R, int LB, bool WIDE, bool SCALE>
int occupancy_bbwd(int block, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_bbwd<MP, R, LB, WIDE, SCALE>, block,
                                                     lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int MP, int R, int LB, bool WIDE>
void launch_fwd(const FwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_bwd(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_bwdl(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bwdl<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_bwds(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_bwds<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_fwds(const FwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_fwds<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_fwdc(const FwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_fwdc<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}
template <int MP, int R, int LB, bool WIDE>
void launch_ibwd(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_ibwd<MP, R, LB, WIDE>), dim3(grid), dim3(block), lds, s, a);
}

template <int R, int LB, bool WIDE>
constexpr FusedEntry entry() {
    if constexpr (LB == 256 || (LB == 512 && R == 1)) {
        return FusedEntry{FR_MP,
                          R,
                          LB,
                          WIDE,
                          recomp_fwd<R, LB, WIDE>(),
                          recomp_bwd<R, LB, WIDE>(),
                          &launch_fwd<FR_MP, R, LB, WIDE>,
                          &launch_bwd<FR_MP, R, LB, WIDE>,
                          &launch_fwdc<FR_MP, R, LB, WIDE>,
                          &launch_ibwd<FR_MP, R, LB, WIDE>,
                          &launch_fwds<FR_MP, R, LB, WIDE>,
                          &launch_bfwd<FR_MP, R, LB, WIDE, false>,
                          &launch_bbwd<FR_MP, R, LB, WIDE, false>,
                          &occupancy_bfwd<FR_MP, R, LB, WIDE, false>,
                          &occupancy_bbwd<FR_MP, R, LB, WIDE, false>,
                          &launch_bfwd<FR_MP, R, LB, WIDE, true>,
                          &occupancy_bfwd<FR_MP, R, LB, WIDE, true>,
                          &launch_bwds<FR_MP, R, LB, WIDE>,
                          &launch_bbwd<FR_MP, R, LB, WIDE, true>,
                          &occupancy_bbwd<FR_MP, R, LB, WIDE, true>,
                          LB == 512 && cb_lds_rows<R, LB, WIDE>() > 0 ? &launch_bwdl<FR_MP, R, LB, WIDE>
                                                                      : nullptr,
                          LB == 512 ? cb_lds_rows<R, LB, WIDE>() : 0};
    } else {
        return FusedEntry{FR_MP, R, LB, WIDE, recomp_fwd<R, LB, WIDE>(), recomp_bwd<R, LB, WIDE>(),
                          &launch_fwd<FR_MP, R, LB, WIDE>, &launch_bwd<FR_MP, R, LB, WIDE>,
                          &launch_fwdc<FR_MP, R, LB, WIDE>, &launch_ibwd<FR_MP, R, LB, WIDE>,
                          &launch_fwds<FR_MP, R, LB, WIDE>, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &launch_bwds<FR_MP, R, LB, WIDE>, nullptr, nullptr,
                          cb_lds_rows<R, LB, WIDE>() > 0 ? &launch_bwdl<FR_MP, R, LB, WIDE>
                                                         : nullptr,
                          cb_lds_rows<R, LB, WIDE>()};
    }
}

// Rows per lane instantiated for this column class.  Narrow teams (several
// per wave) keep R * MP <= 128 costs per lane; wave-wide teams up to 256 at
// launch bounds 256 and 512 and up to 128 at launch bound 1024.
#define FR_NARROW_OK(R) ((R) * FR_MP <= 128)
#define FR_WIDE_OK(R) ((R) * FR_MP <= 256)
#define FR_BIG_OK(R) ((R) * FR_MP <= 128)

const FusedEntry kEntries[] = {
    entry<1, 256, false>(),
#if FR_NARROW_OK(2)
    entry<2, 256, false>(),
#endif
#if FR_NARROW_OK(3)
    entry<3, 256, false>(),
#endif
#if FR_NARROW_OK(4)
    entry<4, 256, false>(),
#endif
#if FR_NARROW_OK(6)
    entry<6, 256, false>(),
#endif
#if FR_NARROW_OK(8)
    entry<8, 256, false>(),
#endif
    entry<1, 256, true>(),
    entry<2, 256, true>(),
#if FR_WIDE_OK(3)
    entry<3, 256, true>(),
#endif
#if FR_WIDE_OK(4)
    entry<4, 256, true>(),
#endif
#if FR_WIDE_OK(6)
    entry<6, 256, true>(),
#endif
#if FR_WIDE_OK(8)
    entry<8, 256, true>(),
#endif
    entry<1, 512, true>(),
    entry<2, 512, true>(),
#if FR_WIDE_OK(3)
    entry<3, 512, true>(),
#endif
#if FR_WIDE_OK(4)
    entry<4, 512, true>(),
#endif
    entry<1, 1024, true>(),
#if FR_BIG_OK(2)
    entry<2, 1024, true>(),
#endif
#if FR_BIG_OK(4)
    entry<4, 1024, true>(),
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
