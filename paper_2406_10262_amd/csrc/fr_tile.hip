// fr_tile.hip -- Sinkhorn forward and adjoint backward of Algorithm 1 for
// large plans (hundreds of items, tens of positions per consumer) on gfx950.
//
// Mapping.  One block of 64 W lanes owns one consumer.  The plan is cut into
// 2-D tiles: lanes are grouped in quads (G = 4 lanes, a DPP quad), the quad
// of lane l is row group rg = 16 w + l / 4 of the block (w its wave), and
// lane l % 4 of the quad (its column group cg) holds the CT consecutive
// columns cg CT .. cg CT + CT - 1 of the RT rows i = j RG + rg (j < RT,
// RG = 16 W row groups).  A row half-step of Sinkhorn (Section 3, problem
// otp) is then a lane-local sum over CT columns and a two-step DPP sum over
// the quad; a column half-step is a lane-local sum over RT rows, a sum over
// the 16 quads of a wave (two DPP rotations inside each 16-lane row and the
// two gfx950 row swaps across rows) and a sum of the W wave partials through
// LDS, one barrier per half-step.
//
// Forward (k_tfwd).  Scaling form with log-domain absorption, the same
// iterates as the log-domain recursion: registers hold the kernel
//   Kt_ik = 2^(a_ik + gam_k + ph_i),  a_ik = -c_ik / (eps ln 2) - o_i,
// (o_i the row maximum at load) and an iteration updates the scalings only,
//   u_i = 1 / sum_k Kt_ik v_k,   v_k = b_k / sum_i Kt_ik u_i,
// with b = (1, ..., 1, I - m + 1) (the dummy column, Section 2).  When a
// column scaling leaves [2^-32, 2^32] (or every `absorb` iterations) the
// scalings move into (gam, ph) and Kt is rebuilt from C.  The base-2 column
// potentials gamma^t = gam + log2 v^t are kept for the reverse sweep.
//
// Backward.  The reverse sweep of the T iterations ("chain rule", Section 3)
// is the recursion of the log-domain kernels: with P^t the row-normalised
// plan of iteration t and gh_k = gbar_k / sig^t_k,
//   fbar_i = [t = T] fbar0_i - sum_k P_ik gh_k,
//   cbar_ik += P_ik (gh_k + fbar_i),   gbar_k <- -sum_i P_ik fbar_i,
// started from X and G = dF/dX (Eqs. Imp, objF).  Within a stretch of
// iterations that share one reference kernel Kt = 2^(a + rho + phi),
// P^t_ik = Kt_ik w_k u_i with w_k = 2^(gamma^{t-1}_k - rho_k) and
// u_i = 1 / sum_k Kt_ik w_k, so each iteration adds a rank-two matrix times
// Kt to the cost adjoint:
//   cbar_ik += Kt_ik [u_i (w_k gh_k) + (u_i fbar_i) w_k].
// The sweep (k_tbwd) therefore never holds cost adjoints: per iteration it
// forms the row sums sum_k Kt w and sum_k Kt w gh (quad sums), the column sum
// sum_i Kt (u fbar), and stores the row factor u fbar (u itself is the
// forward's, kept in the row store) and the column factors (w gh, w).
// k_tgrad then contracts them over the iterations on the matrix cores (BF16
// MFMA on three-piece splits of the FP32 factors, 32 x 32 x 16 tiles),
// multiplies by the reference kernel of each stretch, and applies the update
// (Adam / ascent) or writes dF/dC.  The initial term -G X / eps at t = T has the same form and is the
// last slot of the contraction.  A reference is rebased (a new stretch) when
// a column's w leaves [2^-32, 2^32]; at most kTileEpochs stretches per
// consumer are stored, beyond which the sweep raises FLAG_EPOCHS.
#include <type_traits>

#include "fr_device.h"
#include "fr_internal.h"

namespace fr {
namespace {

constexpr float kScaleHi = 4294967296.0f;         // 2^32
constexpr float kScaleLo = 1.0f / 4294967296.0f;  // 2^-32
constexpr float kTiny = 1.17549435e-38f;

// DPP row rotations (GFX9 encoding): lane p of a 16-lane row reads lane
// (p + n) mod 16.
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ float dpp_max(float v) {
    return fmaxf(v, dpp_mov<CTRL>(v));
}

// Sum over the four lanes of a quad (symmetric: every lane gets the same
// rounded value).
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp_mov<kQuadXor1>(v);
    v += dpp_mov<kQuadXor2>(v);
    return v;
}
__device__ __forceinline__ float quad_max(float v) {
    v = dpp_max<kQuadXor1>(v);
    v = dpp_max<kQuadXor2>(v);
    return v;
}

// ---------------------------------------------------------------------------
// Column reduction of a wave.  p[c] (c < CT) holds the lane's partial sum of
// column cg CT + c over its rows.  Step A adds the four 16-lane rows with the
// two row swaps as a reduce-scatter (CT values to H1, then H2); step B adds
// the four quads of each 16-lane row (rotations by 4 and 8, which keep the
// column group) on the H2 values left.  After it, lane 16 rho + cg + 4 q holds
// in z[q] the wave's sum of column slot slot(rho, q) of column group cg
// (valid where slot_ok).  Only the lanes of quad position 0 (q index of the
// lane, l & 12 == 0) are the wave's writers: the other three lanes of the row
// hold the same sums in another rounding order.
template <int CT>
struct Slots {
    static constexpr int H1 = (CT + 1) / 2;
    static constexpr int H2 = (H1 + 1) / 2;
    // column slot of z[q] in 16-lane row rho
    static constexpr int slot(int rho, int q) {
        return q + ((rho & 1) ? H2 : 0) + ((rho & 2) ? H1 : 0);
    }
    static constexpr bool ok(int rho, int q) {
        return q < ((rho & 1) ? H1 - H2 : H2) && slot(rho, q) < CT;
    }
};

template <int CT>
__device__ __forceinline__ void wave_colsum(float (&p)[CT], float (&z)[Slots<CT>::H2]) {
    constexpr int H1 = Slots<CT>::H1, H2 = Slots<CT>::H2;
    __builtin_amdgcn_sched_barrier(0);
    unsigned x[H1], y[H1];
#pragma unroll
    for (int c = 0; c < H1; ++c) {
        x[c] = __builtin_bit_cast(unsigned, p[c]);
        y[c] = (c + H1 < CT) ? __builtin_bit_cast(unsigned, p[c + H1]) : 0u;
    }
    swap32_batch<H1>(x, y);
    float h[H1];
#pragma unroll
    for (int c = 0; c < H1; ++c) h[c] = __builtin_bit_cast(float, x[c]) + __builtin_bit_cast(float, y[c]);
    unsigned x2[H2], y2[H2];
#pragma unroll
    for (int c = 0; c < H2; ++c) {
        x2[c] = __builtin_bit_cast(unsigned, h[c]);
        y2[c] = (c + H2 < H1) ? __builtin_bit_cast(unsigned, h[c + H2]) : 0u;
    }
    swap16_batch<H2>(x2, y2);
#pragma unroll
    for (int c = 0; c < H2; ++c) z[c] = __builtin_bit_cast(float, x2[c]) + __builtin_bit_cast(float, y2[c]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < H2; ++c) z[c] += dpp_mov<kRowRor4>(z[c]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < H2; ++c) z[c] += dpp_mov<kRowRor8>(z[c]);
    __builtin_amdgcn_sched_barrier(0);
}

// Lane roles of a block.
template <int CT, int W>
struct TLane {
    int l, w, cg, rg, rho, q;   // lane, wave, column group, row group, 16-lane row, quad position
    bool writer;                // holds the wave's column sums (q == 0)
    int rcol;                   // column this lane reduces across waves (or -1)
    int rslot;                  // its slot in the column group (cg * 16 + slot)
    int pslot;                  // where its wave sum sits in a wave's partials (cg * 16 + 4 rho + q)
    __device__ __forceinline__ TLane() {
        const int tid = threadIdx.x;
        l = tid & 63;
        w = tid >> 6;
        cg = l & 3;
        rg = w * 16 + (l >> 2);
        rho = l >> 4;
        q = (l >> 2) & 3;
        writer = q == 0;
        rcol = -1;
        rslot = 0;
        pslot = cg * 16 + rho * 4 + q;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                if (r == rho && qq == q && Slots<CT>::ok(r, qq)) {
                    rslot = cg * 16 + Slots<CT>::slot(r, qq);
                    rcol = cg * CT + Slots<CT>::slot(r, qq);
                }
    }
};

// Each writer (lane 16 rho + cg) stores its row's four sums z[0..3] with one
// 16-byte write at part[w][cg][rho][0..3]: the 16 writers of a wave fill its 64
// words (every slot written, unused ones with finite filler sums).
template <int CT, int W>
__device__ __forceinline__ void put_partials(const TLane<CT, W>& t, const float (&z)[Slots<CT>::H2],
                                             float* part) {
    constexpr int H2 = Slots<CT>::H2;
    static_assert(H2 <= 4, "four column slots per 16-lane row");
    if (!t.writer) return;
    float4 v;
    v.x = z[0];
    v.y = H2 > 1 ? z[H2 > 1 ? 1 : 0] : 0.f;
    v.z = H2 > 2 ? z[H2 > 2 ? 2 : 0] : 0.f;
    v.w = H2 > 3 ? z[H2 > 3 ? 3 : 0] : 0.f;
    *(float4*)(part + t.w * 64 + t.cg * 16 + t.rho * 4) = v;
}

// Team total of the lane's reduced column, summed in wave order (identical in
// every wave); lanes that reduce no column get a finite value they must not
// use.  The W reads are issued together.  Call after the barrier that follows
// put_partials.
template <int CT, int W>
__device__ __forceinline__ float team_total(const TLane<CT, W>& t, const float* part) {
    float x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = part[w * 64 + t.pslot];
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < W; ++w) s += x[w];
    return s;
}

// Per-wave broadcast: the reducing lanes write nv values of their column
// (vb[v][slot]), every lane then reads the values of its CT columns.  The LDS
// performs one wave's operations in the order they are issued, so the reads
// see the writes issued before them and a later write cannot overtake them;
// only the compiler has to keep that order (a compiler barrier, no wait: the
// first values are used while the rest are still arriving).
__device__ __forceinline__ void lds_wave_order() { asm volatile("" ::: "memory"); }

template <int CT, int NV>
__device__ __forceinline__ void spread_cols(float* vb, int rslot, bool has, const float (&val)[NV],
                                            int cg, float (&out)[NV][CT]) {
    if (has) {
#pragma unroll
        for (int v = 0; v < NV; ++v) vb[v * 64 + rslot] = val[v];
    }
    lds_wave_order();
    // 16-byte reads of the group's 16 slots (64-byte aligned), CT of them used
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const float4* src = (const float4*)(vb + v * 64 + cg * 16);
#pragma unroll
        for (int q = 0; q < (CT + 3) / 4; ++q) {
            const float4 x = src[q];
            if (4 * q + 0 < CT) out[v][4 * q + 0] = x.x;
            if (4 * q + 1 < CT) out[v][4 * q + 1] = x.y;
            if (4 * q + 2 < CT) out[v][4 * q + 2] = x.z;
            if (4 * q + 3 < CT) out[v][4 * q + 3] = x.w;
        }
    }
    lds_wave_order();
}

// LDS of one block: column partials (2 parities x 64 slots x W), per-wave
// broadcast areas (W x 4 x 64), and the potentials of a block of iterations.
template <int W>
constexpr size_t tile_lds_floats(bool bwd) {
    return 2 * 64 * W + W * 4 * 64 + (bwd ? (kLoadBlock + 1) * 64 : 0);
}

// Loads are unconditional from clamped, in-bounds addresses (a padded row
// reads row 0, a padded column the row's last column), and padding is made
// harmless arithmetically: padded columns carry the potential kNeg and rows
// beyond I the offset kBig, so that their kernel entries 2^(...) are exactly
// 0.  No per-cell condition stays live across the iterations.
constexpr float kBig = 1.0e30f;

__device__ __forceinline__ float opaque_f(float x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ int opaque_s(int x) {
    asm volatile("" : "+s"(x));
    return x;
}
__device__ __forceinline__ int opaque_v(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
// A wave-uniform pointer the optimiser cannot see through: addresses formed
// from it are computed where they are used instead of being hoisted (and
// kept live, or spilled) across a loop.
template <class P>
__device__ __forceinline__ P* opaque_p(P* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Scaled costs of the lane's cells: a = c c2 - o_i, with o_i the row maximum
// of c c2 over the real columns (quad max); padded columns -> about kNeg,
// rows beyond I -> offset kBig.
template <int CT, int RT, int W>
__device__ __forceinline__ void tile_load(const float* C, int64_t u, int I, int m, float c2,
                                          const TLane<CT, W>& t, float (&a)[RT][CT],
                                          float (&off)[RT], float (&om)[RT]) {
    constexpr int RG = 16 * W;
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        const bool valid = i < I;
        const float* src = C + (u * I + (valid ? i : 0)) * (int64_t)m;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int k = t.cg * CT + c;
            a[j][c] = src[k < m ? k : m - 1];
        }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        float mx = kNeg;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int k = t.cg * CT + c;
            a[j][c] = (k < m) ? a[j][c] * c2 : kNeg;
            mx = fmaxf(mx, a[j][c]);
        }
        mx = quad_max(mx);
        const bool valid = i < I;
        off[j] = valid ? mx : kBig;
        om[j] = valid ? 1.f : 0.f;
#pragma unroll
        for (int c = 0; c < CT; ++c) a[j][c] -= off[j];
    }
}

// Kt = 2^(a + gam + ph) from the costs in HBM (a = c c2 - off); gam is kNeg
// on padded columns.
template <int CT, int RT, int W>
__device__ __forceinline__ void tile_rebuild(const float* C, int64_t u, int I, int m, float c2,
                                             const TLane<CT, W>& t, const float (&off)[RT],
                                             const float (&gam)[CT], const float (&ph)[RT],
                                             float (&kt)[RT][CT]) {
    constexpr int RG = 16 * W;
    const int Io = opaque_s(I), mo = opaque_s(m);
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        const float* src = C + (u * Io + (i < Io ? i : 0)) * (int64_t)mo;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int k = t.cg * CT + c;
            kt[j][c] = src[k < mo ? k : mo - 1];
        }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j)
#pragma unroll
        for (int c = 0; c < CT; ++c) kt[j][c] = ex2((fmaf(kt[j][c], c2, -off[j]) + gam[c]) + ph[j]);
}

// Per-consumer area of the row store (RowStore in fr_internal.h), written by
// the forward for its reverse sweep.  Rows are kept in lane order, row group
// major ([rg][j], row i = j RG + rg), so that a lane's RT rows are contiguous;
// the contraction takes its first row factor from here (slot t - 1 holds u of
// iteration t, which is that factor; slot T, written by the sweep, the
// initial term's).
struct RowView {
    float* us;    // [T + 1][RG][RT]  row scaling u_i of iteration t = 1..T, then slot T
    float* ph;    // [kTileEpochs][RG][RT]  row offsets of each stretch's kernel
    float* gam;   // [kTileEpochs][64]  column potentials of each stretch's kernel
    int* sep;     // [kTileEpochs + 1]: sep[0] = number of stretches (uncapped),
                  // sep[1 + e] = first iteration of stretch e
};

__device__ __forceinline__ RowView row_view(const RowStore& rs, int64_t u, int T, int IP) {
    char* base = rs.base + u * rs.stride;
    RowView v;
    size_t o = 0;
    v.us = (float*)(base + o);
    o += sizeof(float) * (size_t)(T + 1) * IP;
    v.ph = (float*)(base + o);
    o += sizeof(float) * (size_t)kTileEpochs * IP;
    v.gam = (float*)(base + o);
    o += sizeof(float) * (size_t)kTileEpochs * 64;
    v.sep = (int*)(base + o);
    return v;
}

// ---------------------------------------------------------------------------
template <int CT, int RT, int W>
__global__ __launch_bounds__(64 * W) void k_tfwd(FwdArgs a) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    constexpr int RG = 16 * W;
    const TLane<CT, W> t;
    const int64_t u = blockIdx.x;
    const int I = a.I, m = a.m;
    float* part = smem;                      // [2][64][W]
    float* vb = smem + 2 * 64 * W + t.w * 256;   // this wave's [4][64]

    float kt[RT][CT], off[RT], om[RT];
    tile_load<CT, RT, W>(a.C, u, I, m, a.c2, t, kt, off, om);

    // the reducing lane's column: b, scaling, absorbed potential
    const bool live = t.rcol >= 0 && t.rcol < m;
    const float bk = live ? ((t.rcol == m - 1) ? (float)(I - m + 1) : 1.f) : 0.f;
    float vd = live ? 1.f : 0.f, gd = live ? 0.f : kNeg;
    float v[CT], gam[CT];
    {
        float val[2] = {vd, gd}, out[2][CT];
        spread_cols<CT, 2>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            v[c] = out[0][c];
            gam[c] = out[1][c];
        }
    }
    float ph[RT], us[RT];
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        ph[j] = 0.f;
        us[j] = 1.f;
    }
    // the first kernel by the same formula as every rebuild (the reverse
    // sweep rebuilds it bit for bit from the stored references)
    tile_rebuild<CT, RT, W>(a.C, u, I, m, a.c2, t, off, gam, ph, kt);
    // Rows beyond I have Kt = 0 exactly: their row sums start from kTiny, so
    // that u stays finite and Kt u = 0 without a per-row condition (the
    // added kTiny is below half an ulp of any row sum of a real row).

    // row store: the row scaling of every iteration and the references of
    // every stretch (stretch 0: gam = 0 on live columns, ph = 0)
    const bool store = a.rows.base && u < a.rows.n;
    RowView rv{};
    int nst = 0;
    auto put_stretch = [&](int first_it) __attribute__((always_inline)) {
        if (nst < kTileEpochs) {
            if (t.w == 0 && t.rcol >= 0) rv.gam[nst * 64 + t.rcol] = gd;
            if (t.cg == 0) {
                float4* dst = (float4*)(rv.ph + ((size_t)nst * RG + t.rg) * RT);
#pragma unroll
                for (int q = 0; q < RT / 4; ++q)
                    dst[q] = make_float4(ph[4 * q], ph[4 * q + 1], ph[4 * q + 2], ph[4 * q + 3]);
            }
            if (threadIdx.x == 0) rv.sep[1 + nst] = first_it;
        }
        ++nst;
    };
    static_assert(RT == 8, "a lane's rows are two 16-byte words of the row store");
    if (store) {
        rv = row_view(a.rows, u, a.T, RT * RG);
        put_stretch(1);
    }
    float* hist = a.hist ? a.hist + u * (int64_t)a.nck * a.hs : nullptr;
    auto put_hist = [&](float* dst) {
        if (t.w == 0 && t.rcol >= 0 && t.rcol < a.hs) dst[t.rcol] = fmaxf(gd + lg2(vd), kNeg);
    };
    if (hist) put_hist(hist);
    int kleft = a.K, kc = 0;   // iterations to the next checkpoint, checkpoints written

    for (int it = 1; it <= a.T; ++it) {
        // row half-step: u_i = 1 / sum_k Kt_ik v_k (the RT sums interleaved)
        {
            float sr[RT];
#pragma unroll
            for (int j = 0; j < RT; ++j) sr[j] = kTiny;
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int j = 0; j < RT; ++j) sr[j] = fmaf(kt[j][c], v[c], sr[j]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RT; ++j) sr[j] += dpp_mov<kQuadXor1>(sr[j]);
#pragma unroll
            for (int j = 0; j < RT; ++j) sr[j] += dpp_mov<kQuadXor2>(sr[j]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < RT; ++j) us[j] = rcp(sr[j]);
        }
        if (store && t.cg == 0) {   // the quad's four lanes hold the same eight values; one stores them
            float4* dst = (float4*)(rv.us + ((size_t)(it - 1) * RG + t.rg) * RT);
            dst[0] = make_float4(us[0], us[1], us[2], us[3]);
            dst[1] = make_float4(us[4], us[5], us[6], us[7]);
        }
        // column half-step: v_k = b_k / sum_i Kt_ik u_i
        float p[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            float acc = kt[0][c] * us[0];
#pragma unroll
            for (int j = 1; j < RT; ++j) acc = fmaf(kt[j][c], us[j], acc);
            p[c] = acc;
        }
        float z[Slots<CT>::H2];
        wave_colsum<CT>(p, z);
        float* pp = part + (it & 1) * 64 * W;
        put_partials<CT, W>(t, z, pp);
        __syncthreads();
        const float tot = team_total<CT, W>(t, pp);
        vd = live ? bk * rcp(fmaxf(tot, kTiny)) : 0.f;
        const bool bad = __builtin_amdgcn_ballot_w64(live && !(vd >= kScaleLo && vd <= kScaleHi)) != 0;
        if (bad || (a.absorb > 0 && it % a.absorb == 0)) {
            // absorb the scalings into the potentials; rebuild Kt (log-domain step)
            if (live) gd += lg2(vd);
            vd = live ? 1.f : 0.f;
#pragma unroll
            for (int j = 0; j < RT; ++j) {
                ph[j] += lg2(us[j]);
                us[j] = 1.f;
            }
            float val[2] = {vd, gd}, out[2][CT];
            spread_cols<CT, 2>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                v[c] = out[0][c];
                gam[c] = out[1][c];
            }
            tile_rebuild<CT, RT, W>(a.C, u, I, m, a.c2, t, off, gam, ph, kt);
            if (store && it < a.T) put_stretch(it + 1);
        } else {
            float val[1] = {vd}, out[1][CT];
            spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
            for (int c = 0; c < CT; ++c) v[c] = out[0][c];
        }
        if (hist) {   // checkpoints every K iterations and the last (a countdown, not a division)
            if (--kleft == 0) {
                kleft = a.K;
                ++kc;
                put_hist(hist + (int64_t)kc * a.hs);
            } else if (it == a.T) {
                put_hist(hist + (int64_t)(a.nck - 1) * a.hs);
            }
        }
    }

    if (store && threadIdx.x == 0) rv.sep[0] = nst;

    // epilogue: X = Kt v u, y_i = r_i sum_{k < m-1} e_k x_ik, potentials
    const int mo = m;
    float ek[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int k = t.cg * CT + c;
        ek[c] = (k < mo - 1) ? a.e[k] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        const bool valid = i < I;
        const int64_t row = u * I + (valid ? i : 0);
        float yy = 0.f;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int k = t.cg * CT + c;
            const float x = (kt[j][c] * v[c]) * us[j];
            yy = fmaf(ek[c], x, yy);
            if (a.X && valid && k < mo) {
                if (a.x_bf16)
                    ((uint16_t*)a.X)[row * mo + k] = to_bf16(x);
                else
                    ((float*)a.X)[row * mo + k] = x;
            }
        }
        yy = quad_sum(yy);
        if (valid && t.cg == 0) {
            if (a.y) a.y[row] = a.r[row] * yy;
            const float phi = ph[j] + lg2(us[j]) - off[j];
            if (a.pot) a.pot[u * (int64_t)(I + mo) + i] = phi * a.eps_ln2;
        }
    }
    if (a.pot && t.w == 0 && live) a.pot[u * (int64_t)(I + mo) + I + t.rcol] = (gd + lg2(vd)) * a.eps_ln2;
}

// ---------------------------------------------------------------------------
// Factors for the contraction's BF16 matrix products.  Each FP32 factor x is
// split into three BF16 pieces, x = hi + mid + lo to within 2^-24 |x| (each
// piece is the rounding of what the previous ones leave, and every such
// remainder is exact in FP32), so that the six products hi hi, hi mid, mid hi,
// hi lo, mid mid, lo hi carry the FP32 product to about 2^-24.  Slots are
// taken in groups of 8; the K index of slot 8 g + 4 h + j, factor f, within
// group g is 8 h + 2 j + f, which is what lane 32 h + c supplies as element
// 2 j + f of its operand in v_mfma_f32_32x32x16_bf16.  The sweep writes the
// column factors in FP32, [slot][factor][64 columns] (slots T + 1 .. 8 G - 1
// zero); the contraction splits each group's into LDS, where word
// bcol_lds(p, h, c, j) holds piece p of (factor 0, factor 1) of slot
// 8 g + 4 h + j, column c, factor 0 in the low half, so that a lane reads its
// operand of one piece with one 16-byte load.
__host__ __device__ constexpr int tile_bgroups(int T) { return (T + 8) / 8; }
__host__ __device__ constexpr size_t tile_bcol_floats(int T) {
    return (size_t)tile_bgroups(T) * 8 * 2 * 64;
}
__device__ __forceinline__ int bcol_lds(int p, int h, int c, int j) { return ((p * 2 + h) * 64 + c) * 4 + j; }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// (x0, x1) = p[0] + p[1] + p[2], each word a pair of BF16 rounded to nearest
// (x0 in the low half).
__device__ __forceinline__ void bf16_split3(float x0, float x1, uint32_t (&p)[3]) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const f32x2 v = {x0, x1};
        const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
        p[q] = w;
        x0 -= __builtin_bit_cast(float, w << 16);
        x1 -= __builtin_bit_cast(float, w & 0xffff0000u);
    }
}

// the column factors (w0, w1) of slot s, column c
__device__ __forceinline__ void put_bcol(float* Bf, int s, int c, float w0, float w1) {
    Bf[(size_t)(2 * s) * 64 + c] = w0;
    Bf[(size_t)(2 * s + 1) * 64 + c] = w1;
}

// ---------------------------------------------------------------------------
// Per-consumer area of the tile buffer (TileBuf in fr_internal.h).
struct TileView {
    float* A1;     // [T+1][IP]  first row factor u per iteration (slot T: initial term), in
                   // lane order like the row store, which holds it instead when it is kept
    float* A2;     // [T+1][IP]  second row factor u fbar, in lane order
    float* Bf;     // [8 G][2][64]  column factors (w gh, w) per slot; slots past T zero
    float* rho;   // [kTileEpochs][64]  reference column potentials
    float* phi;   // [kTileEpochs][IP]  reference row offsets
    float* off;   // [IP]  row centring offsets of the scaled costs
    int* ep;      // [kTileEpochs + 1]: ep[0] = number of stretches, ep[1 + e] = first t of stretch e
    float* cb;    // [IP][64]  running cost adjoint when a consumer has several stretches
};

__device__ __forceinline__ TileView tile_view(const TileBuf& tb, int64_t b, int T, int IP) {
    char* base = tb.base + b * tb.stride;
    TileView v;
    size_t o = 0;
    v.A1 = (float*)(base + o);
    o += sizeof(float) * (size_t)(T + 1) * IP;
    v.A2 = (float*)(base + o);
    o += sizeof(float) * (size_t)(T + 1) * IP;
    v.Bf = (float*)(base + o);
    o += sizeof(float) * tile_bcol_floats(T);
    v.rho = (float*)(base + o);
    o += sizeof(float) * (size_t)kTileEpochs * 64;
    v.phi = (float*)(base + o);
    o += sizeof(float) * (size_t)kTileEpochs * IP;
    v.off = (float*)(base + o);
    o += sizeof(float) * (size_t)IP;
    v.ep = (int*)(base + o);
    o += sizeof(int) * (size_t)(kTileEpochs + 1);
    o = (o + 255) / 256 * 256;
    v.cb = (float*)(base + o);
    return v;
}

// Reference kernel of a new stretch: Kt = 2^(a + rho + phi), phi_i putting
// each row's largest entry at 1 (quad max of a + rho); rho is kNeg on padded
// columns, off kBig on rows beyond I (phi 0 there).
template <int CT, int RT, int W>
__device__ __forceinline__ void tile_reference(const float* C, int64_t u, int I, int m, float c2,
                                               const TLane<CT, W>& t, const float (&off)[RT],
                                               const float (&rho)[CT], float (&phr)[RT],
                                               float (&kt)[RT][CT]) {
    constexpr int RG = 16 * W;
    const int Io = opaque_s(I), mo = opaque_s(m);
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        const float* src = C + (u * Io + (i < Io ? i : 0)) * (int64_t)mo;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int k = t.cg * CT + c;
            kt[j][c] = src[k < mo ? k : mo - 1];
        }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        float mx = kNeg;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            kt[j][c] = fmaf(kt[j][c], c2, -off[j]) + rho[c];
            mx = fmaxf(mx, kt[j][c]);
        }
        mx = quad_max(mx);
        phr[j] = (i < Io) ? -mx : 0.f;
#pragma unroll
        for (int c = 0; c < CT; ++c) kt[j][c] = ex2(kt[j][c] + phr[j]);
    }
}

// The reverse sweep.  STORED: the forward kept this consumer's row scalings
// and the references of its stretches (RowStore); the sweep then works in the
// forward's stretches, rebuilds each stretch's kernel from the stored
// references (bit for bit the forward's) and takes u_i from the store instead
// of forming the row sums sum_k Kt_ik w_k.  Otherwise it forms them and
// chooses its own references (rebasing where a w leaves [2^-32, 2^32]).
template <int CT, int RT, int W, bool STORED>
__global__ __launch_bounds__(64 * W) void k_tbwd(BwdArgs a, TileBuf tb, int64_t u0, int nb) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    constexpr int RG = 16 * W;
    constexpr int IP = RT * RG;
    const TLane<CT, W> t;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const int64_t u = u0 + b;
    const int I = a.I, m = a.m, T = a.T;
    float* part = smem;                          // [2][64][W]
    float* vb = smem + 2 * 64 * W + t.w * 256;   // this wave's [4][64]
    float* seg = smem + 2 * 64 * W + W * 256;    // [kLoadBlock + 1][64]
    const TileView tv = tile_view(tb, b, T, IP);
    const float* hist = a.hist + u * (int64_t)a.nck * a.hs;
    const int hs = a.hs;
    RowView rv{};
    int f = 0, fstart = 1;   // STORED: the forward's stretch of the current iteration, its first iteration
    float rhod_prev = 0.f;   // STORED: the column potential of stretch f - 1 (reducing lanes)
    if constexpr (STORED) {
        rv = row_view(a.rows, u, T, IP);
        f = __builtin_amdgcn_readfirstlane(rv.sep[0]) - 1;
        if (f >= kTileEpochs) {   // more stretches than the store keeps
            if (threadIdx.x == 0) {
                atomicOr(a.flags, FLAG_EPOCHS);
                tv.ep[0] = 0;
            }
            return;
        }
    }

    float kt[RT][CT], off[RT], om[RT];
    tile_load<CT, RT, W>(a.C, u, I, m, a.c2, t, kt, off, om);
    float rg[RT];   // gF r_i / Imp_i
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int i = j * RG + t.rg;
        rg[j] = (i < I) ? (float)(a.gF * (double)a.r[u * I + i] / a.imp[i]) : 0.f;
        if (t.cg == 0) tv.off[i] = off[j];
    }

    // the reducing lane's column
    const bool live = t.rcol >= 0 && t.rcol < m;
    const float ibc = live ? ((t.rcol == m - 1) ? 1.f / (float)(I - m + 1) : 1.f) : 0.f;
    const float ekd = (live && t.rcol < m - 1) ? a.e[t.rcol] : 0.f;
    float gbar = 0.f, rhod = 0.f;

    // segment of potentials gamma^{t0} .. gamma^{t1} in LDS (every iterate kept)
    int seg_t0 = -1;
    auto load_seg = [&](int tt) __attribute__((always_inline)) {   // block containing gamma^{tt-1}, gamma^{tt}
        const int t0 = ((tt - 1) / kLoadBlock) * kLoadBlock;
        if (t0 == seg_t0) return;
        __syncthreads();
        const int n = min(kLoadBlock, T - t0);
        for (int idx = threadIdx.x; idx < (n + 1) * 64; idx += blockDim.x) {
            const int qq = idx >> 6, k = idx & 63;
            seg[idx] = (k < hs) ? hist[(int64_t)(t0 + qq) * hs + k] : kNeg;
        }
        __syncthreads();
        seg_t0 = t0;
    };
    auto gam_at = [&](int tt) { return seg[(tt - seg_t0) * 64 + (t.rcol >= 0 ? t.rcol : 0)]; };

    // A stretch of the sweep: reference column potentials rho (rhod on the
    // reducing lanes) and row offsets phr; recorded for the contraction as
    // stretch ne, which starts (in the sweep's order) at iteration tt.
    int ne = 0;
    float phr[RT];
    auto record = [&](int tt) __attribute__((always_inline)) {
        const int e = ne < kTileEpochs ? ne : kTileEpochs - 1;
        if (ne >= kTileEpochs && threadIdx.x == 0) atomicOr(a.flags, FLAG_EPOCHS);
        if (t.w == 0 && t.rcol >= 0) tv.rho[e * 64 + t.rcol] = live ? rhod : 0.f;
#pragma unroll
        for (int j = 0; j < RT; ++j)
            if (t.cg == 0) tv.phi[e * IP + j * RG + t.rg] = phr[j];
        if (threadIdx.x == 0) tv.ep[1 + e] = tt;
        ne = (ne < kTileEpochs) ? ne + 1 : ne;
    };
    // own reference: rho = rhod, each row's largest entry at 1
    auto new_stretch = [&](int tt) __attribute__((always_inline)) {
        float val[1] = {live ? rhod : kNeg}, out[1][CT];
        spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
        tile_reference<CT, RT, W>(a.C, u, I, m, a.c2, t, off, out[0], phr, kt);
        record(tt);
    };
    // the forward's stretch f: its column potentials (kNeg on padded columns)
    // and row offsets; rhod must hold its potential on the live columns
    auto stored_stretch = [&](int tt) __attribute__((always_inline)) {
        float val[1] = {t.rcol >= 0 ? rv.gam[f * 64 + t.rcol] : kNeg}, out[1][CT];
        spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
        const float4* src = (const float4*)(rv.ph + ((size_t)f * RG + t.rg) * RT);
#pragma unroll
        for (int q = 0; q < RT / 4; ++q) {
            const float4 x = src[q];
            phr[4 * q] = x.x;
            phr[4 * q + 1] = x.y;
            phr[4 * q + 2] = x.z;
            phr[4 * q + 3] = x.w;
        }
        tile_rebuild<CT, RT, W>(a.C, u, I, m, a.c2, t, off, out[0], phr, kt);
        record(tt);
        // (consumed here, so that no later wait for memory counts these loads)
        fstart = __builtin_amdgcn_readfirstlane(rv.sep[1 + f]);
        rhod_prev = opaque_f((f > 0 && live) ? rv.gam[(f - 1) * 64 + t.rcol] : 0.f);
    };
    // the forward's u_i of iteration tt (0 on rows beyond I)
    auto load_u = [&](int tt, float (&x)[RT]) __attribute__((always_inline)) {
        const float4* src = (const float4*)(rv.us + ((size_t)(tt - 1) * RG + t.rg) * RT);
#pragma unroll
        for (int q = 0; q < RT / 4; ++q) {
            const float4 v4 = src[q];
            x[4 * q] = v4.x;
            x[4 * q + 1] = v4.y;
            x[4 * q + 2] = v4.z;
            x[4 * q + 3] = v4.w;
        }
    };

    load_seg(T);
    float ucur[RT], unext[RT];
    if constexpr (STORED) {
        rhod = live ? rv.gam[f * 64 + t.rcol] : 0.f;
        stored_stretch(T);
        load_u(T, ucur);
    } else {
        rhod = live ? gam_at(T - 1) : 0.f;   // first reference: rho = gamma^{T-1}
        new_stretch(T);
    }

    // Column values of iteration T for the reducing lanes: w = 2^(gamma^{T-1}
    // - rho) and xr = 2^(gamma^T - gamma^{T-1}) = b / sig^T; w spread to the
    // lanes' columns (ow).
    float wd, xr, ow[CT];
    {
        const float gp = live ? gam_at(T - 1) : kNeg, gq = live ? gam_at(T) : kNeg;
        wd = live ? ex2(gp - rhod) : 0.f;
        xr = live ? ex2(gq - gp) : 0.f;
        float val[1] = {wd}, out[1][CT];
        spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
        for (int c = 0; c < CT; ++c) ow[c] = out[0][c];
    }

    // initial term (t = T): X = P^T diag(b / sig^T); cbar = -G X / eps
    float fb0[RT];
    float gmul;   // factor of the next team total: ev for the initial term, then -w
    {
        const float ev = ekd * wd * xr;
        float val[1] = {ev}, out[1][CT];
        spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
        float qr[RT];
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            float s = 0.f, xe = 0.f;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if constexpr (!STORED) s = fmaf(kt[j][c], ow[c], s);
                xe = fmaf(kt[j][c], out[0][c], xe);
            }
            xe = quad_sum(xe);
            float qj;   // 1 / (eps s_i)
            if constexpr (STORED)
                qj = (om[j] > 0.f) ? a.inv_eps * ucur[j] : 0.f;
            else
                qj = (om[j] > 0.f) ? a.inv_eps * rcp(quad_sum(s)) : 0.f;
            const float xs = qj * xe;   // sum_k e_k x_ik / eps
            fb0[j] = rg[j] * xs;
            qr[j] = rg[j] * qj;
            const int i = j * RG + t.rg;
            if (t.cg == 0 && a.dr && i < I) a.dr[u * I + i] = (float)(a.gF / a.imp[i]) * (xs / a.inv_eps);
        }
        {   // slot T: the initial term's row factors (-G / (eps s_i), 0), in lane order
            static_assert(RT == 8, "a lane's rows are two 16-byte words");
            float* a1 = (STORED ? rv.us : tv.A1) + (size_t)T * IP + t.rg * RT;
            float* a2 = tv.A2 + (size_t)T * IP + t.rg * RT;
            *(float4*)a1 = make_float4(-qr[0], -qr[1], -qr[2], -qr[3]);
            *(float4*)(a1 + 4) = make_float4(-qr[4], -qr[5], -qr[6], -qr[7]);
            *(float4*)a2 = make_float4(0.f, 0.f, 0.f, 0.f);
            *(float4*)(a2 + 4) = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (t.w == 0 && t.rcol >= 0) {   // slot T, then the group's unused slots (zero)
            put_bcol(tv.Bf, T, t.rcol, ev, 0.f);
            for (int s = T + 1; s < 8 * tile_bgroups(T); ++s) put_bcol(tv.Bf, s, t.rcol, 0.f, 0.f);
        }
        float p[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < RT; ++j) acc = fmaf(kt[j][c], qr[j], acc);
            p[c] = acc;
        }
        float z[Slots<CT>::H2];
        wave_colsum<CT>(p, z);
        put_partials<CT, W>(t, z, part);
        gmul = ev;
    }

    // reverse sweep t = T .. 1.  Each pass starts at the barrier that completes
    // the previous pass's column partials; the team-total reads and the next
    // pass's potentials are issued together, the row sums (which need only w)
    // are formed while they are in flight, and the pass's w gh and the next
    // pass's w are spread in one exchange.
    int par = 0;
    for (int tt = T; tt >= 1; --tt) {
        __syncthreads();
        const float* pp = part + par * 64 * W;
        float x[W];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = pp[w * 64 + t.pslot];
        const bool more = tt > 1;
        const bool same_seg = more && tt - 2 >= seg_t0;
        float gp_n = 0.f, gq_n = 0.f;
        if (same_seg) {
            gp_n = live ? gam_at(tt - 2) : kNeg;
            gq_n = live ? gam_at(tt - 1) : kNeg;
        }
        if constexpr (STORED) {
            if (more) load_u(tt - 1, unext);
        }
        __builtin_amdgcn_sched_barrier(0);
        float uj[RT];
        if constexpr (STORED) {
            // rows beyond I: the forward's u is finite (its row sums start
            // from kTiny) and their Kt is 0, so every product with it is 0
#pragma unroll
            for (int j = 0; j < RT; ++j) uj[j] = ucur[j];
        } else {
            float sr[RT];
#pragma unroll
            for (int j = 0; j < RT; ++j) sr[j] = 0.f;
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int j = 0; j < RT; ++j) sr[j] = fmaf(kt[j][c], ow[c], sr[j]);
#pragma unroll
            for (int j = 0; j < RT; ++j) uj[j] = (om[j] > 0.f) ? rcp(quad_sum(sr[j])) : 0.f;
        }
        __builtin_amdgcn_sched_barrier(0);
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < W; ++w) tot += x[w];
        gbar = gmul * tot;
        const float gh = live ? gbar * xr * ibc : 0.f;   // gbar / sig^t
        const float wg = wd * gh;
        // the next pass's column values (a new stretch is started after this
        // pass's column sums, which still need the current reference)
        float wd_n = 0.f, xr_n = 0.f, rhod_n = rhod;
        bool restart = false;
        if (more) {
            if (!same_seg) {
                load_seg(tt - 1);
                gp_n = live ? gam_at(tt - 2) : kNeg;
                gq_n = live ? gam_at(tt - 1) : kNeg;
            }
            if constexpr (STORED) {
                restart = tt - 1 < fstart;   // iteration tt - 1 lies in the forward's stretch f - 1
                if (restart) rhod_n = rhod_prev;
                wd_n = live ? ex2(gp_n - rhod_n) : 0.f;
            } else {
                wd_n = live ? ex2(gp_n - rhod) : 0.f;
                restart = __builtin_amdgcn_ballot_w64(live && !(wd_n >= kScaleLo && wd_n <= kScaleHi)) != 0 ||
                          (a.absorb > 0 && (T - tt + 1) % a.absorb == 0);
            }
            xr_n = live ? ex2(gq_n - gp_n) : 0.f;
        }
        float og[CT], ow_n[CT];
        {
            float val[2] = {wg, wd_n}, out[2][CT];
            spread_cols<CT, 2>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                og[c] = out[0][c];
                ow_n[c] = out[1][c];
            }
        }
        float aa[RT];
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < CT; ++c) d = fmaf(kt[j][c], og[c], d);
            d = quad_sum(d);
            const float fb = (tt == T ? fb0[j] : 0.f) - uj[j] * d;
            aa[j] = uj[j] * fb;
        }
        // the row factors of slot tt - 1 in lane order: u fbar, and u itself
        // unless the row store holds it.  The quad's four lanes hold the same
        // eight values and each stores them all (no branch: the wait for a
        // load issued earlier in the pass can then count these stores).
        {
            static_assert(RT == 8, "a lane's rows are two 16-byte words");
            float* a2 = tv.A2 + (size_t)(tt - 1) * IP + t.rg * RT;
            *(float4*)a2 = make_float4(aa[0], aa[1], aa[2], aa[3]);
            *(float4*)(a2 + 4) = make_float4(aa[4], aa[5], aa[6], aa[7]);
            if constexpr (!STORED) {
                float* a1 = tv.A1 + (size_t)(tt - 1) * IP + t.rg * RT;
                *(float4*)a1 = make_float4(uj[0], uj[1], uj[2], uj[3]);
                *(float4*)(a1 + 4) = make_float4(uj[4], uj[5], uj[6], uj[7]);
            }
        }
        if (t.w == 0 && t.rcol >= 0) put_bcol(tv.Bf, tt - 1, t.rcol, wg, wd);
        if (!more) break;   // gbar after the first iteration is not needed
        float p[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < RT; ++j) acc = fmaf(kt[j][c], aa[j], acc);
            p[c] = acc;
        }
        float z[Slots<CT>::H2];
        wave_colsum<CT>(p, z);
        par ^= 1;
        put_partials<CT, W>(t, z, part + par * 64 * W);
        gmul = -wd;
        wd = wd_n;
        xr = xr_n;
#pragma unroll
        for (int c = 0; c < CT; ++c) ow[c] = ow_n[c];
        if constexpr (STORED) {
#pragma unroll
            for (int j = 0; j < RT; ++j) ucur[j] = unext[j];
            if (restart) {
                --f;
                rhod = rhod_n;
                stored_stretch(tt - 1);
            }
        } else if (restart) {
            rhod = live ? gp_n : 0.f;
            new_stretch(tt - 1);
            wd = live ? 1.f : 0.f;
            float val[1] = {wd}, out[1][CT];
            spread_cols<CT, 1>(vb, t.rslot, t.rcol >= 0, val, t.cg, out);
#pragma unroll
            for (int c = 0; c < CT; ++c) ow[c] = out[0][c];
        }
    }
    if (threadIdx.x == 0) tv.ep[0] = ne;
}

// ---------------------------------------------------------------------------
// Contraction of the sweep's factors.  Block (b, rb): 4 waves, wave v takes
// the row tiles 2 (4 rb + v) and 2 (4 rb + v) + 1 (64 rows) of consumer
// u0 + b, counted in the row factors' lane order (row S = rg RT + j is plan
// row j RG + rg), and both 32-column tiles.  Per stretch it sums, over the
// stretch's slots s and factors f, A[s][f][i] B[s][f][k] with
// v_mfma_f32_32x32x16_bf16 on the three-piece BF16 split of both factors (six
// products, see bf16_split3): a group of 8 slots is 16 K values, 24 MFMAs per
// wave.  Both factors are read in FP32 and split here, the column factors
// once per block as they are staged in LDS.
// Result lane layout of the 32x32 MFMAs (checked on the device): lane l
// holds D[row][l % 32] for row = (v % 4) + 8 (v / 4) + 4 (l / 32), v < 16;
// in the x16 BF16 form lane l supplies A[l % 32][8 (l / 32) + q] and
// B[8 (l / 32) + q][l % 32] as its operand elements q < 8.
typedef float f32x16 __attribute__((ext_vector_type(16)));

// row of result v of lane l, formed where it is used (the lane's part opaque, so
// that the epilogue's 32 row indices are not hoisted and kept live across the
// MFMA loop)
__device__ __forceinline__ int mfma_row_here(int v, int l) { return (v & 3) + 8 * (v >> 2) + opaque_v(4 * (l >> 5)); }

// Raw buffer resources (stride 0): a load at a byte offset at or past n reads
// 0 and a store there is dropped (the update epilogue sends the cells outside
// a consumer's block there).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t buf_rsrc(const void* base, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)n, 0x00020000);
}
constexpr int kOffNone = 0x7ffffff0;   // past every range used here

// Row-factor operands of one group of 8 slots, loaded raw: the lane's 4 slots
// (both row tiles, both factors) in FP32; the MFMAs mask slots outside the
// stretch.  A1p, A2p: the two row factors + (row of tile 0); slots past T are
// read at T.  The factors are read once, as a stream (non-temporal: they do
// not displace the column factors and costs from the caches).
struct GOpd {
    float a[2][4][2];   // [row tile][slot 4 h + j][factor]
};
template <int IP>
__device__ __forceinline__ void load_ga(GOpd& o, const float* A1p, const float* A2p, int g, int h, int T) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int sl = min(8 * g + 4 * h + j, T);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            o.a[r][j][0] = __builtin_nontemporal_load(A1p + (size_t)sl * IP + 32 * r);
            o.a[r][j][1] = __builtin_nontemporal_load(A2p + (size_t)sl * IP + 32 * r);
        }
    }
}

// The column factors of a group are the same for the block's 4 waves: they
// are split once per group into LDS (two buffers of 1536 words, bcol_lds).
// Wave v takes the two slots 8 g + 4 h + 2 jp + {0, 1} (h = v & 1, jp = v / 2)
// of column l: four FP32 loads, two splits, three 8-byte LDS writes.
struct GBc {
    float v[2][2];   // [slot][factor]
};
__device__ __forceinline__ void load_gbc(GBc& o, const float* Bf, int g, int wv, int l) {
    const int s0 = 8 * g + 4 * (wv & 1) + 2 * (wv >> 1);
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int f = 0; f < 2; ++f) o.v[jj][f] = Bf[(size_t)(2 * (s0 + jj) + f) * 64 + l];
}
__device__ __forceinline__ void store_gbc(const GBc& o, uint32_t* dst, int wv, int l) {
    uint32_t w[2][3];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) bf16_split3(o.v[jj][0], o.v[jj][1], w[jj]);
#pragma unroll
    for (int pc = 0; pc < 3; ++pc) {
        const u32x2 x = {w[0][pc], w[1][pc]};
        *(u32x2*)(dst + bcol_lds(pc, wv & 1, l, 2 * (wv >> 1))) = x;
    }
}
// A block barrier that waits for this wave's LDS operations only, so that
// its row-factor loads in flight stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The epilogue needs the costs of the wave's 64 rows (the reference kernel
// Kt = 2^(c c2 - off + rho + phi) is rebuilt from them): they are copied into
// LDS by direct global-to-LDS loads issued at the start, which complete while
// the MFMAs run and occupy no registers.  The kernel writes dF/dC: into dC
// when it is asked for, else into the batch's gradient buffer, from which
// the last stretch's epilogue applies the update.

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// The linear block id is mapped so that the NRB row blocks of one consumer
// share an XCD and are dispatched close together: id = (b / 8) * 8 NRB +
// rb * 8 + b % 8, so that the consumer's column factors are read from HBM
// once and then hit that XCD's L2.
constexpr int kXcds = 8;

typedef float __attribute__((address_space(1))) gfloat;
typedef float __attribute__((address_space(3))) lfloat;

// MODE 0 writes gF dF/dC (into dC, or into the batch's gradient buffer);
// MODE 1 applies Adam and MODE 2 plain ascent to C (and Adam's moments) with
// the finished gradient in the epilogue of the last stretch, reading the
// costs from the LDS copy and Adam's moments ahead of their use.
template <int IP, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tgrad(
    BwdArgs a, TileBuf tb, int64_t u0, int nb, int stored) {
    extern __shared__ float smem[];
    if (a.stop && *a.stop) return;   // the outer loop has ended
    constexpr int NRB = (IP + 255) / 256;   // row blocks per consumer (grid: 8 NRB blocks per 8 consumers)
    const int id = blockIdx.x;
    const int grp = id / (kXcds * NRB), rem = id - grp * (kXcds * NRB);
    const int rb = rem / kXcds;
    const int b = grp * kXcds + (rem - rb * kXcds);
    if (b >= nb) return;
    const int64_t u = u0 + b;
    const int l = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform in the wave
    const int rt0 = (rb * 4 + wv) * 2;   // first row tile, in the row factors' lane order
    const int I = a.I, m = a.m, T = a.T;
    const TileView tv = tile_view(tb, b, T, IP);
    // plan row of lane-order row S (S = rg RT + j holds row j RG + rg, RT = 8);
    // every wave's 64 rows include rows below 4 RG = IP / 2 < I
    auto prow = [](int S) { return (S & 7) * (IP / 8) + (S >> 3); };
    const int col = l & 31;
    const int half = l >> 5;
    const bool c0ok = col < m, c1ok = 32 + col < m;

    // this wave's LDS: the costs of its rows (row-major, m per row), then the
    // row term phi - off of the current stretch
    float* cl = smem + wv * (64 * m + 64);
    float* bl = cl + 64 * m;
    uint32_t* bsh = (uint32_t*)(smem + 4 * (64 * m + 64));   // [2][6 chunks][256 words]
    // The wave's 64 rows are 8 runs j = 0..7 of 8 consecutive plan rows
    // j RG + rg0 .. j RG + rg0 + 7: copied run by run into LDS rows 8 j .. 8 j + 7
    // (lane-order row S0 + 8 r + j sits in LDS row 8 j + r)
    for (int j = 0; j < 8; ++j) {
        const int i0 = j * (IP / 8) + rt0 * 4;
        const int len = min(8, I - i0) * m;   // floats (none for a run past I)
        const float* src = a.C + (u * I + i0) * (int64_t)m;
        for (int o = 0; o < len; o += 64) {
            if (o + l < len)
                __builtin_amdgcn_global_load_lds((const gfloat*)(src + o + l), (lfloat*)(cl + j * 8 * m + o), 4,
                                                 0, 0);
        }
    }
    auto crow = [](int il) { return (il & 7) * 8 + (il >> 3); };   // LDS row of the wave's row il
    const float* A1p = (stored ? row_view(a.rows, u, T, IP).us : tv.A1) + rt0 * 32 + col;
    const float* A2p = tv.A2 + rt0 * 32 + col;
    const int ne = min(tv.ep[0], kTileEpochs);
    float* gout = a.dC ? a.dC + u * (int64_t)I * m : tv.cb;   // [I][m]

    for (int e = 0; e < ne; ++e) {
        const int hi = tv.ep[1 + e];                    // first (largest) t of the stretch
        const int lo = (e + 1 < ne) ? tv.ep[2 + e] : 0; // first t of the next stretch
        // slots lo .. hi-1 (iterations lo+1 .. hi), then the initial term in stretch 0
        // groups g0 .. g1-1 hold slots lo .. hi-1; slot T (the initial term,
        // stretch 0) may sit in a group of its own after them
        const int g0 = lo >> 3;
        const int g1 = hi > lo ? ((hi - 1) >> 3) + 1 : g0;
        const int ng = g1 - g0 + ((e == 0 && (T >> 3) >= g1) ? 1 : 0);
        auto grp = [&](int q) { return q < g1 - g0 ? g0 + q : (T >> 3); };
        f32x16 acc[2][2] = {};
        auto mfma_grp = [&](const GOpd& o, const uint32_t* bb, int q) __attribute__((always_inline)) {
            const int g = grp(q);
            u32x4 bv[2][3];
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int pc = 0; pc < 3; ++pc)
                    bv[ct][pc] = *(const u32x4*)(bb + bcol_lds(pc, half, ct * 32 + col, 0));
            bool ok[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int sl = 8 * g + 4 * half + j;
                ok[j] = (sl >= lo && sl < hi) || (e == 0 && sl == T);
            }
            // per row tile: split its factors, then the six products, smallest
            // first: lo hi, mid mid, hi lo, mid hi, hi mid, hi hi
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                uint32_t pa[3][4];   // [piece][word j]
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint32_t w[3];
                    bf16_split3(ok[j] ? o.a[r][j][0] : 0.f, ok[j] ? o.a[r][j][1] : 0.f, w);
#pragma unroll
                    for (int pc = 0; pc < 3; ++pc) pa[pc][j] = w[pc];
                }
                constexpr int kPa[6] = {2, 1, 0, 1, 0, 0}, kPb[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
                for (int pr = 0; pr < 6; ++pr) {
                    const u32x4 av = {pa[kPa[pr]][0], pa[kPa[pr]][1], pa[kPa[pr]][2], pa[kPa[pr]][3]};
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[r][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv[ct][kPb[pr]]),
                            acc[r][ct], 0, 0, 0);
                }
            }
        };
        // two operand buffers (registers for the row factors, LDS for the
        // column factors), alternating: one group's loads are in flight while
        // the other group's MFMAs run, and its column chunks are written to
        // the free LDS buffer after them (the barrier that follows also
        // ensures that every wave is done reading that buffer's previous
        // group).  The loop body has no branch (a load skipped on one path
        // would make the wait before the next MFMAs count every load in
        // flight); its last loads read a group past the stretch, which is not
        // used.  Every wave of the block runs the same groups.
        if (ng > 0) {
            GOpd p0, p1;
            GBc bc;
            load_gbc(bc, tv.Bf, grp(0), wv, l);
            load_ga<IP>(p0, A1p, A2p, grp(0), half, T);
            store_gbc(bc, bsh, wv, l);
            lds_barrier();
            int q = 0;
            for (; q + 1 < ng; q += 2) {
                load_gbc(bc, tv.Bf, grp(q + 1), wv, l);
                load_ga<IP>(p1, A1p, A2p, grp(q + 1), half, T);
                __builtin_amdgcn_sched_barrier(0);
                mfma_grp(p0, bsh, q);
                __builtin_amdgcn_sched_barrier(0);
                store_gbc(bc, bsh + 1536, wv, l);
                lds_barrier();
                load_gbc(bc, tv.Bf, grp(q + 2), wv, l);
                load_ga<IP>(p0, A1p, A2p, grp(q + 2), half, T);
                __builtin_amdgcn_sched_barrier(0);
                mfma_grp(p1, bsh + 1536, q + 1);
                __builtin_amdgcn_sched_barrier(0);
                store_gbc(bc, bsh, wv, l);
                lds_barrier();
            }
            if (q < ng) mfma_grp(p0, bsh, q);
            lds_barrier();   // the buffers are free before the next stretch writes them
        }
        // the stretch's row term phi - off of the wave's 64 rows
        {
            const int i = prow(rt0 * 32 + l);
            bl[l] = tv.phi[e * IP + i] - tv.off[i];
        }
        __builtin_amdgcn_s_waitcnt(0);   // the cost copy and the row terms are in LDS
        __builtin_amdgcn_wave_barrier();
        float rk[2] = {tv.rho[e * 64 + col], tv.rho[e * 64 + 32 + col]};
        rk[0] = c0ok ? rk[0] : kNeg;
        rk[1] = c1ok ? rk[1] : kNeg;
        // dF/dC = sum over stretches of Kt (.) acc: stretches before the last
        // add into gout, the last writes it (or applies the update)
        const bool first = e == 0, last = e + 1 == ne;
        if (MODE == 0 || !last) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    // one row of cells at a time, addresses formed here (opaque
                    // operands keep them from being hoisted and kept live)
                    const int Io = opaque_s(I), mo = opaque_s(m);
                    const int il = r * 32 + mfma_row_here(v, l);   // row within the wave's 64
                    const int i = prow(rt0 * 32 + il);
                    if (i < Io) {
                        const float base = bl[il];
                        float* gp = opaque_p(gout) + (int64_t)i * mo;
#pragma unroll
                        for (int ct = 0; ct < 2; ++ct) {
                            const int k = ct * 32 + col;
                            if (k < mo) {
                                float g = ex2(fmaf(cl[crow(il) * mo + k], a.c2, base) + rk[ct]) * acc[r][ct][v];
                                if (!first) g += gp[k];
                                gp[k] = g;
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else {
            float bc1 = 1.f, bc2 = 1.f;   // Adam's bias corrections (once per wave, uniform)
            if (MODE == 1) {
                const int64_t st = a.step_ptr ? *a.step_ptr : a.step_const;
                bc1 = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(
                    int, (float)(1.0 - pow((double)a.b1, (double)st)))));
                bc2 = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(
                    int, (float)(1.0 - pow((double)a.b2, (double)st)))));
            }
            // The consumer's [I][m] blocks of C, Adam's moments and the running
            // adjoint as buffer resources: a cell outside the block (row past
            // I, padded column) takes an offset past the range, so its loads
            // read 0 and its stores are dropped, with no branch.  The 64 cells
            // of a lane go in 8 chunks of 4 rows; each chunk's loads are issued
            // one chunk ahead of its arithmetic.
            const uint32_t nb = (uint32_t)(I * m * 4);
            const int64_t cu = u * (int64_t)I * m;
            const rsrc_t rC = buf_rsrc(a.Cw + cu, nb);
            const rsrc_t rM = buf_rsrc(MODE == 1 ? a.mom + cu : a.Cw + cu, nb);
            const rsrc_t rV = buf_rsrc(MODE == 1 ? a.vel + cu : a.Cw + cu, nb);
            const rsrc_t rG = buf_rsrc(gout, nb);
            auto cell_off = [&](int c, int q, int ct) {
                const int i = prow(rt0 * 32 + (c >> 2) * 32 + mfma_row_here((c & 3) * 4 + q, l));
                const int k = ct * 32 + col;
                return (i < I && k < m) ? (i * m + k) * 4 : kOffNone;
            };
            auto epi = [&](auto prev) __attribute__((always_inline)) {
                constexpr bool PREV = decltype(prev)::value;   // add the earlier stretches' adjoint
                float mv[2][4][2], vv[2][4][2], gq[2][4][2];
                auto load = [&](int c, int bf) __attribute__((always_inline)) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int ct = 0; ct < 2; ++ct) {
                            const int o = cell_off(c, q, ct);
                            if (MODE == 1) {
                                mv[bf][q][ct] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rM, o, 0, 0));
                                vv[bf][q][ct] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rV, o, 0, 0));
                            }
                            if (PREV)
                                gq[bf][q][ct] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rG, o, 0, 0));
                        }
                };
                load(0, 0);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (c + 1 < 8) load(c + 1, (c + 1) & 1);
                    __builtin_amdgcn_sched_barrier(0);
                    const int bf = c & 1, r = c >> 2;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int il = r * 32 + mfma_row_here((c & 3) * 4 + q, l);   // row within the wave's 64
                        const float base = bl[il];
#pragma unroll
                        for (int ct = 0; ct < 2; ++ct) {
                            const int o = cell_off(c, q, ct);
                            // cl[row m + k] stays within the wave's LDS area for k < 64
                            const float cold = cl[crow(il) * m + ct * 32 + col];
                            float g = ex2(fmaf(cold, a.c2, base) + rk[ct]) * acc[r][ct][(c & 3) * 4 + q];
                            if (PREV) g += gq[bf][q][ct];
                            float cn;
                            if (MODE == 1) {
                                const float gl = -g;   // Adam minimises -F
                                const float mn = a.b1 * mv[bf][q][ct] + (1.f - a.b1) * gl;
                                const float vn = a.b2 * vv[bf][q][ct] + (1.f - a.b2) * gl * gl;
                                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, mn), rM, o, 0, 0);
                                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, vn), rV, o, 0, 0);
                                cn = cold - a.lr * (mn / bc1) / (sqrtf(vn / bc2) + a.aeps);
                            } else {
                                cn = cold + a.lr * g;
                            }
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, cn), rC, o, 0, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            if (first)
                epi(std::false_type{});
            else
                epi(std::true_type{});
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int CT, int RT, int W>
void launch_tfwd(const FwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    (void)block;
    (void)lds;
    hipLaunchKernelGGL((k_tfwd<CT, RT, W>), dim3(grid), dim3(64 * W),
                       tile_lds_floats<W>(false) * sizeof(float), s, a);
}

// The backward in batches of tb.batch consumers: the sweep writes the factors
// of a batch into the tile buffer, the contraction consumes them.
template <int CT, int RT, int W>
void launch_tbwd(const BwdArgs& a, int grid, int block, size_t lds, hipStream_t s) {
    (void)grid;
    (void)block;
    (void)lds;
    constexpr int IP = RT * 16 * W;
    const TileBuf& tb = a.tile;
    for (int64_t u0 = 0; u0 < a.U; u0 += tb.batch) {
        const int nb = (int)((a.U - u0) < tb.batch ? (a.U - u0) : tb.batch);
        const int stored = (a.rows.base && u0 + nb <= a.rows.n) ? 1 : 0;
        if (stored)   // the forward kept these consumers' row scalings
            hipLaunchKernelGGL((k_tbwd<CT, RT, W, true>), dim3(nb), dim3(64 * W),
                               tile_lds_floats<W>(true) * sizeof(float), s, a, tb, u0, nb);
        else
            hipLaunchKernelGGL((k_tbwd<CT, RT, W, false>), dim3(nb), dim3(64 * W),
                               tile_lds_floats<W>(true) * sizeof(float), s, a, tb, u0, nb);
        constexpr int NRB = (IP + 255) / 256;
        const int groups = (nb + kXcds - 1) / kXcds;
        if (!a.dC && !a.Cw) continue;
        // dF/dC into dC when asked for, else applied to C (Adam or ascent)
        const dim3 gg(groups * kXcds * NRB);
        const size_t lds = (4 * (64 * a.m + 64) + 2 * 1536) * sizeof(float);
        if (a.dC)
            hipLaunchKernelGGL((k_tgrad<IP, 0>), gg, dim3(256), lds, s, a, tb, u0, nb, stored);
        else if (a.rule == 0)
            hipLaunchKernelGGL((k_tgrad<IP, 1>), gg, dim3(256), lds, s, a, tb, u0, nb, stored);
        else
            hipLaunchKernelGGL((k_tgrad<IP, 2>), gg, dim3(256), lds, s, a, tb, u0, nb, stored);
    }
}

}  // namespace

// Instantiated tile shapes: G = 4 lanes per row, CT columns per lane, RT rows
// per lane, W waves per block.  13 columns per lane serve 40 <= m <= 50 (the
// column classes 40, 48 and 50, whose potentials the forward writes in
// full); 8 rows per lane over 128 row groups serve 512 < I <= 1024.
struct TileShape {
    int mmin;
    TileEntry e;
};
static const TileShape kTileShapes[] = {
    {40, {50, 8 * 16 * 8, 8 * 16 * 8 / 2, &launch_tfwd<13, 8, 8>, &launch_tbwd<13, 8, 8>}},
};

const TileEntry* tile_entry(int m, int I) {
    for (const TileShape& t : kTileShapes)
        if (m >= t.mmin && m <= t.e.cmax && I <= t.e.imax && I > t.e.imin) return &t.e;
    return nullptr;
}

size_t tile_row_bytes(const TileEntry* e, int T) {
    const size_t IP = (size_t)e->imax;
    size_t o = sizeof(float) * (size_t)(T + 1) * IP;
    o += sizeof(float) * (size_t)kTileEpochs * IP;
    o += sizeof(float) * (size_t)kTileEpochs * 64;
    o += sizeof(int) * (size_t)(kTileEpochs + 1);
    return (o + 255) / 256 * 256;
}

size_t tile_consumer_bytes(const TileEntry* e, int T) {
    const size_t IP = (size_t)e->imax;
    size_t o = 0;
    o += sizeof(float) * (size_t)(T + 1) * 2 * IP;   // A1, A2
    o += sizeof(float) * tile_bcol_floats(T);
    o += sizeof(float) * (size_t)kTileEpochs * 64;
    o += sizeof(float) * (size_t)kTileEpochs * IP;
    o += sizeof(float) * IP;
    o += sizeof(int) * (size_t)(kTileEpochs + 1);
    o = (o + 255) / 256 * 256;
    o += sizeof(float) * IP * 64;
    return (o + 255) / 256 * 256;
}

}  // namespace fr
