// fr_api.hip -- host side of the fair-ranking C ABI (include/fairrank.h):
// argument validation, workspace layout, launch-configuration choice, and
// the HIP-graph driven outer loop of Algorithm 1.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/fairrank.h"
#include "../../include/fairrank_diag.h"
#include "fr_internal.h"

using namespace fr;

struct fr_ctx {
    int device = 0;
    hipStream_t own = nullptr;                           // used when the caller passes NULL
    std::map<std::pair<int, int>, std::pair<int, int>> launch;  // (I, m) -> (lanes, rows)
    bool timing = false;                                  // per-kernel event timing
    int form = FR_FORM_SCALING;                           // Sinkhorn form of the fixed-T forward
    int absorb = 0;                                       // scaling form: forced absorption period
    // batched solver: side streams (default priority) on which the column
    // classes of a phase run concurrently, and the events that fork and join them
    static constexpr int kSide = 4;
    static constexpr int kMaxClasses = 64;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxClasses] = {};
    double fwd_ms = 0.0, bwd_ms = 0.0;
    int64_t fwd_n = 0, bwd_n = 0;
    size_t max_lds = 64 * 1024;                           // LDS a block may use on the device
    bool row_store = true;     // tile plans: the forward keeps its row scalings for the sweep
    void* scratch = nullptr;   // device address of this device's fr_step_noalloc array
};

// Device memory of fr_step_noalloc, for callers that cannot allocate: the
// workspace fr_step takes from its caller (header, impacts, impact partials,
// the per-row impact contributions y) lives here instead, up to
// kScratchBytes.  Every GPU the library runs on holds one copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the device (scratch_address), never
// through the array's name.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_addr[kScratchDevices] = {};

// The device address of `scratch` on `device`, resolved once per device (the
// device must be current).  nullptr if the runtime cannot resolve it.
void* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_addr[device] = ptr;
        else (void)hipGetLastError();   // leave no sticky error for the caller's next call
    }
    return g_scratch_addr[device];
}
}  // namespace

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxItems = 4096;
constexpr int kMaxM = 64;
constexpr size_t kMaxLds = 64 * 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// HIP events released on every exit path (error returns included).
struct EventSet {
    std::vector<hipEvent_t> ev;
    explicit EventSet(size_t n) : ev(n, nullptr) {}
    hipError_t create() {
        for (auto& e : ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    ~EventSet() {
        for (auto e : ev)
            if (e) hipEventDestroy(e);
    }
};

// Runs f when the scope ends, however it ends.
template <class F>
struct OnExit {
    F f;
    ~OnExit() { f(); }
};
template <class F>
OnExit<F> on_exit(F f) { return OnExit<F>{f}; }

#define FR_TRY(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return FR_E_DEVICE;     \
    } while (0)

// ---------------------------------------------------------------- registry
struct Registry {
    std::vector<FusedEntry> all;
    Registry() {
#define FR_ADD(mp)                                               \
    {                                                            \
        int n = 0;                                               \
        const FusedEntry* p = fused_entries_##mp(&n);            \
        for (int q = 0; q < n; ++q) all.push_back(p[q]);         \
    }
        FR_MP_CLASSES(FR_ADD)
#undef FR_ADD
    }
    int mp_for(int m) const {
        int best = 1 << 30;
        for (auto& e : all)
            if (e.mp >= m && e.mp < best) best = e.mp;
        return best == (1 << 30) ? -1 : best;
    }
    const FusedEntry* find(int mp, int rows, int lb, bool wide) const {
        for (auto& e : all)
            if (e.mp == mp && e.rows == rows && e.lb == lb && e.wide == wide) return &e;
        return nullptr;
    }
    // Kernel for teams of L lanes in blocks of `block` threads.
    const FusedEntry* pick(int mp, int rows, int L, int block) const {
        const int lb = block <= 256 ? 256 : (block <= 512 ? 512 : 1024);
        return find(mp, rows, lb, L >= 64);
    }
};

const Registry& registry() {
    static Registry r;
    return r;
}

bool lanes_ok(int L) {
    if (L >= 1 && L <= 64) return (L & (L - 1)) == 0;
    return L > 64 && L <= 1024 && L % 64 == 0;
}

// Threads per block for teams of L lanes: several teams of up to one wave
// share a 256-thread block; larger teams take a block each.
int block_for(int L) { return L <= 64 ? 256 : L; }

// Launch shape of the fused kernels for one problem.
struct Shape {
    const FusedEntry* fe;
    FwdLaunch fwd;       // fixed-T forward of the context's Sinkhorn form
    BwdLaunch bwd;       // reverse sweep (the scaling form needs K = 1)
    int absorb;
    int L, R, mp, block, teams, grid;
    size_t lds_fwd, lds_bwd;
    size_t lds_cb;       // part of lds_bwd holding cost adjoints (reverse sweep fe->bwdl only)
    const TileEntry* te; // tile kernels run the forward (and the reverse sweep if tile_bwd)
    bool tile_bwd;
};

// Issue model of one Sinkhorn iteration (forward and backward) of U consumers
// with teams of L lanes and R rows per lane.  A wave issues R*MP cells at ~13
// VALU operations (~18 when the kernel recomputes the exponentials), plus the
// column reduction and update: per column log2 L butterfly steps and the
// update for teams narrower than a wave, ~4 operations per column for the
// reduce-scatter of wave-wide teams, plus an LDS exchange for teams of
// several waves.  Each of the 1024 SIMDs runs its share of the waves back to
// back, and a SIMD with a single wave hides its latencies poorly.
// scaling: both kernels run the scaling form (no recompute pass), about
// 2.5 VALU operations per cell fewer than the log domain (measured).
double model_cost(int64_t U, int mp, int L, const FusedEntry& e, bool scaling = false) {
    const double cell = scaling ? 10.5 : (e.recomp_f ? 7.0 : 5.0) + (e.recomp_b ? 11.0 : 8.0);
    double red;
    if (L < 64) {
        int lv = 0;
        while ((1 << lv) < L) ++lv;
        red = 2.0 * mp * (std::min(lv, 4) + (L > 16 ? 2 : 0) + 3.0);
    } else {
        red = 2.0 * (4.0 * mp + 10.0) + mp + (L > 64 ? 2.0 * (40.0 + L / 64) : 0.0);
    }
    // registers the backward keeps per lane (costs, cost adjoints, and a row
    // of exponentials or the recompute pass's chunk) against those its launch
    // bound leaves; every register short costs spill traffic
    const int budget = std::min(256, 131072 / e.lb);
    const int need = 2 * e.rows * mp + (e.recomp_b ? 30 : 2 * mp);
    const double spill = 1.0 + std::max(0, need - budget) / 32.0;
    const double per_wave = e.rows * mp * cell * spill + red;
    const double waves = (double)U * (L < 64 ? L / 64.0 : (double)(L / 64));
    const double per_simd = waves / 1024.0;
    return std::max(1.0, per_simd) * per_wave * (per_simd <= 1.0 ? 1.25 : 1.0);
}

std::pair<int, int> default_launch(int64_t U, int I, int m) {
    const Registry& reg = registry();
    const int mp = reg.mp_for(m);
    double best = 1e300;
    std::pair<int, int> out{0, 0};   // stays {0, 0} if no instantiated kernel holds I rows
    const int Ls[] = {8, 16, 32, 64, 128, 192, 256, 320, 384, 448, 512, 576, 640, 704,
                      768, 832, 896, 960, 1024};
    for (int L : Ls) {
        for (auto& e : reg.all) {
            if (e.mp != mp) continue;
            const int R = e.rows;
            if ((int64_t)L * R < I) continue;
            if (&e != reg.pick(mp, R, L, block_for(L))) continue;
            // no more lanes than rows need
            if ((int64_t)L * (R - 1) >= I) continue;
            const double c = model_cost(U, mp, L, e);
            if (c < best) {
                best = c;
                out = {L, R};
            }
        }
    }
    return out;
}

fr_status make_shape(fr_ctx* ctx, int64_t U, int I, int m, int K, Shape* sh) {
    const Registry& reg = registry();
    const int mp = reg.mp_for(m);
    if (mp < 0) return FR_E_UNSUPPORTED;
    std::pair<int, int> lr;
    auto it = ctx->launch.find({I, m});
    const bool pinned = it != ctx->launch.end();
    lr = pinned ? it->second : default_launch(U, I, m);
    // the tile kernels (scaling form): the default for the plans they take,
    // or a launch pinned as (512 lanes, 0 rows)
    const TileEntry* te = tile_entry(m, I);
    const bool want_tile = te && ctx->form == FR_FORM_SCALING &&
                           (pinned ? lr.second == 0 : true);
    if (pinned && lr.second == 0 && !want_tile) return FR_E_UNSUPPORTED;
    if (want_tile && lr.second == 0) lr = default_launch(U, I, m);
    const int L = lr.first, R = lr.second;
    if (L == 0) return FR_E_UNSUPPORTED;   // more rows than any instantiated kernel holds
    if (!lanes_ok(L) || (int64_t)L * R < I) return FR_E_PARAM;
    int block = block_for(L);
    const FusedEntry* fe = reg.pick(mp, R, L, block);
    if (!fe) return FR_E_UNSUPPORTED;
    const int W = (L + 63) / 64;
    const int BL = (K <= 1) ? kLoadBlock : K;
    auto per_team_bwd = [&](void) { return (size_t)((BL + 1) * mp + 2 * W * mp) * sizeof(float); };
    int teams = block / L;
    while (teams > 1 && teams * per_team_bwd() > kMaxLds) {
        teams /= 2;
    }
    if (teams * per_team_bwd() > kMaxLds) return FR_E_UNSUPPORTED;
    block = teams * L;
    sh->fe = fe;
    sh->fwd = (ctx->form == FR_FORM_SCALING && fe->fwds) ? fe->fwds : fe->fwd;
    // the scaling-form sweep where it keeps a row of products in registers; the
    // two-pass (recompute) shapes spill more in that form and keep the log domain
    sh->bwd = (ctx->form == FR_FORM_SCALING && K <= 1 && fe->bwds && !fe->recomp_b) ? fe->bwds
                                                                                    : fe->bwd;
    // wide recompute sweeps keep some rows of cost adjoints in LDS where it fits
    sh->lds_cb = 0;
    if (sh->bwd == fe->bwd && fe->bwdl) {
        const size_t cb = (size_t)teams * fe->cb_rows * mp * L * sizeof(float);
        if (teams * per_team_bwd() + cb <= ctx->max_lds) {
            sh->bwd = fe->bwdl;
            sh->lds_cb = cb;
        }
    }
    sh->te = want_tile ? te : nullptr;
    sh->tile_bwd = want_tile && K <= 1;
    if (want_tile) {
        sh->fwd = te->fwd;
        if (K <= 1) sh->bwd = te->bwd;
    }
    sh->absorb = ctx->absorb;
    sh->L = L;
    sh->R = R;
    sh->mp = mp;
    sh->block = block;
    sh->teams = teams;
    sh->grid = (int)((U + teams - 1) / teams);
    sh->lds_fwd = (size_t)teams * 2 * W * mp * sizeof(float);
    sh->lds_bwd = (size_t)teams * per_team_bwd() + sh->lds_cb;
    return FR_OK;
}

// ---------------------------------------------------------------- workspace
struct Layout {
    size_t hdr, imp, partial, y, hist, grad, gpart, gw, phi, tile, total;
    int nchunk, nck, hs;
    size_t tile_stride;    // bytes per consumer of the tile reverse sweep's buffer (0: none)
    int64_t tile_batch;    // consumers per batch
    size_t rows;           // the tile forward's row scalings for the sweep
    size_t rows_stride;    // bytes per consumer (0: none)
    int64_t rows_n;        // consumers kept: all, or whole batches within kRowStoreCap
};

int n_checkpoints(int T, int K) { return (T + K - 1) / K + 1; }

// tol: room for the gradient and its norm partials (gradient-norm stop);
// conv: the converged-map form's potentials.
Layout layout(const fr_problem* p, int K, bool tol = false, bool conv = false) {
    Layout L;
    const int64_t U = p->n_users;
    const int I = p->n_items;
    L.nchunk = impact_chunks(U, I);
    L.nck = n_checkpoints(p->sinkhorn_iters, K);
    L.hs = registry().mp_for(p->m);   // potentials padded to the column class
    size_t off = 0;
    L.hdr = off;
    off += align_up(sizeof(WsHeader));
    L.imp = off;
    off += align_up(sizeof(double) * I);
    L.partial = off;
    off += align_up(sizeof(double) * (size_t)L.nchunk * I);
    L.y = off;
    off += align_up(sizeof(float) * (size_t)U * I);
    L.hist = off;
    off += align_up(sizeof(float) * (size_t)U * L.nck * L.hs);
    L.grad = L.gpart = off;
    if (tol) {
        const int64_t n = U * (int64_t)I * p->m;
        L.grad = off;
        off += align_up(sizeof(float) * (size_t)n);
        L.gpart = off;
        off += align_up(sizeof(double) * (size_t)gnorm_blocks(n));
    }
    L.gw = L.phi = off;
    if (conv) {
        L.gw = off;
        off += align_up(sizeof(float) * (size_t)U * L.hs);
        L.phi = off;
        off += align_up(sizeof(float) * (size_t)U * I);
    }
    // the tile reverse sweep's factors, for the plans the tile kernels take
    // (whichever kernels a context then picks)
    L.tile = off;
    L.tile_stride = 0;
    L.tile_batch = 0;
    L.rows_stride = 0;
    L.rows_n = 0;
    if (K <= 1 && !conv) {
        if (const TileEntry* te = tile_entry(p->m, I)) {
            L.tile_stride = tile_consumer_bytes(te, p->sinkhorn_iters);
            L.tile_batch = std::min<int64_t>(U, kTileBatch);
            off += align_up(L.tile_stride * (size_t)L.tile_batch);
            L.rows_stride = tile_row_bytes(te, p->sinkhorn_iters);
            const int64_t fit = (int64_t)(kRowStoreCap / L.rows_stride);
            L.rows_n = U <= fit ? U : fit / L.tile_batch * L.tile_batch;
        }
    }
    L.rows = off;
    off += align_up(L.rows_stride * (size_t)L.rows_n);
    L.total = off;
    return L;
}

fr_status check_problem(const fr_problem* p) {
    if (!p) return FR_E_NULL;
    if (p->n_users < 1 || p->n_items < 2 || p->n_items > kMaxItems || p->m < 2 ||
        p->m > p->n_items || p->m > kMaxM)
        return FR_E_SHAPE;
    if (!(p->eps > 0.f) || !isfinite(p->eps) || p->sinkhorn_iters < 1) return FR_E_PARAM;
    if (!p->r || !p->e) return FR_E_NULL;
    return FR_OK;
}

int resolve_k(int K) { return K <= 0 ? 1 : K; }

// A checkpoint interval beyond T means one segment of T iterations (the same
// checkpoints); the segment buffers are sized by the clamped interval.
int clamp_k(int K, int T) { return K <= 1 ? K : std::max(2, std::min(K, T)); }

struct PlainLayout {
    size_t hdr, imp, partial, y, fh, gh, cbar, fbar, fbar0, gbar, gpart, total;
    int nchunk;
};

PlainLayout plain_layout(const fr_problem* p) {
    PlainLayout L;
    const int64_t U = p->n_users;
    const int I = p->n_items, m = p->m, T = p->sinkhorn_iters;
    L.nchunk = impact_chunks(U, I);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align_up(bytes);
        return at;
    };
    L.hdr = take(sizeof(WsHeader));
    L.imp = take(sizeof(double) * I);
    L.partial = take(sizeof(double) * (size_t)L.nchunk * I);
    L.y = take(sizeof(float) * (size_t)U * I);
    L.fh = take(sizeof(float) * (size_t)T * U * I);
    L.gh = take(sizeof(float) * (size_t)(T + 1) * U * m);
    L.cbar = take(sizeof(float) * (size_t)U * I * m);
    L.fbar = take(sizeof(float) * (size_t)U * I);
    L.fbar0 = take(sizeof(float) * (size_t)U * I);
    L.gbar = take(sizeof(float) * (size_t)U * m);
    L.gpart = take(sizeof(double) * (size_t)gnorm_blocks(U * (int64_t)I * m));
    L.total = off;
    return L;
}

fr_status check_optim(const fr_optim* o, const float* mom, const float* vel, int64_t start_step) {
    if (o->rule != FR_ADAM && o->rule != FR_GD) return FR_E_PARAM;
    if (o->rule == FR_ADAM && (!mom || !vel)) return FR_E_NULL;
    if (o->outer_steps < 0 || start_step < 0 || !isfinite(o->lr) || o->lr < 0.f) return FR_E_PARAM;
    if (o->rule == FR_ADAM &&
        (!(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) ||
         !(o->adam_eps >= 0.f)))
        return FR_E_PARAM;
    if (!(o->grad_tol >= 0.0) || !isfinite(o->grad_tol)) return FR_E_PARAM;
    if (!(o->sinkhorn_tol >= 0.f) || !isfinite(o->sinkhorn_tol) || o->cg_iters < 0)
        return FR_E_PARAM;
    return FR_OK;
}

// Asynchronous calls run on the caller's stream; NULL is the null stream.
hipStream_t pick_stream(fr_ctx*, void* s) { return (hipStream_t)s; }

// fr_solve captures a graph, which the null stream cannot do: a NULL stream
// is replaced by the context's own stream, ordered after the null stream's
// prior work (the call synchronises its own stream before returning).
hipStream_t capture_stream(fr_ctx* ctx, void* s) { return s ? (hipStream_t)s : ctx->own; }

FwdArgs fwd_args(const fr_problem* p, const Shape& sh, const float* C) {
    FwdArgs a{};
    a.C = C;
    a.r = p->r;
    a.e = p->e;
    a.U = p->n_users;
    a.I = p->n_items;
    a.m = p->m;
    a.T = p->sinkhorn_iters;
    a.K = 1;
    a.nck = 0;
    a.hs = registry().mp_for(p->m);
    a.L = sh.L;
    a.c2 = (float)(-1.0 / ((double)p->eps * M_LN2));
    a.eps_ln2 = (float)((double)p->eps * M_LN2);
    a.absorb = sh.absorb;
    return a;
}

BwdArgs bwd_args(const fr_problem* p, const Shape& sh, const float* C) {
    BwdArgs a{};
    a.C = C;
    a.r = p->r;
    a.e = p->e;
    a.U = p->n_users;
    a.I = p->n_items;
    a.m = p->m;
    a.T = p->sinkhorn_iters;
    a.K = 1;   // every iterate kept; callers that checkpoint set K
    a.absorb = sh.absorb;
    a.hs = registry().mp_for(p->m);
    a.L = sh.L;
    a.c2 = (float)(-1.0 / ((double)p->eps * M_LN2));
    a.inv_eps = (float)(1.0 / (double)p->eps);
    a.gF = 1.0;
    return a;
}

// The tile reverse sweep's buffer and the flag word, from the workspace, and
// the row store that the forward a fills and the sweep b reads (unless the
// context keeps no row scalings).
void attach_tile(FwdArgs& a, BwdArgs& b, const Layout& Lw, char* w, const fr_ctx* ctx) {
    b.tile.base = w + Lw.tile;
    b.tile.stride = Lw.tile_stride;
    b.tile.batch = Lw.tile_batch;
    b.flags = &((WsHeader*)(w + Lw.hdr))->flags;
    RowStore rs{};
    if (ctx->row_store && Lw.rows_n > 0) rs = {w + Lw.rows, Lw.rows_stride, Lw.rows_n};
    a.rows = rs;
    b.rows = rs;
}

fr_status launch_fwd(const Shape& sh, const FwdArgs& a, hipStream_t s) {
    sh.fwd(a, sh.grid, sh.block, sh.lds_fwd, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status launch_bwd(const Shape& sh, const BwdArgs& a, hipStream_t s) {
    if (sh.tile_bwd && (!a.tile.base || a.tile.stride == 0 || a.tile.batch < 1))
        return FR_E_WORKSPACE;
    sh.bwd(a, sh.grid, sh.block, sh.lds_bwd, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

__global__ void k_init_header(WsHeader* h, int64_t step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->flags = 0;
        h->stopped = 0;
        h->step = step;
        for (int q = 0; q < 8; ++q) h->work[q] = 0;
        h->F = 0.0;
        h->rep = 0;
        h->gnorm = 0.0;
        h->sk_iters = 0;
    }
}

// Column potentials of the converged-map form before its first forward:
// 0 on the real columns, the padding value on the padded ones.
__global__ void k_warm_init(float* gw, int64_t U, int m, int hs) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= U * hs) return;
    gw[j] = ((int)(j % hs) < m) ? 0.f : -1.0e30f;
}

int cg_cap(int m, int requested) { return requested > 0 ? requested : 2 * m + 8; }
constexpr float kCgTol = 1e-6f;

__global__ void k_set_step(WsHeader* h, int64_t step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) h->step = step;
}

fr_status read_flags(WsHeader* h, hipStream_t s, bool clear) {
    uint32_t fl = 0;
    FR_TRY(hipMemcpyAsync(&fl, &h->flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    FR_TRY(hipStreamSynchronize(s));
    if (clear && fl) {
        uint32_t z = 0;
        FR_TRY(hipMemcpyAsync(&h->flags, &z, sizeof(z), hipMemcpyHostToDevice, s));
        FR_TRY(hipStreamSynchronize(s));
    }
    if (fl & FLAG_NONFINITE) return FR_E_NONFINITE;
    if (fl & FLAG_ZERO_IMPACT) return FR_E_ZERO_IMPACT;
    if (fl & FLAG_EPOCHS) return FR_E_UNSUPPORTED;
    return FR_OK;
}

// ---------------------------------------------------------------- batched
// Launch shape of one instance inside the persistent kernels: blocks of 256
// threads with teams of L <= 256 lanes, or of 512 threads with one team of
// 512 lanes (one row per lane), LDS within 64 KB.
struct BatchShape {
    const FusedEntry* fe;
    int L, R, mp, teams;
    size_t lds_fwd, lds_bwd;
};

fr_status batch_shape(fr_ctx* ctx, int I, int m, int K, BatchShape* bs) {
    const Registry& reg = registry();
    const int mp = reg.mp_for(m);
    if (mp < 0) return FR_E_UNSUPPORTED;
    const int BL = (K <= 1) ? kLoadBlock : K;
    // blocks of 256 threads (teams of up to 256 lanes) or of 512 (one team)
    auto fits = [&](int L, int R, const FusedEntry** fe_out, size_t* lf, size_t* lb) {
        const int block = L <= 256 ? 256 : 512;
        if (!lanes_ok(L) || L > 512 || block % L != 0 || (int64_t)L * R < I) return false;
        const FusedEntry* fe = reg.pick(mp, R, L, block);
        if (!fe || !fe->bfwd) return false;
        const int W = (L + 63) / 64;
        const int teams = block / L;
        const size_t per_b = (size_t)((BL + 1) * mp + 2 * W * mp) * sizeof(float);
        if (teams * per_b > kMaxLds) return false;
        *fe_out = fe;
        *lf = (size_t)teams * 2 * W * mp * sizeof(float);
        *lb = teams * per_b;
        return true;
    };
    auto it = ctx->launch.find({I, m});
    if (it != ctx->launch.end()) {
        const FusedEntry* fe;
        size_t lf, lb;
        if (fits(it->second.first, it->second.second, &fe, &lf, &lb)) {
            *bs = BatchShape{fe, it->second.first, it->second.second, mp, fe->lb / it->second.first, lf, lb};
            return FR_OK;
        }
    }
    double best = 1e300;
    bool found = false;
    const int Ls[] = {8, 16, 32, 64, 128, 256, 512};
    for (int L : Ls) {
        for (auto& e : reg.all) {
            if (e.mp != mp || e.lb != (L <= 256 ? 256 : 512) || e.wide != (L >= 64) || !e.bfwd) continue;
            const int R = e.rows;
            if ((int64_t)L * (R - 1) >= I) continue;
            const FusedEntry* fe;
            size_t lf, lb;
            if (!fits(L, R, &fe, &lf, &lb)) continue;
            // the batch as a whole fills the device: cost in the saturated regime
            const bool sc = ctx->form == FR_FORM_SCALING && K <= 1 && fe->bbwds && !fe->recomp_b &&
                            !fe->recomp_f;
            const double c = model_cost((int64_t)1 << 20, mp, L, *fe, sc);
            if (c < best) {
                best = c;
                *bs = BatchShape{fe, L, R, mp, fe->lb / L, lf, lb};
                found = true;
            }
        }
    }
    return found ? FR_OK : FR_E_UNSUPPORTED;
}

struct BatchInst {
    BatchShape sh;
    size_t imp, partial, y, hist;   // workspace offsets
    int nchunk, nck;
};

struct BatchPlan {
    std::vector<BatchInst> inst;
    std::vector<const FusedEntry*> classes;           // distinct kernels
    std::vector<std::vector<BatchItem>> items;        // per class, longest first
    std::vector<size_t> lds_fwd, lds_bwd;             // per class
    std::vector<int2> tab1, tab2;                     // reduction tables
    size_t hdr, counters, d_fwd, d_fin, d_bwd, d_red, d_items, d_tab1, d_tab2, total;
    size_t n_items_total;
};

fr_status plan_batch(fr_ctx* ctx, int n, const fr_problem* probs, int K, BatchPlan* P) {
    P->inst.resize(n);
    size_t off = 0;
    P->hdr = off;
    off += align_up(sizeof(WsHeader));
    for (int j = 0; j < n; ++j) {
        const fr_problem& p = probs[j];
        BatchInst& b = P->inst[j];
        fr_status st = batch_shape(ctx, p.n_items, p.m, K, &b.sh);
        if (st) return st;
        b.nchunk = impact_chunks(p.n_users, p.n_items);
        b.nck = n_checkpoints(p.sinkhorn_iters, K);
        b.imp = off;
        off += align_up(sizeof(double) * p.n_items);
        b.partial = off;
        off += align_up(sizeof(double) * (size_t)b.nchunk * p.n_items);
        b.y = off;
        off += align_up(sizeof(float) * (size_t)p.n_users * p.n_items);
        b.hist = off;
        off += align_up(sizeof(float) * (size_t)p.n_users * b.nck * b.sh.mp);
    }
    // classes and items
    P->classes.clear();
    P->items.clear();
    std::vector<std::vector<std::pair<double, BatchItem>>> tmp;
    for (int j = 0; j < n; ++j) {
        const FusedEntry* fe = P->inst[j].sh.fe;
        size_t c = 0;
        while (c < P->classes.size() && P->classes[c] != fe) ++c;
        if (c == P->classes.size()) {
            P->classes.push_back(fe);
            tmp.emplace_back();
            P->lds_fwd.push_back(0);
            P->lds_bwd.push_back(0);
        }
        P->lds_fwd[c] = std::max(P->lds_fwd[c], P->inst[j].sh.lds_fwd);
        P->lds_bwd[c] = std::max(P->lds_bwd[c], P->inst[j].sh.lds_bwd);
        const int teams = P->inst[j].sh.teams;
        const double cost = (double)teams * probs[j].n_items * probs[j].m * probs[j].sinkhorn_iters;
        for (int64_t u0 = 0; u0 < probs[j].n_users; u0 += teams) {
            BatchItem it;
            it.inst = j;
            it.pad = 0;
            it.u0 = u0;
            tmp[c].push_back({cost, it});
        }
    }
    P->n_items_total = 0;
    for (auto& v : tmp) {
        std::stable_sort(v.begin(), v.end(), [](const std::pair<double, BatchItem>& a,
                                                const std::pair<double, BatchItem>& b) {
            return a.first > b.first;
        });
        std::vector<BatchItem> its;
        its.reserve(v.size());
        for (auto& x : v) its.push_back(x.second);
        P->n_items_total += its.size();
        P->items.push_back(std::move(its));
    }
    // reduction tables
    P->tab1.clear();
    P->tab2.clear();
    for (int j = 0; j < n; ++j) {
        for (int c = 0; c < P->inst[j].nchunk; ++c) P->tab1.push_back(make_int2(j, c));
        for (int g = 0; g < impact_item_groups(probs[j].n_items); ++g) P->tab2.push_back(make_int2(j, g));
    }
    // table sizes are bounded independently of the launch choices, so that
    // fr_workspace_bytes_batched does not depend on a context's overrides
    int64_t users = 0;
    for (int j = 0; j < n; ++j) users += probs[j].n_users;
    P->counters = off;
    off += align_up(sizeof(unsigned) * n);
    P->d_fwd = off;
    off += align_up(sizeof(FwdArgs) * n);
    P->d_fin = off;
    off += align_up(sizeof(FwdArgs) * n);
    P->d_bwd = off;
    off += align_up(sizeof(BwdArgs) * n);
    P->d_red = off;
    off += align_up(sizeof(RedDesc) * n);
    P->d_items = off;
    off += align_up(sizeof(BatchItem) * (size_t)users);
    P->d_tab1 = off;
    off += align_up(sizeof(int2) * P->tab1.size());
    P->d_tab2 = off;
    off += align_up(sizeof(int2) * P->tab2.size());
    P->total = off;
    return FR_OK;
}

__global__ void k_batch_phase(WsHeader* h, unsigned* counters, int n, int advance) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int q = 0; q < n; ++q) counters[q] = 0u;
        if (advance) h->step = h->step + 1;
    }
}

}  // namespace

// ======================================================================== ABI
extern "C" {

const char* fr_status_string(fr_status s) {
    switch (s) {
        case FR_OK: return "ok";
        case FR_E_NULL: return "a required pointer is NULL";
        case FR_E_SHAPE: return "sizes out of range (need 1<=U, 2<=m<=I, I<=4096, m<=64)";
        case FR_E_PARAM: return "invalid parameter (eps, iteration or step counts, optimiser)";
        case FR_E_WORKSPACE: return "workspace smaller than fr_workspace_bytes";
        case FR_E_DEVICE: return "HIP runtime error";
        case FR_E_NONFINITE: return "non-finite value in impacts or objective";
        case FR_E_ZERO_IMPACT: return "an item impact is <= 0 (log undefined)";
        case FR_E_UNSUPPORTED: return "request not supported by this build";
    }
    return "unknown status";
}

fr_status fr_ctx_create(int device, fr_ctx** out) {
    if (!out) return FR_E_NULL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FR_E_DEVICE;
    FR_TRY(hipSetDevice(device));
    fr_ctx* c = new fr_ctx();
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        lds > 0)
        c->max_lds = (size_t)lds;
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return FR_E_DEVICE;
    }
    c->scratch = scratch_address(device);   // fr_step_noalloc reports FR_E_DEVICE if null
    (void)registry();
    *out = c;
    return FR_OK;
}

void fr_ctx_destroy(fr_ctx* ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    if (ctx->own) hipStreamDestroy(ctx->own);
    for (auto st : ctx->side)
        if (st) hipStreamDestroy(st);
    if (ctx->fork) hipEventDestroy(ctx->fork);
    for (auto ev : ctx->join)
        if (ev) hipEventDestroy(ev);
    delete ctx;
}

fr_status fr_workspace_bytes(const fr_problem* prob, const fr_optim* optim, size_t* out) {
    if (!out) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (optim && (!(optim->grad_tol >= 0.0) || !isfinite(optim->grad_tol) ||
                  !(optim->sinkhorn_tol >= 0.f) || !isfinite(optim->sinkhorn_tol) ||
                  optim->cg_iters < 0))
        return FR_E_PARAM;
    const int K = optim ? resolve_k(optim->checkpoint_every) : 1;
    *out = layout(prob, K, optim && optim->grad_tol > 0.0, optim && optim->sinkhorn_tol > 0.f)
               .total;
    return FR_OK;
}

fr_status fr_workspace_init(fr_ctx* ctx, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !ws) return FR_E_NULL;
    if (ws_bytes < kAlign) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, (WsHeader*)ws, (int64_t)0);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status fr_set_launch(fr_ctx* ctx, int32_t n_items, int32_t m, int32_t lanes, int32_t rows) {
    if (!ctx) return FR_E_NULL;
    if (n_items < 2 || m < 2 || m > n_items || m > kMaxM || n_items > kMaxItems) return FR_E_SHAPE;
    if (lanes == 512 && rows == 0) {   // the tile kernels
        if (!tile_entry(m, n_items)) return FR_E_UNSUPPORTED;
        ctx->launch[{n_items, m}] = {512, 0};
        return FR_OK;
    }
    if (!lanes_ok(lanes) || rows < 1 || (int64_t)lanes * rows < n_items) return FR_E_PARAM;
    const Registry& reg = registry();
    const int mp = reg.mp_for(m);
    if (!reg.pick(mp, rows, lanes, block_for(lanes))) return FR_E_UNSUPPORTED;
    ctx->launch[{n_items, m}] = {lanes, rows};
    return FR_OK;
}

fr_status fr_get_launch(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m, int32_t* lanes,
                        int32_t* rows) {
    if (!ctx || !lanes || !rows) return FR_E_NULL;
    if (n_items < 2 || m < 2 || m > n_items || m > kMaxM || n_items > kMaxItems) return FR_E_SHAPE;
    auto it = ctx->launch.find({n_items, m});
    if (n_users < 1) return FR_E_SHAPE;
    std::pair<int, int> lr =
        (it != ctx->launch.end()) ? it->second : default_launch(n_users, n_items, m);
    if (tile_entry(m, n_items) && ctx->form == FR_FORM_SCALING &&
        (it == ctx->launch.end() || lr.second == 0))
        lr = {512, 0};   // the tile kernels
    if (lr.first == 0) return FR_E_UNSUPPORTED;
    *lanes = lr.first;
    *rows = lr.second;
    return FR_OK;
}

}  // extern "C"

namespace {
// fr_step on a given workspace w of at least layout(prob, 1).hist bytes;
// clear_header: reset the header first (its flags are sticky otherwise).
fr_status step_on(fr_ctx* ctx, const fr_problem* prob, const float* C, void* X, fr_dtype x_dtype,
                  float* pot, double* imp, double* F, char* w, bool clear_header, void* stream) {
    const Layout Lw = layout(prob, 1);
    Shape sh;
    fr_status st;
    if ((st = make_shape(ctx, prob->n_users, prob->n_items, prob->m, 1, &sh))) return st;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    WsHeader* hdr = (WsHeader*)(w + Lw.hdr);
    if (clear_header) hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, hdr, (int64_t)0);
    FwdArgs a = fwd_args(prob, sh, C);
    a.y = (float*)(w + Lw.y);
    a.X = X;
    a.x_bf16 = (x_dtype == FR_BF16);
    a.pot = pot;
    if ((st = launch_fwd(sh, a, s))) return st;
    launch_impact(a.y, prob->n_users, prob->n_items, (double*)(w + Lw.partial), Lw.nchunk,
                  imp ? imp : (double*)(w + Lw.imp), F, nullptr, 0, hdr, 0, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}
}  // namespace

extern "C" {

fr_status fr_step(fr_ctx* ctx, const fr_problem* prob, const float* C, void* X, fr_dtype x_dtype,
                  float* pot, double* imp, double* F, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!C || !ws) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    // fr_step needs everything but the history
    if (ws_bytes < layout(prob, 1).hist) return FR_E_WORKSPACE;
    return step_on(ctx, prob, C, X, x_dtype, pot, imp, F, (char*)ws, false, stream);
}

fr_status fr_step_noalloc(fr_ctx* ctx, const fr_problem* prob, const float* C, void* X,
                          fr_dtype x_dtype, float* pot, double* imp, double* F, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!C || !imp || !F) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    if (layout(prob, 1).hist > kScratchBytes) return FR_E_WORKSPACE;
    if (!ctx->scratch) return FR_E_DEVICE;
    return step_on(ctx, prob, C, X, x_dtype, pot, imp, F, (char*)ctx->scratch, true, stream);
}

fr_status fr_nsw(fr_ctx* ctx, const fr_problem* prob, const void* X, fr_dtype x_dtype, double* imp,
                 double* F, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!X || !ws) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    const Layout Lw = layout(prob, 1);
    if (ws_bytes < Lw.hist) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    char* w = (char*)ws;
    float* y = (float*)(w + Lw.y);
    launch_rows_from_plan(X, x_dtype == FR_BF16, prob->r, prob->e, prob->n_users, prob->n_items,
                          prob->m, y, s);
    launch_impact(y, prob->n_users, prob->n_items, (double*)(w + Lw.partial), Lw.nchunk,
                  imp ? imp : (double*)(w + Lw.imp), F, nullptr, 0, (WsHeader*)(w + Lw.hdr), 0, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

// ---------------------------------------------------------------- metrics
struct MetricsLayout {
    size_t hdr, W, partial, rsum, pmax, diag, epart, total;
    int nchunk, tiles, splits;
};

MetricsLayout metrics_layout(const fr_problem* p) {
    MetricsLayout L;
    const int64_t U = p->n_users;
    const int I = p->n_items;
    L.nchunk = impact_chunks(U, I);
    L.tiles = metrics_tiles(I);
    size_t off = 0;
    L.hdr = off;
    off += align_up(sizeof(WsHeader));
    L.W = off;
    off += align_up(sizeof(double) * (size_t)U * I);
    L.partial = off;
    off += align_up(sizeof(double) * (size_t)L.nchunk * I);
    L.rsum = off;
    off += align_up(sizeof(double) * I);
    L.pmax = off;
    off += align_up(sizeof(double) * (size_t)I * L.tiles);
    L.diag = off;
    off += align_up(sizeof(double) * I);
    L.splits = metrics_splits(U, I);
    L.epart = off;
    if (L.splits > 1) off += align_up(sizeof(double) * (size_t)L.splits * I * I);
    L.total = off;
    return L;
}

fr_status fr_workspace_bytes_metrics(const fr_problem* prob, size_t* out) {
    if (!out) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    *out = metrics_layout(prob).total;
    return FR_OK;
}

fr_status fr_metrics(fr_ctx* ctx, const fr_problem* prob, const void* X, fr_dtype x_dtype,
                     double* out, double* envy, double* imp, void* ws, size_t ws_bytes,
                     void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!X || !out || !ws) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    const MetricsLayout Lw = metrics_layout(prob);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    char* w = (char*)ws;
    MetricsBufs b;
    b.hdr = (WsHeader*)(w + Lw.hdr);
    b.W = (double*)(w + Lw.W);
    b.partial = (double*)(w + Lw.partial);
    b.nchunk = Lw.nchunk;
    b.rsum = (double*)(w + Lw.rsum);
    b.pmax = (double*)(w + Lw.pmax);
    b.diag = (double*)(w + Lw.diag);
    b.epart = (double*)(w + Lw.epart);
    b.splits = Lw.splits;
    launch_metrics(X, x_dtype == FR_BF16, prob->r, prob->e, prob->n_users, prob->n_items, prob->m,
                   b, out, envy, imp, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status fr_backward(fr_ctx* ctx, const fr_problem* prob, const float* C, const double* imp,
                      double gF, float* dC, float* dr, int32_t checkpoint_every, void* ws,
                      size_t ws_bytes, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!C || !imp || !dC || !ws) return FR_E_NULL;
    if (checkpoint_every < 1 || !isfinite(gF)) return FR_E_PARAM;
    const int K = clamp_k(checkpoint_every, prob->sinkhorn_iters);
    const Layout Lw = layout(prob, K);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    Shape sh;
    if ((st = make_shape(ctx, prob->n_users, prob->n_items, prob->m, K, &sh))) return st;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    char* w = (char*)ws;
    FwdArgs a = fwd_args(prob, sh, C);
    a.hist = (float*)(w + Lw.hist);
    a.K = K;
    a.nck = Lw.nck;
    BwdArgs b = bwd_args(prob, sh, C);
    b.hist = a.hist;
    b.K = K;
    b.nck = Lw.nck;
    b.imp = imp;
    b.gF = gF;
    b.dC = dC;
    b.dr = dr;
    attach_tile(a, b, Lw, w, ctx);
    if ((st = launch_fwd(sh, a, s))) return st;
    return launch_bwd(sh, b, s);
}

fr_status fr_solve(fr_ctx* ctx, const fr_problem* prob, const fr_optim* optim, float* C,
                   float* adam_m, float* adam_v, int64_t start_step, void* X_out, fr_dtype x_dtype,
                   double* F_hist, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !optim) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if ((st = check_optim(optim, adam_m, adam_v, start_step))) return st;
    if (!C || !F_hist || !ws) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    const int K = clamp_k(resolve_k(optim->checkpoint_every), prob->sinkhorn_iters);
    const bool tol = optim->grad_tol > 0.0;
    const bool conv = optim->sinkhorn_tol > 0.f;
    const Layout Lw = layout(prob, K, tol, conv);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    Shape sh;
    if ((st = make_shape(ctx, prob->n_users, prob->n_items, prob->m, K, &sh))) return st;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = capture_stream(ctx, stream);
    if (!stream) FR_TRY(hipStreamSynchronize(nullptr));
    char* w = (char*)ws;
    WsHeader* hdr = (WsHeader*)(w + Lw.hdr);
    const int64_t ncell = prob->n_users * (int64_t)prob->n_items * prob->m;
    double* imp = (double*)(w + Lw.imp);
    double* partial = (double*)(w + Lw.partial);
    float* y = (float*)(w + Lw.y);
    float* hist = (float*)(w + Lw.hist);

    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, hdr, start_step);
    FR_TRY(hipGetLastError());

    FwdArgs a = fwd_args(prob, sh, C);
    a.y = y;
    a.hist = hist;
    a.K = K;
    a.nck = Lw.nck;
    BwdArgs b = bwd_args(prob, sh, C);
    b.hist = hist;
    b.K = K;
    b.nck = Lw.nck;
    b.imp = imp;
    attach_tile(a, b, Lw, w, ctx);
    b.Cw = C;
    b.mom = adam_m;
    b.vel = adam_v;
    b.step_ptr = &hdr->step;
    b.rule = optim->rule;
    b.lr = optim->lr;
    b.b1 = optim->beta1;
    b.b2 = optim->beta2;
    b.aeps = optim->adam_eps;
    if (tol) {
        // Algorithm 1's loop test: the backward writes the gradient, its norm
        // decides, and every launch of the replayed step is skipped after a stop
        a.stop = &hdr->stopped;
        b.stop = &hdr->stopped;
        b.Cw = nullptr;
        b.dC = (float*)(w + Lw.grad);
    }
    if (conv) {
        // converged-map form: warm-started forward to tolerance, implicit gradient
        float* gw = (float*)(w + Lw.gw);
        const int64_t ng = prob->n_users * (int64_t)Lw.hs;
        hipLaunchKernelGGL(k_warm_init, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, gw,
                           prob->n_users, prob->m, Lw.hs);
        a.hist = nullptr;
        a.gw = gw;
        a.phi = (float*)(w + Lw.phi);
        a.tol = optim->sinkhorn_tol;
        a.iters = &hdr->sk_iters;
        b.gw = gw;
        b.phi = a.phi;
        b.cg_max = cg_cap(prob->m, optim->cg_iters);
        b.cg_tol = kCgTol;
    }
    auto outer_step = [&]() {
        (conv ? sh.fe->fwdc : sh.fwd)(a, sh.grid, sh.block, sh.lds_fwd, s);
        launch_impact(y, prob->n_users, prob->n_items, partial, Lw.nchunk, imp, nullptr, F_hist,
                      start_step, hdr, tol ? ADV_REP : ADV_REP_STEP, s);
        if (conv)
            sh.fe->ibwd(b, sh.grid, sh.block, sh.lds_fwd, s);
        else
            sh.bwd(b, sh.grid, sh.block, sh.lds_bwd, s);
        if (tol)
            launch_gnorm_update(b.dC, C, adam_m, adam_v, ncell, optim->rule, optim->lr,
                                optim->beta1, optim->beta2, optim->adam_eps,
                                (double*)(w + Lw.gpart), optim->grad_tol, hdr, s);
    };

    const int N = optim->outer_steps;
    if (N > 0 && ctx->timing && !tol && !conv) {
        // direct launches, each fused kernel bracketed by events
        EventSet evs(4 * (size_t)N);
        FR_TRY(evs.create());
        const std::vector<hipEvent_t>& ev = evs.ev;
        for (int n = 0; n < N; ++n) {
            FR_TRY(hipEventRecord(ev[4 * n + 0], s));
            sh.fwd(a, sh.grid, sh.block, sh.lds_fwd, s);
            FR_TRY(hipEventRecord(ev[4 * n + 1], s));
            launch_impact(y, prob->n_users, prob->n_items, partial, Lw.nchunk, imp, nullptr, F_hist,
                          start_step, hdr, ADV_REP_STEP, s);
            FR_TRY(hipEventRecord(ev[4 * n + 2], s));
            sh.bwd(b, sh.grid, sh.block, sh.lds_bwd, s);
            FR_TRY(hipEventRecord(ev[4 * n + 3], s));
        }
        FR_TRY(hipGetLastError());
        FR_TRY(hipStreamSynchronize(s));
        for (int n = 0; n < N; ++n) {
            float t1 = 0.f, t2 = 0.f;
            FR_TRY(hipEventElapsedTime(&t1, ev[4 * n + 0], ev[4 * n + 1]));
            FR_TRY(hipEventElapsedTime(&t2, ev[4 * n + 2], ev[4 * n + 3]));
            ctx->fwd_ms += t1;
            ctx->bwd_ms += t2;
        }
        ctx->fwd_n += N;
        ctx->bwd_n += N;
    } else if (N > 0) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        FR_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        outer_step();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (ce != hipSuccess) return FR_E_DEVICE;
        ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ce != hipSuccess) {
            hipGraphDestroy(graph);
            return FR_E_DEVICE;
        }
        for (int n = 0; n < N && ce == hipSuccess; ++n) ce = hipGraphLaunch(exec, s);
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        if (ce != hipSuccess) return FR_E_DEVICE;
    }
    // final forward: X(C_N) and F_N (also after a stop)
    a.hist = nullptr;
    a.stop = nullptr;
    a.rows = RowStore{};
    a.X = X_out;
    a.x_bf16 = (x_dtype == FR_BF16);
    if (conv) {
        sh.fe->fwdc(a, sh.grid, sh.block, sh.lds_fwd, s);
        FR_TRY(hipGetLastError());
    } else if ((st = launch_fwd(sh, a, s))) {
        return st;
    }
    launch_impact(y, prob->n_users, prob->n_items, partial, Lw.nchunk, imp, nullptr, F_hist,
                  start_step, hdr, ADV_NONE, s);
    FR_TRY(hipGetLastError());
    return read_flags(hdr, s, false);
}

fr_status fr_solve_progress(fr_ctx* ctx, void* ws, void* stream, int64_t* steps,
                            double* last_gnorm, int64_t* sinkhorn_iters) {
    if (!ctx || !ws) return FR_E_NULL;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    FR_TRY(hipStreamSynchronize(s));
    WsHeader h;
    FR_TRY(hipMemcpy(&h, ws, sizeof(WsHeader), hipMemcpyDeviceToHost));
    if (steps) *steps = h.step;
    if (last_gnorm) *last_gnorm = h.gnorm;
    if (sinkhorn_iters) *sinkhorn_iters = h.sk_iters;
    return FR_OK;
}

fr_status fr_grad_converged(fr_ctx* ctx, const fr_problem* prob, const float* C,
                            float sinkhorn_tol, int32_t cg_iters, double gF, double* imp_out,
                            double* F, float* dC, float* dr, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!C || !dC || !ws) return FR_E_NULL;
    if (!(sinkhorn_tol > 0.f) || !isfinite(sinkhorn_tol) || cg_iters < 0 || !isfinite(gF))
        return FR_E_PARAM;
    const Layout Lw = layout(prob, 1, false, true);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    Shape sh;
    if ((st = make_shape(ctx, prob->n_users, prob->n_items, prob->m, 1, &sh))) return st;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    char* w = (char*)ws;
    WsHeader* hdr = (WsHeader*)(w + Lw.hdr);
    double* imp = imp_out ? imp_out : (double*)(w + Lw.imp);
    float* gw = (float*)(w + Lw.gw);
    const int64_t ng = prob->n_users * (int64_t)Lw.hs;
    hipLaunchKernelGGL(k_warm_init, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, gw,
                       prob->n_users, prob->m, Lw.hs);
    FwdArgs a = fwd_args(prob, sh, C);
    a.y = (float*)(w + Lw.y);
    a.gw = gw;
    a.phi = (float*)(w + Lw.phi);
    a.tol = sinkhorn_tol;
    a.iters = &hdr->sk_iters;
    sh.fe->fwdc(a, sh.grid, sh.block, sh.lds_fwd, s);
    launch_impact(a.y, prob->n_users, prob->n_items, (double*)(w + Lw.partial), Lw.nchunk, imp, F,
                  nullptr, 0, hdr, ADV_NONE, s);
    BwdArgs b = bwd_args(prob, sh, C);
    b.imp = imp;
    b.gF = gF;
    b.dC = dC;
    b.dr = dr;
    b.gw = gw;
    b.phi = a.phi;
    b.cg_max = cg_cap(prob->m, cg_iters);
    b.cg_tol = kCgTol;
    sh.fe->ibwd(b, sh.grid, sh.block, sh.lds_fwd, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status fr_rank_maxrele(fr_ctx* ctx, const fr_problem* prob, int32_t* sel, void* X,
                          int32_t x_dtype, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!sel) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    launch_maxrele(prob->r, prob->n_users, prob->n_items, prob->m, sel, s);
    if (X) launch_plan_from_sel(sel, prob->n_users, prob->n_items, prob->m, X, x_dtype == FR_BF16, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status fr_rank_greedy(fr_ctx* ctx, const fr_problem* prob, int32_t* sel, void* X,
                         int32_t x_dtype, double* imp, void* stream) {
    if (!ctx) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (!sel) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    launch_greedy(prob->r, prob->e, prob->n_users, prob->n_items, prob->m, sel, imp, s);
    if (X) launch_plan_from_sel(sel, prob->n_users, prob->n_items, prob->m, X, x_dtype == FR_BF16, s);
    FR_TRY(hipGetLastError());
    return FR_OK;
}

fr_status fr_ctx_set_form(fr_ctx* ctx, int32_t form, int32_t absorb_every) {
    if (!ctx) return FR_E_NULL;
    if ((form != FR_FORM_LOG && form != FR_FORM_SCALING) || absorb_every < 0) return FR_E_PARAM;
    ctx->form = form;
    ctx->absorb = absorb_every;
    return FR_OK;
}

fr_status fr_ctx_set_row_store(fr_ctx* ctx, int enable) {
    if (!ctx) return FR_E_NULL;
    ctx->row_store = enable != 0;
    return FR_OK;
}

fr_status fr_ctx_kernel_forms(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m,
                              int32_t checkpoint_every, int32_t* fwd_form, int32_t* bwd_form) {
    if (!ctx) return FR_E_NULL;
    if (n_users < 1 || n_items < 2 || m < 2 || m > n_items || m > kMaxM || n_items > kMaxItems)
        return FR_E_SHAPE;
    Shape sh;
    fr_status st = make_shape(ctx, n_users, n_items, m, resolve_k(checkpoint_every), &sh);
    if (st) return st;
    if (fwd_form)
        *fwd_form = sh.te ? 2 : (sh.fwd == sh.fe->fwds) ? FR_FORM_SCALING : FR_FORM_LOG;
    if (bwd_form)
        *bwd_form = sh.tile_bwd ? 2 : (sh.bwd == sh.fe->bwds) ? FR_FORM_SCALING : FR_FORM_LOG;
    return FR_OK;
}

fr_status fr_ctx_bwd_lds_rows(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m,
                              int32_t checkpoint_every, int32_t* rows) {
    if (!ctx || !rows) return FR_E_NULL;
    if (n_users < 1 || n_items < 2 || m < 2 || m > n_items || m > kMaxM || n_items > kMaxItems)
        return FR_E_SHAPE;
    Shape sh;
    fr_status st = make_shape(ctx, n_users, n_items, m, resolve_k(checkpoint_every), &sh);
    if (st) return st;
    *rows = (sh.bwd == sh.fe->bwdl) ? sh.fe->cb_rows : 0;
    return FR_OK;
}

fr_status fr_ctx_set_timing(fr_ctx* ctx, int enable) {
    if (!ctx) return FR_E_NULL;
    ctx->timing = enable != 0;
    ctx->fwd_ms = ctx->bwd_ms = 0.0;
    ctx->fwd_n = ctx->bwd_n = 0;
    return FR_OK;
}

fr_status fr_ctx_kernel_times(fr_ctx* ctx, double* fwd_ms, int64_t* fwd_launches, double* bwd_ms,
                              int64_t* bwd_launches) {
    if (!ctx) return FR_E_NULL;
    if (fwd_ms) *fwd_ms = ctx->fwd_ms;
    if (fwd_launches) *fwd_launches = ctx->fwd_n;
    if (bwd_ms) *bwd_ms = ctx->bwd_ms;
    if (bwd_launches) *bwd_launches = ctx->bwd_n;
    return FR_OK;
}

fr_status fr_sync_status(fr_ctx* ctx, void* ws, void* stream) {
    if (!ctx || !ws) return FR_E_NULL;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    FR_TRY(hipStreamSynchronize(s));
    return read_flags((WsHeader*)ws, s, true);
}

fr_status fr_workspace_bytes_plain(const fr_problem* prob, size_t* out) {
    if (!out) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    *out = plain_layout(prob).total;
    return FR_OK;
}

fr_status fr_solve_plain(fr_ctx* ctx, const fr_problem* prob, const fr_optim* optim, float* C,
                         float* adam_m, float* adam_v, int64_t start_step, void* X_out,
                         fr_dtype x_dtype, double* F_hist, void* ws, size_t ws_bytes,
                         void* stream) {
    if (!ctx || !optim) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if ((st = check_optim(optim, adam_m, adam_v, start_step))) return st;
    if (!C || !F_hist || !ws) return FR_E_NULL;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    if (optim->sinkhorn_tol > 0.f) return FR_E_UNSUPPORTED;   // fused form only
    const PlainLayout Lw = plain_layout(prob);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = capture_stream(ctx, stream);
    if (!stream) FR_TRY(hipStreamSynchronize(nullptr));
    char* w = (char*)ws;
    PlainBufs b;
    b.hdr = (WsHeader*)(w + Lw.hdr);
    b.imp = (double*)(w + Lw.imp);
    b.partial = (double*)(w + Lw.partial);
    b.y = (float*)(w + Lw.y);
    b.fh = (float*)(w + Lw.fh);
    b.gh = (float*)(w + Lw.gh);
    b.cbar = (float*)(w + Lw.cbar);
    b.fbar = (float*)(w + Lw.fbar);
    b.fbar0 = (float*)(w + Lw.fbar0);
    b.gbar = (float*)(w + Lw.gbar);
    b.nchunk = Lw.nchunk;
    const int64_t U = prob->n_users;
    const int I = prob->n_items, m = prob->m, T = prob->sinkhorn_iters;
    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, b.hdr, start_step);
    const bool tol = optim->grad_tol > 0.0;
    for (int n = 0; n < optim->outer_steps; ++n) {
        // after a gradient-norm stop C no longer changes, so F repeats
        plain_forward(C, prob->r, prob->e, U, I, m, prob->eps, T, b, nullptr, 0, s);
        launch_impact(b.y, U, I, b.partial, b.nchunk, b.imp, nullptr, F_hist, start_step, b.hdr,
                      tol ? ADV_REP : ADV_REP_STEP, s);
        plain_backward_update(C, prob->r, prob->e, U, I, m, prob->eps, T, b, adam_m, adam_v,
                              optim->rule, optim->lr, optim->beta1, optim->beta2, optim->adam_eps,
                              !tol, s);
        if (tol)
            launch_gnorm_update(b.cbar, C, adam_m, adam_v, U * (int64_t)I * m, optim->rule,
                                optim->lr, optim->beta1, optim->beta2, optim->adam_eps,
                                (double*)(w + Lw.gpart), optim->grad_tol, b.hdr, s);
        FR_TRY(hipGetLastError());
    }
    plain_forward(C, prob->r, prob->e, U, I, m, prob->eps, T, b, X_out, x_dtype == FR_BF16, s);
    launch_impact(b.y, U, I, b.partial, b.nchunk, b.imp, nullptr, F_hist, start_step, b.hdr,
                  ADV_NONE, s);
    FR_TRY(hipGetLastError());
    return read_flags(b.hdr, s, false);
}

fr_status fr_workspace_bytes_batched(int32_t n_inst, const fr_problem* probs,
                                     const fr_optim* optim, size_t* out) {
    if (!out || !probs) return FR_E_NULL;
    if (n_inst < 1) return FR_E_SHAPE;
    for (int j = 0; j < n_inst; ++j) {
        fr_status st = check_problem(&probs[j]);
        if (st) return st;
    }
    fr_ctx tmp;   // default launch choices
    BatchPlan P;
    fr_status st = plan_batch(&tmp, n_inst, probs, optim ? resolve_k(optim->checkpoint_every) : 1, &P);
    if (st) return st;
    *out = P.total;
    return FR_OK;
}

fr_status fr_solve_batched(fr_ctx* ctx, int32_t n_inst, const fr_problem* probs,
                           const fr_optim* optim, float* const* C, float* const* adam_m,
                           float* const* adam_v, int64_t start_step, void* const* X,
                           fr_dtype x_dtype, double* const* F_hist, void* ws, size_t ws_bytes,
                           void* stream) {
    if (!ctx || !optim || !probs || !C || !F_hist || !ws) return FR_E_NULL;
    // the gradient-norm test of Algorithm 1 is per instance: not offered for
    // the batched solve
    if (optim->grad_tol != 0.0 || optim->sinkhorn_tol != 0.f) return FR_E_UNSUPPORTED;
    if (n_inst < 1) return FR_E_SHAPE;
    if (x_dtype != FR_F32 && x_dtype != FR_BF16) return FR_E_PARAM;
    for (int j = 0; j < n_inst; ++j) {
        fr_status st = check_problem(&probs[j]);
        if (st) return st;
        if (!C[j] || !F_hist[j]) return FR_E_NULL;
        st = check_optim(optim, adam_m ? adam_m[j] : nullptr, adam_v ? adam_v[j] : nullptr,
                         start_step);
        if (st) return st;
    }
    const int K = resolve_k(optim->checkpoint_every);
    BatchPlan P;
    fr_status st = plan_batch(ctx, n_inst, probs, K, &P);
    if (st) return st;
    if (ws_bytes < P.total) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = capture_stream(ctx, stream);
    if (!stream) FR_TRY(hipStreamSynchronize(nullptr));
    char* w = (char*)ws;
    WsHeader* hdr = (WsHeader*)(w + P.hdr);
    unsigned* counters = (unsigned*)(w + P.counters);

    // descriptors
    std::vector<FwdArgs> fa(n_inst), ff(n_inst);
    std::vector<BwdArgs> ba(n_inst);
    std::vector<RedDesc> rd(n_inst);
    for (int j = 0; j < n_inst; ++j) {
        const fr_problem* p = &probs[j];
        const BatchInst& b = P.inst[j];
        Shape sh{};
        sh.L = b.sh.L;
        FwdArgs a = fwd_args(p, sh, C[j]);
        a.y = (float*)(w + b.y);
        a.hist = (float*)(w + b.hist);
        a.K = K;
        a.nck = b.nck;
        fa[j] = a;
        a.hist = nullptr;
        a.X = X ? X[j] : nullptr;
        a.x_bf16 = (x_dtype == FR_BF16);
        ff[j] = a;
        BwdArgs g = bwd_args(p, sh, C[j]);
        g.hist = (float*)(w + b.hist);
        g.K = K;
        g.nck = b.nck;
        g.imp = (double*)(w + b.imp);
        g.Cw = C[j];
        g.mom = adam_m ? adam_m[j] : nullptr;
        g.vel = adam_v ? adam_v[j] : nullptr;
        g.step_ptr = &hdr->step;
        g.rule = optim->rule;
        g.lr = optim->lr;
        g.b1 = optim->beta1;
        g.b2 = optim->beta2;
        g.aeps = optim->adam_eps;
        ba[j] = g;
        RedDesc r;
        r.y = (const float*)(w + b.y);
        r.partial = (double*)(w + b.partial);
        r.imp = (double*)(w + b.imp);
        r.F_hist = F_hist[j];
        r.U = p->n_users;
        r.I = p->n_items;
        r.nchunk = b.nchunk;
        rd[j] = r;
    }
    std::vector<BatchItem> all_items;
    std::vector<size_t> item_off;
    for (auto& v : P.items) {
        item_off.push_back(all_items.size());
        all_items.insert(all_items.end(), v.begin(), v.end());
    }
    FR_TRY(hipMemcpyAsync(w + P.d_fwd, fa.data(), sizeof(FwdArgs) * n_inst, hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_fin, ff.data(), sizeof(FwdArgs) * n_inst, hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_bwd, ba.data(), sizeof(BwdArgs) * n_inst, hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_red, rd.data(), sizeof(RedDesc) * n_inst, hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_items, all_items.data(), sizeof(BatchItem) * all_items.size(),
                          hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_tab1, P.tab1.data(), sizeof(int2) * P.tab1.size(),
                          hipMemcpyHostToDevice, s));
    FR_TRY(hipMemcpyAsync(w + P.d_tab2, P.tab2.data(), sizeof(int2) * P.tab2.size(),
                          hipMemcpyHostToDevice, s));
    FR_TRY(hipStreamSynchronize(s));   // host vectors are released below

    int cus = 0;
    FR_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int ncls = (int)P.classes.size();
    const FwdArgs* dfa = (const FwdArgs*)(w + P.d_fwd);
    const FwdArgs* dff = (const FwdArgs*)(w + P.d_fin);
    const BwdArgs* dba = (const BwdArgs*)(w + P.d_bwd);
    const RedDesc* drd = (const RedDesc*)(w + P.d_red);
    const BatchItem* ditems = (const BatchItem*)(w + P.d_items);
    const int2* dt1 = (const int2*)(w + P.d_tab1);
    const int2* dt2 = (const int2*)(w + P.d_tab2);
    std::vector<int> grid_f(ncls), grid_b(ncls);
    const bool scaling = ctx->form == FR_FORM_SCALING;   // the batched forward follows the context
    // and so does the reverse sweep, under the single-instance rule (K = 1, no recompute)
    std::vector<char> sweep_s(ncls);
    for (int c = 0; c < ncls; ++c)
        sweep_s[c] = scaling && K <= 1 && P.classes[c]->bbwds && !P.classes[c]->recomp_b;
    for (int c = 0; c < ncls; ++c) {
        const int nit = (int)P.items[c].size();
        const Occupancy occ_f = scaling ? P.classes[c]->occ_bfwds : P.classes[c]->occ_bfwd;
        const int blk = P.classes[c]->lb;
        grid_f[c] = std::max(1, std::min(nit, occ_f(blk, P.lds_fwd[c]) * cus));
        const Occupancy occ_b = sweep_s[c] ? P.classes[c]->occ_bbwds : P.classes[c]->occ_bbwd;
        grid_b[c] = std::max(1, std::min(nit, occ_b(blk, P.lds_bwd[c]) * cus));
    }
    // The column classes of a phase share nothing (own work lists, counters and
    // outputs), so they run concurrently: forked from s onto the side streams
    // and joined back (inside a capture this becomes parallel graph branches).
    const bool fan = ncls > 1 && ncls <= fr_ctx::kMaxClasses;   // else one after another
    if (fan && !ctx->fork) {
        for (auto& st : ctx->side) FR_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        FR_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
        for (auto& ev : ctx->join) FR_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    hipError_t perr = hipSuccess;   // first fork / join error of the phases below
    auto keep = [&](hipError_t e) {
        if (perr == hipSuccess) perr = e;
    };
    auto run_classes = [&](auto&& launch_class) {
        if (!fan) {
            for (int c = 0; c < ncls; ++c) launch_class(c, s);
            return;
        }
        keep(hipEventRecord(ctx->fork, s));
        for (int c = 0; c < ncls; ++c) {
            hipStream_t sc = ctx->side[c % fr_ctx::kSide];
            keep(hipStreamWaitEvent(sc, ctx->fork, 0));
            launch_class(c, sc);
            keep(hipEventRecord(ctx->join[c], sc));
        }
        for (int c = 0; c < ncls; ++c) keep(hipStreamWaitEvent(s, ctx->join[c], 0));
    };
    auto forward_phase = [&](const FwdArgs* descs) {
        hipLaunchKernelGGL(k_batch_phase, dim3(1), dim3(64), 0, s, hdr, counters, ncls, 0);
        run_classes([&](int c, hipStream_t sc) {
            (scaling ? P.classes[c]->bfwds : P.classes[c]->bfwd)(
                descs, ditems + item_off[c], (int)P.items[c].size(), counters + c, grid_f[c],
                P.classes[c]->lb, P.lds_fwd[c], sc);
        });
        launch_impact_batched(drd, n_inst, dt1, (int)P.tab1.size(), dt2, (int)P.tab2.size(),
                              start_step, hdr, s);
    };
    auto backward_phase = [&]() {
        hipLaunchKernelGGL(k_batch_phase, dim3(1), dim3(64), 0, s, hdr, counters, ncls, 1);
        run_classes([&](int c, hipStream_t sc) {
            (sweep_s[c] ? P.classes[c]->bbwds : P.classes[c]->bbwd)(
                dba, ditems + item_off[c], (int)P.items[c].size(), counters + c, grid_b[c],
                P.classes[c]->lb, P.lds_bwd[c], sc);
        });
    };

    hipLaunchKernelGGL(k_init_header, dim3(1), dim3(64), 0, s, hdr, start_step);
    FR_TRY(hipGetLastError());
    const int N = optim->outer_steps;
    if (N > 0) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        FR_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        forward_phase(dfa);
        backward_phase();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (ce != hipSuccess || perr != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return FR_E_DEVICE;
        }
        ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ce != hipSuccess) {
            hipGraphDestroy(graph);
            return FR_E_DEVICE;
        }
        for (int q = 0; q < N && ce == hipSuccess; ++q) ce = hipGraphLaunch(exec, s);
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        if (ce != hipSuccess) return FR_E_DEVICE;
    }
    forward_phase(dff);
    FR_TRY(perr);
    FR_TRY(hipGetLastError());
    return read_flags(hdr, s, false);
}

fr_status fr_autotune(fr_ctx* ctx, const fr_problem* prob, const float* C, int32_t batched,
                      int32_t iters, void* ws, size_t ws_bytes, void* stream, int32_t* lanes_out,
                      int32_t* rows_out) {
    if (!ctx || !C || !ws) return FR_E_NULL;
    fr_status st = check_problem(prob);
    if (st) return st;
    if (iters < 1) return FR_E_PARAM;
    fr_problem p = *prob;
    p.sinkhorn_iters = std::min(prob->sinkhorn_iters, iters);
    const Layout Lw = layout(&p, 1);
    if (ws_bytes < Lw.total) return FR_E_WORKSPACE;
    FR_TRY(hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    char* w = (char*)ws;
    const Registry& reg = registry();
    const int mp = reg.mp_for(p.m);
    if (mp < 0) return FR_E_UNSUPPORTED;
    const int I = p.n_items;
    const auto saved = ctx->launch;
    // the candidates are tried through the context's launch cache; it is put
    // back on every exit but a successful one, error returns included
    bool done = false;
    auto restore = on_exit([&] {
        if (!done) ctx->launch = saved;
    });
    EventSet evs(2);
    FR_TRY(evs.create());
    hipEvent_t e0 = evs.ev[0], e1 = evs.ev[1];
    float best = 1e30f;
    std::pair<int, int> best_lr{0, 0};
    // candidates: the tile kernels where they take the plan, then every
    // instantiated (lanes, rows per lane) shape
    std::vector<std::pair<int, int>> cands;
    if (!batched && tile_entry(p.m, I) && ctx->form == FR_FORM_SCALING) cands.push_back({512, 0});
    const int Ls[] = {8, 16, 32, 64, 128, 192, 256, 320, 384, 448, 512, 640, 768, 896, 1024};
    for (int L : Ls) {
        // the batched kernels' blocks: 256 threads, or 512 for one team of 512 lanes
        const int bblk = L <= 256 ? 256 : 512;
        if (batched && (L > 512 || bblk % L != 0)) continue;
        for (auto& e : reg.all) {
            if (e.mp != mp) continue;
            const int R = e.rows;
            if ((int64_t)L * R < I || (int64_t)L * (R - 1) >= I) continue;
            if (&e != reg.pick(mp, R, L, batched ? bblk : block_for(L))) continue;
            if (batched && (R * mp > 128 || !e.bfwd)) continue;
            cands.push_back({L, R});
        }
    }
    for (const auto& lr : cands) {
        {
            const int L = lr.first, R = lr.second;
            ctx->launch[{I, p.m}] = {L, R};
            Shape sh;
            if (make_shape(ctx, p.n_users, I, p.m, 1, &sh) != FR_OK) continue;
            if (R > 0 && (sh.te || sh.fe != reg.pick(mp, R, L, batched ? (L <= 256 ? 256 : 512)
                                                                       : block_for(L))))
                continue;
            FwdArgs a = fwd_args(&p, sh, C);
            a.y = (float*)(w + Lw.y);
            a.hist = (float*)(w + Lw.hist);
            a.nck = Lw.nck;
            BwdArgs b = bwd_args(&p, sh, C);
            b.hist = a.hist;
            b.nck = Lw.nck;
            double* impw = (double*)(w + Lw.imp);
            b.imp = impw;
            attach_tile(a, b, Lw, w, ctx);
            if (sh.tile_bwd && Lw.tile_stride == 0) continue;
            // one warm-up repetition, then the fastest of three
            float tot = 1e30f;
            for (int rep = 0; rep < 4; ++rep) {
                FR_TRY(hipEventRecord(e0, s));
                sh.fwd(a, sh.grid, sh.block, sh.lds_fwd, s);
                launch_impact(a.y, p.n_users, I, (double*)(w + Lw.partial), Lw.nchunk, impw,
                              nullptr, nullptr, 0, (WsHeader*)(w + Lw.hdr), 0, s);
                sh.bwd(b, sh.grid, sh.block, sh.lds_bwd, s);
                FR_TRY(hipEventRecord(e1, s));
                FR_TRY(hipEventSynchronize(e1));
                FR_TRY(hipGetLastError());
                float ms = 0.f;
                FR_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) tot = std::min(tot, ms);
            }
            if (tot < best) {
                best = tot;
                best_lr = {L, R};
            }
        }
    }
    if (best_lr.first == 0) return FR_E_UNSUPPORTED;
    ctx->launch = saved;
    ctx->launch[{I, p.m}] = best_lr;
    done = true;
    if (lanes_out) *lanes_out = best_lr.first;
    if (rows_out) *rows_out = best_lr.second;
    return FR_OK;
}

}  // extern "C"
