// fr_internal.h -- structures shared by the HIP kernels and the host side of
// the fair-ranking library.  Not part of the public ABI (see fairrank.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr {

// Device-side flag bits written into the workspace header.
enum : uint32_t { FLAG_NONFINITE = 1u, FLAG_ZERO_IMPACT = 2u, FLAG_EPOCHS = 4u };

// Workspace header (first 256 bytes of every workspace).
struct WsHeader {
    uint32_t flags;       // FLAG_* bits, sticky until fr_sync_status clears them
    int32_t stopped;      // the gradient-norm test of Algorithm 1 ended the loop
    int64_t step;         // Adam step count (advanced once per update applied)
    uint32_t work[8];     // work-queue counters of the batched kernels
    double F;             // last objective value
    int64_t rep;          // outer steps recorded in the F history since the start
    double gnorm;         // ||dF/dC||_F of the last gradient tested
    int64_t sk_iters;     // Sinkhorn iterations used, summed over consumers and forwards
};

// ---------------------------------------------------------------------------
// Fused forward: one team of L lanes per consumer, R plan rows per lane held
// in registers, MP (>= m) columns per row.
// Row scalings of the tile forward (fr_tile.hip), kept for its reverse sweep:
// per consumer u < n, the row scaling of every iteration and the reference
// kernel of every stretch between rebases.
struct RowStore {
    char* base;        // n consumers x stride bytes (or null: not kept)
    size_t stride;     // bytes per consumer
    int64_t n;         // consumers 0 .. n-1 are kept
};

struct FwdArgs {
    const float* C;        // [U][I][m]
    const float* r;        // [U][I]
    const float* e;        // [m-1]
    float* y;              // [U][I]  r_ui * sum_{k<m-1} e_k x_uik  (or null)
    float* hist;           // [U][nck][hs] base-2 column potentials (or null)
    void* X;               // [U][I][m] plan (or null)
    float* pot;            // [U][I+m] potentials in cost units (or null)
    const int32_t* stop;   // skip the launch when *stop != 0 (or null)
    float* gw;             // [U][hs] base-2 column potentials: start (warm) and result, or null
    float* phi;            // [U][I] base-2 row potentials of the uncentred costs (or null)
    int64_t* iters;        // sum of the iterations used, added per consumer (or null)
    float tol;             // > 0: stop a consumer once no potential moves by more than tol
    int absorb;            // scaling form: also absorb every `absorb` iterations (0: on range only)
    RowStore rows;         // tile forward: row scalings for the reverse sweep (or base null)
    int64_t U;
    int I, m, T, K, nck, hs, L, x_bf16;
    float c2;              // -1 / (eps ln 2): exponent scale of a cost
    float eps_ln2;         // eps ln 2: base-2 potential -> cost units
};

// Buffer of the tile reverse sweep (fr_tile.hip): per consumer of a batch,
// the row and column factors of every iteration and the reference kernels.
struct TileBuf {
    char* base;        // batch consumers x stride bytes
    size_t stride;     // bytes per consumer
    int64_t batch;     // consumers per batch
};
// Reference rebases of the tile reverse sweep kept per consumer.
constexpr int kTileEpochs = 16;

struct BwdArgs {
    const float* C;        // [U][I][m] cost (read)
    const float* r;        // [U][I]
    const float* e;        // [m-1]
    const float* hist;     // [U][nck][hs] checkpoints written by the forward
    const double* imp;     // [I]
    float* dC;             // [U][I][m] gF * dF/dC (or null)
    float* dr;             // [U][I] gF * dF/dr (or null)
    float* Cw;             // cost to update in place (or null)
    float* mom;            // Adam first moment (or null)
    float* vel;            // Adam second moment (or null)
    const int64_t* step_ptr;  // device Adam step counter (or null: use step_const)
    const int32_t* stop;      // skip the launch when *stop != 0 (or null)
    const float* gw;          // implicit form: converged column potentials [U][hs]
    const float* phi;         // implicit form: row potentials [U][I]
    int cg_max;               // implicit form: conjugate-gradient iteration cap
    int absorb;               // scaling-form sweep: also rebase every `absorb` iterations
    float cg_tol;             // implicit form: relative residual to stop at
    int64_t step_const;
    TileBuf tile;             // tile reverse sweep: factor buffer (fr_tile.hip)
    RowStore rows;            // tile reverse sweep: the forward's row scalings (or base null)
    uint32_t* flags;          // device flag word (FLAG_EPOCHS), or null
    double gF;
    int64_t U;
    int I, m, T, K, nck, hs, L, rule;
    float c2, inv_eps, lr, b1, b2, aeps;
};

// One work item of the batched kernels: a block of consumers of one instance.
struct BatchItem {
    int inst;
    int pad;
    int64_t u0;   // first consumer of the block
};

typedef void (*FwdLaunch)(const FwdArgs&, int grid, int block, size_t lds, hipStream_t);
typedef void (*BwdLaunch)(const BwdArgs&, int grid, int block, size_t lds, hipStream_t);
typedef void (*BFwdLaunch)(const FwdArgs*, const BatchItem*, int n, unsigned* counter, int grid,
                           int block, size_t lds, hipStream_t);
typedef void (*BBwdLaunch)(const BwdArgs*, const BatchItem*, int n, unsigned* counter, int grid,
                           int block, size_t lds, hipStream_t);
typedef int (*Occupancy)(int block, size_t lds);

struct FusedEntry {
    int mp, rows, lb;   // padded columns, rows per lane, launch bound (max block)
    bool wide;          // teams of whole waves (L >= 64); else L < 64
    bool recomp_f;      // forward recomputes each row's exponentials (register budget)
    bool recomp_b;      // backward likewise
    FwdLaunch fwd;
    BwdLaunch bwd;
    FwdLaunch fwdc;     // converged-map forward (warm start, tolerance)
    BwdLaunch ibwd;     // implicit-function gradient at a converged plan
    FwdLaunch fwds;     // scaling-form forward (same iterates as fwd)
    BFwdLaunch bfwd;    // persistent batched forms (launch bound 256, and 512 with one row)
    BBwdLaunch bbwd;
    Occupancy occ_bfwd;
    Occupancy occ_bbwd;
    BFwdLaunch bfwds;   // batched scaling-form forward
    Occupancy occ_bfwds;
    BwdLaunch bwds;     // scaling-form reverse sweep (K = 1)
    BBwdLaunch bbwds;   // batched scaling-form reverse sweep (K = 1)
    Occupancy occ_bbwds;
    BwdLaunch bwdl;     // reverse sweep with cb_rows rows of cost adjoints in LDS (or null)
    int cb_rows;
};

// Instantiated column classes.  Each class is compiled in its own translation
// unit (fr_fused.hip with -DFR_MP=<mp>).
#define FR_MP_CLASSES(X) X(5) X(8) X(10) X(11) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(50) X(64)
#define FR_DECL_ENTRIES(mp) const FusedEntry* fused_entries_##mp(int* n);
FR_MP_CLASSES(FR_DECL_ENTRIES)
#undef FR_DECL_ENTRIES

// Reverse-sweep block length when every iterate is kept (K == 1).
constexpr int kLoadBlock = 32;

// Tile kernels for large plans (fr_tile.hip): one consumer per block of 512
// lanes, plans of imin < I <= imax rows and m <= cmax columns, scaling form.
struct TileEntry {
    int cmax, imax, imin;
    FwdLaunch fwd;   // grid and block arguments ignored: one block per consumer
    BwdLaunch bwd;   // every iterate kept (K = 1); uses BwdArgs::tile
};
const TileEntry* tile_entry(int m, int I);
size_t tile_consumer_bytes(const TileEntry* e, int T);
size_t tile_row_bytes(const TileEntry* e, int T);
// Most bytes of row scalings the workspace keeps (consumers beyond are swept
// without them, in whole batches).
constexpr size_t kRowStoreCap = (size_t)144 << 30;
// Consumers per batch of the tile reverse sweep.
constexpr int64_t kTileBatch = 6144;

// Reductions over consumers (fr_reduce.hip).  F_hist[hdr->rep] receives F;
// advance: 0 leaves the counters, ADV_REP advances rep, ADV_REP_STEP rep and
// the Adam step.
enum { ADV_NONE = 0, ADV_REP = 1, ADV_REP_STEP = 2 };
void launch_impact(const float* y, int64_t U, int I, double* partial, int nchunk, double* imp,
                   double* F, double* F_hist, int64_t start_step, WsHeader* hdr, int advance,
                   hipStream_t s);

// Gradient-norm test of Algorithm 1 and the update it guards: ||g||_F in FP64
// (fixed order); if it is <= tol the loop stops (hdr->stopped), otherwise the
// Adam step advances and C is updated from g.  Every kernel returns at once
// once the loop has stopped.
int gnorm_blocks(int64_t n);
void launch_gnorm_update(const float* g, float* C, float* mom, float* vel, int64_t n, int rule,
                         float lr, float b1, float b2, float aeps, double* partial, double tol,
                         WsHeader* hdr, hipStream_t s);
void launch_rows_from_plan(const void* X, int x_bf16, const float* r, const float* e, int64_t U,
                           int I, int m, float* y, hipStream_t s);
int impact_chunks(int64_t U, int I);

// Batched impact reduction: one descriptor per instance.
struct RedDesc {
    const float* y;     // [U][I]
    double* partial;    // [nchunk][I]
    double* imp;        // [I]
    double* F_hist;     // F history of the instance (device)
    int64_t U;
    int I, nchunk;
};
void launch_impact_batched(const RedDesc* descs, int n_inst, const int2* tab1, int n1,
                           const int2* tab2, int n2, int64_t start_step, WsHeader* hdr,
                           hipStream_t s);
int impact_item_groups(int I);

// Evaluation metrics (fr_metrics.hip).
struct MetricsBufs {
    double* W;          // [U][I] exposure matrix
    double* partial;    // [nchunk][I] reduction partials
    int nchunk;
    double* rsum;       // [I] sum_u r_ui
    double* pmax;       // [I][tiles] row maxima of E per column tile
    double* diag;       // [I] E_ii
    WsHeader* hdr;      // scratch header for the reduction
    double* epart;      // [splits][I][I] partial E when the consumers are split
    int splits;
};
int metrics_tiles(int I);
int metrics_splits(int64_t U, int I);
void launch_metrics(const void* X, int x_bf16, const float* r, const float* e, int64_t U, int I,
                    int m, const MetricsBufs& b, double* out, double* envy, double* imp,
                    hipStream_t s);

// Unfused baseline form (fr_plain.hip).
struct PlainBufs {
    float *fh, *gh, *y, *cbar, *fbar, *fbar0, *gbar;
    double *imp, *partial;
    WsHeader* hdr;
    int nchunk;
};
void plain_forward(const float* C, const float* r, const float* e, int64_t U, int I, int m,
                   float eps, int T, const PlainBufs& b, void* X, int bf16, hipStream_t s);
void plain_backward_update(float* C, const float* r, const float* e, int64_t U, int I, int m,
                           float eps, int T, const PlainBufs& b, float* mom, float* vel, int rule,
                           float lr, float b1, float b2, float aeps, bool apply, hipStream_t s);

// Baseline rankings (fr_baselines.hip).
void launch_maxrele(const float* r, int64_t U, int I, int m, int32_t* sel, hipStream_t s);
void launch_greedy(const float* r, const float* e, int64_t U, int I, int m, int32_t* sel,
                   double* imp, hipStream_t s);
void launch_plan_from_sel(const int32_t* sel, int64_t U, int I, int m, void* X, int bf16,
                          hipStream_t s);

}  // namespace fr
