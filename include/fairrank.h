/*
 * fairrank.h -- C ABI of the MI355X (gfx950) impact-based fair ranking solver.
 *
 * The solver implements the gradient-ascent method of Uehara et al., "Fast
 * solution to the fair ranking problem using the Sinkhorn algorithm":
 *
 *   * Section 2 (problem nsw): one plan X_u in R^{I x m} per consumer u, rows
 *     summing to 1 (Eq. dsm1), the m-1 real position columns summing to 1
 *     (Eq. dsm2), x >= 0 (Eq. dsm4), and the last column a dummy position
 *     whose column sums to I - m + 1.  Item impact (Eq. Imp)
 *         Imp_i = sum_u sum_{k<m} r(u,i) e(k) x_uik
 *     and objective (Eq. objF) F = sum_i log Imp_i  (log of the Nash social
 *     welfare).
 *   * Section 3 (problem otp): X_u is the entropic optimal transport plan of a
 *     cost matrix C_u, computed by T log-domain Sinkhorn iterations from a cold
 *     start; F is maximised over C (problem nsw2) by gradient ascent
 *     (Algorithm 1), the gradient taken by the chain rule through the T
 *     iterations, the step by Adam (Section 4.1) or plain ascent.
 *
 * Conventions shared by every entry point
 *   * Pointers are DEVICE pointers unless marked (host).  Layouts are dense
 *     row-major: C, X, dC, Adam moments [U][I][m] with m fastest; r, dr
 *     [U][I]; potentials [U][I+m] (f then g); e [m-1]; impacts [I] (double).
 *   * The caller owns and allocates every buffer, including the workspace
 *     sized by fr_workspace_bytes; the library never frees caller memory.
 *     A context owns only its launch-configuration (autotune) cache and its
 *     captured graphs.
 *   * All calls are asynchronous on the given stream (a hipStream_t passed
 *     as void*; NULL = the null stream) unless documented otherwise.
 *     fr_solve and fr_solve_plain return synchronised; given NULL they wait
 *     for the null stream, run on a stream of the context (a graph cannot be
 *     captured on the null stream) and wait for it.  A context must not be
 *     used from two host threads at once.
 *   * Every call returns an fr_status and never aborts.  Argument errors are
 *     detected on the host and returned before anything is enqueued.
 *     Conditions found on the device (a non-finite value, an impact <= 0) set
 *     a flag word in the workspace; fr_solve reports them (it synchronises),
 *     after the asynchronous calls fr_sync_status does.
 *   * Sizes: 1 <= U, 2 <= m <= I (the dummy mass I-m+1 must be >= 1),
 *     m <= 64, I <= 4096, eps > 0 finite, T >= 1 (FR_E_SHAPE / FR_E_PARAM
 *     outside).  The fused kernels hold a consumer's plan in the registers
 *     of at most 1024 lanes, which covers I <= 4096 for m <= 32 and
 *     I <= 2048 for 32 < m <= 64; larger plans get FR_E_UNSUPPORTED from the
 *     solver entry points (the plain form, fr_nsw, fr_metrics and the
 *     baselines take every valid size).
 */
#ifndef FAIRRANK_H
#define FAIRRANK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FR_OK = 0,
    FR_E_NULL = 1,        /* a required pointer is NULL                          */
    FR_E_SHAPE = 2,       /* sizes out of range (see above)                      */
    FR_E_PARAM = 3,       /* eps, T, step counts or optimiser settings invalid   */
    FR_E_WORKSPACE = 4,   /* workspace smaller than fr_workspace_bytes           */
    FR_E_DEVICE = 5,      /* a HIP runtime call failed                           */
    FR_E_NONFINITE = 6,   /* device found a NaN/Inf in an impact or objective    */
    FR_E_ZERO_IMPACT = 7, /* device found Imp_i <= 0, so log Imp_i is undefined  */
    FR_E_UNSUPPORTED = 8  /* valid request this build does not handle            */
} fr_status;

typedef enum { FR_F32 = 0, FR_BF16 = 1 } fr_dtype;   /* storage type of X     */
typedef enum { FR_ADAM = 0, FR_GD = 1 } fr_rule;     /* ascent rule           */
typedef enum { FR_FORM_LOG = 0, FR_FORM_SCALING = 1 } fr_form;  /* Sinkhorn form */

typedef struct fr_ctx fr_ctx;

/* One fair-ranking instance (Section 2 notation). */
typedef struct {
    int64_t n_users;        /* |U| >= 1                                          */
    int32_t n_items;        /* |I|, 2 <= |I| <= 4096                             */
    int32_t m;              /* columns of X_u incl. the dummy, 2 <= m <= min(I,64)*/
    const float* r;         /* [U][I] relevance r(u,i) (device)                   */
    const float* e;         /* [m-1] exposure of the real positions (device)      */
    float eps;              /* entropic weight of problem otp, > 0                */
    int32_t sinkhorn_iters; /* T >= 1 full (row + column) iterations, cold start  */
} fr_problem;

/* Outer loop of Algorithm 1. */
typedef struct {
    int32_t rule;             /* fr_rule                                            */
    float lr;                 /* step size (Adam lr, or ascent step for FR_GD)     */
    float beta1, beta2;       /* Adam moment decays, e.g. 0.9 and 0.999            */
    float adam_eps;           /* Adam denominator guard, e.g. 1e-8                 */
    int32_t outer_steps;      /* N >= 0 ascent steps                               */
    int32_t checkpoint_every; /* K: Sinkhorn potentials kept every K iterations for
                                 the reverse sweep (1 = keep all, no recomputation;
                                 0 = let the library choose)                       */
    double grad_tol;          /* t of Algorithm 1: ascend only while ||dF/dC||_F > t;
                                 0 = off (exactly outer_steps updates).  With t > 0
                                 the gradient goes through the workspace, its norm
                                 is tested in FP64, and after a stop C (and so F)
                                 no longer changes                                 */
    float sinkhorn_tol;       /* 0: the paper's Algorithm 1 (T iterations from g = 0,
                                 gradient by reverse mode through them).  > 0: the
                                 converged-map form: each outer step's Sinkhorn
                                 starts from the previous step's column potentials
                                 and stops once no potential moves by more than
                                 sinkhorn_tol (log2 units; at most T iterations),
                                 and the gradient is the implicit-function gradient
                                 of the balanced plan (no reverse sweep).  Not for
                                 fr_solve_plain or fr_solve_batched.               */
    int32_t cg_iters;         /* converged-map form: conjugate-gradient cap of the
                                 implicit gradient's m x m solve (0 = 2m + 8)     */
} fr_optim;

/* ---------------------------------------------------------------- context */
/* Creates a context bound to HIP device `device` (made current by every call). */
fr_status fr_ctx_create(int device, fr_ctx** out);
void fr_ctx_destroy(fr_ctx* ctx);

/* Form of the fixed-T Sinkhorn forward that every later call on this context
 * runs (fr_step, fr_solve, fr_solve_batched, fr_autotune; the plain solve and
 * the backward's checkpoint recomputation keep the log domain).  Both forms
 * compute the same T iterates (Section 3's Sinkhorn iteration from g = 0);
 * they differ in arithmetic only.
 *   FR_FORM_LOG     log-domain: one base-2 exponential per cell and
 *                   iteration on centred scaled costs.
 *   FR_FORM_SCALING (default) matrix scaling u = 1/(K v), v = b/(K^T u) on a
 *                   kernel K = 2^(a + gamma + phi) held in registers: two
 *                   multiply-adds per cell and iteration, no exponential; the
 *                   scalings are absorbed into the potentials (and K rebuilt
 *                   from C, one exponential per cell) whenever a column
 *                   scaling leaves [2^-32, 2^32], and also every absorb_every
 *                   iterations if absorb_every > 0.  With every iterate stored (K = 1)
 *                   the reverse sweep (fr_backward, fr_solve) runs in the
 *                   same form on launch shapes whose rows fit the registers
 *                   (a reference kernel rebased from C when a column
 *                   scaling leaves the range); other shapes keep the log
 *                   domain.  The gradient is the same.
 * FR_E_PARAM for an unknown form or absorb_every < 0.  Host only. */
fr_status fr_ctx_set_form(fr_ctx* ctx, int32_t form, int32_t absorb_every);

/* Bytes of workspace every call below needs for this problem (optim may be
 * NULL: then K = 1 and no Adam state; a positive grad_tol or sinkhorn_tol adds
 * the room those modes need).  Written to *out (host).  FR_E_PARAM for a
 * negative or non-finite tolerance or negative cg_iters. */
fr_status fr_workspace_bytes(const fr_problem* prob, const fr_optim* optim, size_t* out);

/* Prepares a newly allocated workspace (clears its device flags and step
 * counter; enqueued on the stream).  Call once per allocation, before the
 * workspace's first use; the flags then persist across calls until
 * fr_sync_status reads and clears them.  ws_bytes >= 256. */
fr_status fr_workspace_init(fr_ctx* ctx, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- forward */
/* Section 3 + Eqs. Imp, objF: X_u = Sinkhorn_T(C_u) for every consumer (T
 * iterations from g = 0, each a row then a column half-step; computed in the
 * scaling form with log-domain absorption by default, or in the log domain
 * after fr_ctx_set_form -- the same iterates), then Imp and F.  C [U][I][m]
 * float.  Outputs, each optional (NULL = not written):
 * X [U][I][m] in x_dtype (BF16 rounds to nearest even; the impacts are always
 * taken from the FP32 plan), pot [U][I+m] float potentials f then g in cost
 * units, imp [I] double, F [1] double.  Impacts are summed over consumers in
 * FP64 in a fixed order (bitwise reproducible). */
fr_status fr_step(fr_ctx* ctx, const fr_problem* prob, const float* C, void* X,
                  fr_dtype x_dtype, float* pot, double* imp, double* F,
                  void* ws, size_t ws_bytes, void* stream);

/* fr_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as fr_step, with no workspace argument.  The
 * workspace fr_step would take (header, impacts, impact partials, the per-row
 * impact contributions) lives in a device array that the library holds on
 * every GPU it runs on, 64 MiB, which limits the problem to about
 * |U| |I| <= 14.9 million (precisely: the bytes fr_step needs before its
 * history, 4 |U| |I| + 8 |I| ceil(|U|/16) + 8 |I| + 256, rounded up per part
 * to 256).  Larger problems return FR_E_WORKSPACE before anything is
 * enqueued.  imp [I] and F [1] are required here (FR_E_NULL otherwise): the
 * device conditions fr_sync_status reports for fr_step are not reported for
 * this call; an impact <= 0 or non-finite shows as a non-finite F.  The call
 * allocates nothing (no hipMalloc, no library allocation).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams or threads without ordering between them) race and their results
 * are undefined.  FR_E_DEVICE if the array's address could not be resolved
 * when the context was created. */
fr_status fr_step_noalloc(fr_ctx* ctx, const fr_problem* prob, const float* C, void* X,
                          fr_dtype x_dtype, float* pot, double* imp, double* F, void* stream);

/* Eqs. Imp and objF for a given plan X [U][I][m] (x_dtype): imp [I] and F [1]
 * (double, either optional).  X need not be a Sinkhorn output. */
fr_status fr_nsw(fr_ctx* ctx, const fr_problem* prob, const void* X, fr_dtype x_dtype,
                 double* imp, double* F, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- baselines */
/* The deterministic rankings compared with Algorithm 1 in Section 4.1.  Both
 * write sel [U][m-1] int32 (device): the item each consumer sees at each real
 * position; every other item goes to the dummy position.  X (optional, NULL =
 * not written) receives the 0/1 plan [U][I][m] in x_dtype, a feasible point of
 * problem otp's polytope.  Asynchronous on the stream; argument errors return
 * before anything is enqueued (the problem is checked as for fr_step; eps and
 * T are not used).
 *
 * fr_rank_maxrele: MaxRele -- each consumer's items in descending order of
 *   relevance (equal relevances by item index).  One wave per consumer.
 * fr_rank_greedy: NSW(Greedy).  The paper says only that greedy picks items
 *   by F(X) for each position; the rule fixed here: positions k = 0..m-2 in
 *   order, consumers in index order within a position, each taking the item
 *   it has not placed yet whose placement raises F = sum_i log Imp_i (Eq.
 *   objF) the most, i.e. the largest r_ui / Imp_i in FP64 (Imp_i = 0 counts as
 *   +inf), then the larger r_ui, then the smaller index.  The U (m-1)
 *   decisions form one chain and run in a single block.  imp (optional, FP64
 *   [I], device) receives the impacts of the result, accumulated in decision
 *   order. */
fr_status fr_rank_maxrele(fr_ctx* ctx, const fr_problem* prob, int32_t* sel, void* X,
                          int32_t x_dtype, void* stream);
fr_status fr_rank_greedy(fr_ctx* ctx, const fr_problem* prob, int32_t* sel, void* X,
                         int32_t x_dtype, double* imp, void* stream);

/* Evaluation metrics of a plan X [U][I][m] (x_dtype), from the list of
 * evaluation metrics in Section 4.1.  With W_uj = sum_{k<m-1} e_k x_ujk and
 * E_ij = sum_u r_ui W_uj (the impact item i would get with item j's
 * allocation; E_ii is Eq. Imp):
 *   out[0] user utility        = sum_i E_ii / U
 *   out[1] mean max envy       = mean_i (max_j E_ij - E_ii)
 *   out[2] items better off    = fraction of i with E_ii > 1.1 Imp_i^unif
 *   out[3] items worse off     = fraction of i with E_ii < 0.9 Imp_i^unif
 * where Imp_i^unif = (sum_u r_ui)(sum_{k<m-1} e_k) / I is the impact under the
 * uniform ranking policy.  out: 4 doubles (device).  Optional (device, NULL =
 * not written): envy [I] (max_j E_ij - E_ii) and imp [I] (E_ii).  W and E are
 * FP64 (E on FP64 matrix cores; E is reduced tile by tile and never stored);
 * the better / worse decisions are taken in FP64.  Asynchronous on the stream.
 * Workspace from fr_workspace_bytes_metrics (independent of the solver's). */
fr_status fr_workspace_bytes_metrics(const fr_problem* prob, size_t* out);
fr_status fr_metrics(fr_ctx* ctx, const fr_problem* prob, const void* X, fr_dtype x_dtype,
                     double* out, double* envy, double* imp, void* ws, size_t ws_bytes,
                     void* stream);

/* --------------------------------------------------------------- backward */
/* Value and gradient of the converged map (the converged-map form of
 * fr_optim.sinkhorn_tol): Sinkhorn from g = 0 until no column potential moves
 * by more than sinkhorn_tol (log2 units; at most T iterations), Imp and F of
 * that plan, then gF * dF/dC by the implicit function theorem at the balanced
 * plan: dF/dc_ik = -(1/eps) x_ik (G_ik - lam_i - mu_k) with (lam, mu) from the
 * optimality conditions (gauge mu_{m-1} = 0; an m x m Schur system solved by
 * preconditioned conjugate gradients, at most cg_iters iterations, 0 = 2m + 8),
 * and dr = gF * dF/dr.  imp [I], F [1], dC [U][I][m]; imp, F and dr optional.
 * Workspace: fr_workspace_bytes with an optim whose sinkhorn_tol > 0. */
fr_status fr_grad_converged(fr_ctx* ctx, const fr_problem* prob, const float* C,
                            float sinkhorn_tol, int32_t cg_iters, double gF, double* imp,
                            double* F, float* dC, float* dr, void* ws, size_t ws_bytes,
                            void* stream);

/* Section 3 ("chain rule"): reverse mode through the T unrolled Sinkhorn
 * iterations.  Given C and the impacts imp [I] of X(C) (from fr_step), writes
 * dC = gF * dF/dC [U][I][m] and, if dr is not NULL, dr = gF * dF/dr [U][I].
 * The forward is recomputed from C; potentials are kept every
 * checkpoint_every iterations (>= 1) and the segments between them are
 * recomputed during the reverse sweep.  Asynchronous: conditions found on the
 * device (a tile plan whose sweep needs more than 16 reference kernels,
 * FR_E_UNSUPPORTED) are reported by fr_sync_status on the same workspace. */
fr_status fr_backward(fr_ctx* ctx, const fr_problem* prob, const float* C, const double* imp,
                      double gF, float* dC, float* dr, int32_t checkpoint_every,
                      void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------- Algorithm 1 */
/* N = optim->outer_steps ascent steps on C (in: C_0, out: C_N).  Step n runs
 * the forward at C_n, records F_n, takes dF/dC and updates C.  A final forward
 * gives X(C_N) and F_N, so F_hist [N+1] (double) holds F_0..F_N.  Adam state
 * adam_m, adam_v [U][I][m] (in/out; zero them for a fresh start; ignored for
 * FR_GD) and start_step (Adam's step count before this call) make a run of
 * N1 steps followed by one of N2 steps identical to one run of N1+N2 steps.
 * X_out (x_dtype, optional) receives X(C_N).  The step is captured once as a
 * HIP graph and replayed N times.  Synchronises the stream before returning
 * and reports device flags. */
fr_status fr_solve(fr_ctx* ctx, const fr_problem* prob, const fr_optim* optim, float* C,
                   float* adam_m, float* adam_v, int64_t start_step, void* X_out,
                   fr_dtype x_dtype, double* F_hist, void* ws, size_t ws_bytes, void* stream);

/* Same method, but one kernel launch per Sinkhorn half-iteration with the
 * potentials in HBM and the reverse sweep reading every stored iterate: the
 * unfused GPU form used as the performance baseline.  Same arguments and
 * results as fr_solve (up to rounding); workspace from
 * fr_workspace_bytes_plain. */
fr_status fr_solve_plain(fr_ctx* ctx, const fr_problem* prob, const fr_optim* optim, float* C,
                         float* adam_m, float* adam_v, int64_t start_step, void* X_out,
                         fr_dtype x_dtype, double* F_hist, void* ws, size_t ws_bytes,
                         void* stream);
fr_status fr_workspace_bytes_plain(const fr_problem* prob, size_t* out);

/* Many independent instances of uneven (U, I, m) solved together: every phase
 * of an outer step (forward, impact/F reduction, backward + update) is one
 * persistent kernel per column class whose blocks take (instance, consumer
 * block) work items, longest first, from a device counter until the list is
 * exhausted; the outer step is captured as one HIP graph and replayed N
 * times.  probs (host array of n_inst fr_problem, device r and e), and host
 * arrays of device pointers: C [n_inst] (each [U][I][m], in/out), adam_m,
 * adam_v [n_inst] (NULL or entries ignored for FR_GD), X [n_inst] (NULL or
 * NULL entries: not written) and F_hist [n_inst] (each N+1 doubles).  Each
 * instance's results equal those of fr_solve on it.  Synchronises. */
fr_status fr_workspace_bytes_batched(int32_t n_inst, const fr_problem* probs,
                                     const fr_optim* optim, size_t* out);
fr_status fr_solve_batched(fr_ctx* ctx, int32_t n_inst, const fr_problem* probs,
                           const fr_optim* optim, float* const* C, float* const* adam_m,
                           float* const* adam_v, int64_t start_step, void* const* X,
                           fr_dtype x_dtype, double* const* F_hist, void* ws, size_t ws_bytes,
                           void* stream);

/* ------------------------------------------------------------ utilities */
/* Synchronises the stream and returns the device flags recorded in ws
 * (FR_E_NONFINITE / FR_E_ZERO_IMPACT), then clears them. */
fr_status fr_sync_status(fr_ctx* ctx, void* ws, void* stream);

/* Static description of a status code. */
const char* fr_status_string(fr_status s);

/* Adam's step count held in the workspace after fr_solve / fr_solve_plain:
 * start_step plus the number of updates applied (fewer than outer_steps when
 * the gradient-norm test of Algorithm 1 stopped the loop), the norm
 * ||dF/dC||_F of the last gradient tested (0 when grad_tol was 0), and, for
 * the converged-map form, the Sinkhorn iterations used summed over consumers
 * and forward passes (0 otherwise).  Synchronises the stream; out pointers
 * are host memory (each optional). */
fr_status fr_solve_progress(fr_ctx* ctx, void* ws, void* stream, int64_t* steps,
                            double* last_gnorm, int64_t* sinkhorn_iters);

/* Launch configuration of the fused kernels for plans of a given shape:
 * lanes per consumer (1..64 as a power of two, or a multiple of 64 up to
 * 1024) and plan rows held by each lane.  fr_set_launch overrides the
 * library's choice for (I, m) (FR_E_UNSUPPORTED if no kernel is instantiated
 * for it); fr_get_launch reports the shape a problem of n_users consumers
 * and this (I, m) runs with: the override if one is set, else the library's
 * choice from its issue model, which depends on n_users. */
fr_status fr_set_launch(fr_ctx* ctx, int32_t n_items, int32_t m, int32_t lanes,
                        int32_t rows_per_lane);
fr_status fr_get_launch(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m, int32_t* lanes,
                        int32_t* rows_per_lane);

/* Autotuner: times every instantiated launch shape (lanes, rows per lane)
 * that covers the problem's I rows, running the fused forward, the impact
 * reduction and the fused backward on this problem and cost tensor C with
 * min(T, iters) Sinkhorn iterations (HIP events on the stream; synchronises),
 * and keeps the fastest for (I, m) in the context.  batched != 0 restricts the
 * search to shapes the batched kernels accept (teams of at most 256 lanes).
 * Needs the workspace of fr_workspace_bytes.  The choice is written to
 * *lanes_out, *rows_out (host, optional). */
fr_status fr_autotune(fr_ctx* ctx, const fr_problem* prob, const float* C, int32_t batched,
                      int32_t iters, void* ws, size_t ws_bytes, void* stream, int32_t* lanes_out,
                      int32_t* rows_out);

#ifdef __cplusplus
}
#endif
#endif /* FAIRRANK_H */
