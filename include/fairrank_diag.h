/*
 * fairrank_diag.h -- diagnostics of libfairrank: per-kernel timing of the
 * fused solver and microbenchmarks of the device ceilings it is measured
 * against.  Not needed to use the solver (include/fairrank.h).
 */
#ifndef FAIRRANK_DIAG_H
#define FAIRRANK_DIAG_H

#include <stddef.h>
#include <stdint.h>

#include "fairrank.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Kernel timing.  While enabled, fr_solve launches its kernels directly
 * (no graph) and brackets every fused forward and backward launch with HIP
 * events on the call's stream.  fr_ctx_kernel_times returns the milliseconds
 * and launch counts accumulated since timing was last enabled (host
 * pointers, each optional). */
fr_status fr_ctx_set_timing(fr_ctx* ctx, int enable);
fr_status fr_ctx_kernel_times(fr_ctx* ctx, double* fwd_ms, int64_t* fwd_launches,
                              double* bwd_ms, int64_t* bwd_launches);

/* The arithmetic form (FR_FORM_LOG or FR_FORM_SCALING) of the fused forward
 * and reverse sweep that fr_solve runs on this context for a problem of this
 * shape with checkpoint interval K (0 = every iterate), at the launch shape
 * fr_get_launch reports; 2 for the scaling form on the tile kernels of large
 * plans (launch shape reported as 512 lanes, 0 rows).  Host pointers, each
 * optional. */
fr_status fr_ctx_kernel_forms(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m,
                              int32_t checkpoint_every, int32_t* fwd_form, int32_t* bwd_form);

/* Rows of cost adjoints per lane that the log-domain reverse sweep keeps in
 * LDS for a problem of this shape (same arguments as fr_ctx_kernel_forms):
 * 0 when they all stay in registers.  Teams of more than 256 lanes whose
 * costs, cost adjoints and a pass's temporaries exceed the registers (the
 * two-pass kernels, e.g. m = 50 with two rows per lane) keep as many of the
 * rows of cost adjoints as fit in LDS, all but one at most, when the block's
 * LDS allows it (the kernel then shows as k_bwdl).
 * *rows is a host pointer. */
fr_status fr_ctx_bwd_lds_rows(fr_ctx* ctx, int64_t n_users, int32_t n_items, int32_t m,
                              int32_t checkpoint_every, int32_t* rows);

/* Row store of the tile kernels (plans of 40..50 columns and 513..1024
 * items, every iterate kept): while enabled (the default), the forward that
 * precedes a reverse sweep keeps each consumer's row scaling of every
 * iteration and the reference kernel of each stretch between rebases in the
 * workspace, and the sweep works in those stretches and takes the row
 * scalings from there instead of forming the row sums again (one multiply-add
 * per plan cell and iteration fewer).  The workspace (fr_workspace_bytes)
 * reserves T * 1024 + 16 * 1088 floats per consumer for it, for all consumers
 * or, beyond 144 GiB, for whole batches of 6144 consumers; the others are
 * swept without it.  A forward that had more than 16 stretches makes the
 * sweep report FR_E_UNSUPPORTED.  enable = 0 sweeps every consumer without
 * the store (its own rebases; the same limit of 16 applies to them). */
fr_status fr_ctx_set_row_store(fr_ctx* ctx, int enable);

/* ALU microbenchmark on the current device, default stream, synchronous:
 * kind 0 = dependent chains of v_exp_f32, 1 = chains of FP32 FMA, 2 = one
 * exponential followed by five FMAs.  `blocks` blocks of 256 threads, each
 * lane running `iters` steps on 8 independent chains.  *ms_out = kernel time,
 * *ops_out = lane-steps executed (exps, FMAs, or exp+5 FMA groups). */
fr_status fr_diag_alu(int kind, int blocks, int iters, double* ms_out, double* ops_out);

/* HBM copy of `bytes` (multiple of 16) from src to dst (device), `reps`
 * timed repetitions after one warm-up on `stream`; *ms_out = mean time per
 * copy.  Moves 2 * bytes per repetition; its profiler byte counts calibrate
 * those of the solver's kernels. */
fr_status fr_diag_copy(const void* src, void* dst, size_t bytes, int reps, double* ms_out,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FAIRRANK_DIAG_H */
