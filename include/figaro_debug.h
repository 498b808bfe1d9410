/*
 * figaro_debug.h -- inspection entry points for tests (not needed for normal
 * use).
 */
#ifndef FIGARO_DEBUG_H
#define FIGARO_DEBUG_H

#include "figaro.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Run the forward pass up to (not including) the post-processing TSQR and
 * copy the stack of partial R factors and root rows to the host:
 * host_out receives figaro_debug_stack_rows() rows of n columns, column-major
 * with leading dimension figaro_debug_stack_rows().  Synchronises `stream`.
 * FIGARO_EUNSUPPORTED for plans of more than 128 columns. */
int64_t figaro_debug_stack_rows(figaro_plan_t plan);
figaro_status figaro_debug_stack(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                                 double *host_out, hipStream_t stream);

/* Rows per register tile of one wave of the dense TSQR kernel for n columns
 * and a kernel variant (as in figaro_plan_options), or -1 if out of range. */
int64_t figaro_debug_tile_rows(int32_t n, int32_t variant);

/* Rows that one workgroup of the dense TSQR kernel folds with
 * tiles_per_wave tile steps (the waves of a workgroup fold separate tiles
 * for n <= 40 and share each tile for wider matrices), or -1. */
int64_t figaro_debug_dense_rows(int32_t n, int32_t variant, int64_t tiles_per_wave);

/* One launch of the dense TSQR step (section "Post-processing") on a plain
 * matrix: `in` is a device column-major rows x n matrix (ld_in >= rows);
 * workgroup b folds rows [b*W, (b+1)*W), W = figaro_debug_dense_rows(n,
 * variant, tiles_per_wave), into one n x n R.  With workgroups ==
 * 1 and final_r != NULL the sign-normalised R is written to final_r (n x n,
 * column-major); otherwise workgroup b writes its R to rows b*n..b*n+n-1 of
 * `out` (column-major, ld_out >= workgroups * n).  FIGARO_EINVAL when the
 * workgroups do not cover the rows or an argument is out of range. */
figaro_status figaro_debug_dense_step(int32_t n, int64_t rows, const double *in, int64_t ld_in,
                                      int32_t workgroups, int64_t tiles_per_wave, int32_t variant,
                                      double *out, int64_t ld_out, double *final_r, hipStream_t stream);

/* Layout of the stack: up to max_regions triples (block id, first row, rows)
 * written to regions_host; returns the number of regions (-1 for plans of
 * more than 128 columns, which reduce their stack in place). */
int32_t figaro_debug_stack_layout(figaro_plan_t plan, int64_t *regions_host, int32_t max_regions);

#ifdef __cplusplus
}
#endif

#endif
