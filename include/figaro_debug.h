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
 * with leading dimension figaro_debug_stack_rows().  Synchronises `stream`. */
int64_t figaro_debug_stack_rows(figaro_plan_t plan);
figaro_status figaro_debug_stack(figaro_plan_t plan, const double *const *values, const int64_t *ld,
                                 double *host_out, hipStream_t stream);

/* Layout of the stack: up to max_regions triples (block id, first row, rows)
 * written to regions_host; returns the number of regions. */
int32_t figaro_debug_stack_layout(figaro_plan_t plan, int64_t *regions_host, int32_t max_regions);

#ifdef __cplusplus
}
#endif

#endif
