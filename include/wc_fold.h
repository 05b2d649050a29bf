/* Float map-reduce of Section 4.2 of "MapReduce for Counting Word Frequencies with MPI and
 * GPUs": a sum over i = 1..n of a term mapped from the index, the paper's second workload for
 * comparing map-reduce implementations. Part of libwc.so; statuses as in wc.h. */
#ifndef WC_FOLD_H
#define WC_FOLD_H

#include "wc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define WC_FOLD_SQRT         0u /* term i = sqrt(i) */
#define WC_FOLD_ALT_HARMONIC 1u /* term i = (-1)^(i+1) / i; the sums tend to ln 2 */

/* Device workspace bytes wc_fold_sum needs for n terms (one double per workgroup). */
wc_status wc_fold_sum_plan(uint64_t n, uint64_t* workspace_bytes);

/* *d_out (device, one double) = sum over i = 1..n of term i, in binary64; 0 for n = 0.
 * Each term is correctly rounded; the terms are added in a fixed order (per-thread runs of
 * consecutive indices, then fixed trees), so a call gives the same bits every time and is
 * within (m + 23) * 2^-53 * sum |term| of the exactly rounded sum of the rounded terms, where
 * m = ceil(n / (256 * min(2048, ceil(n / 256)))) is the run length. d_workspace: device
 * memory of wc_fold_sum_plan() bytes, 8-byte aligned, owned by the caller. Asynchronous on
 * `stream` (a hipStream_t; NULL = default stream): *d_out is ready when the stream is.
 * Errors: WC_EINVAL for an unknown kind, n > 2^53 (indices must convert to double exactly),
 * NULL d_out or d_workspace, or a workspace smaller than the plan; WC_EDEVICE on a launch
 * failure. */
wc_status wc_fold_sum(uint32_t kind, uint64_t n, double* d_out, void* d_workspace,
                      uint64_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WC_FOLD_H */
