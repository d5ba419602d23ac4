/*
 * tucker_batch.h -- many independent decompositions in one call. Each tensor
 * is decomposed exactly as tucker_mp / tucker_hooi would (Sections 4.4 and
 * 4.2); the call overlaps them on the GPU by running one host worker per
 * stream, each taking the next undecomposed tensor until none is left.
 * Conventions ([dev], [host], ownership, status codes) are those of
 * tucker.h.
 */
#ifndef TUCKER_BATCH_H
#define TUCKER_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "tucker.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of ONE per-stream workspace of tucker_batched: the largest
   tucker_workspace_bytes over the `count` tensors (algo TK_ALGO_HOOI or
   TK_ALGO_MP), each with its own launch choices when `tunes` is given.
   Host only. */
int tucker_batched_workspace_bytes(int32_t algo, int32_t count, const tk_coo *X, const int32_t *core_dims,
                                   const tk_opts *opt, const tk_tune *tunes, size_t *bytes);

/* Decompose tensors X[0..count) with core sizes core_dims[3t..3t+3).
     cores        [host] count [dev] pointers (J1*J2*J3 doubles each)
     factors      [host] 3*count [dev] pointers: factors[3t + n] is In x Jn
     fit_history  [host] count * opt->max_iters doubles, row t for tensor t
     iters_done   [host] count
     status       [host] count: each tensor's own status code
     stats        [host] count tk_stats, or NULL
     tunes        [host] count launch choices (tensor t uses tunes[t] in place
                  of opt->tune), or NULL
     nstreams     1..64 streams; workspaces[s] (bytes each) serves streams[s]
   Returns TK_OK when every tensor succeeded, TK_WARN_NOCONV if one only
   warned, else the first (lowest index) error status; TK_ERR_ARG (before
   any device work) for a bad count, nstreams, pointer array, opt->trace
   set (one trace cannot take the events of concurrent decompositions), or
   any tensor that tucker_workspace_bytes would reject. The device of the calling
   thread is used by every worker. */
int tucker_batched(int32_t algo, int32_t count, const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                   double *const *cores, double *const *factors, double *fit_history, int32_t *iters_done,
                   int32_t *status, tk_stats *stats, const tk_tune *tunes, int32_t nstreams,
                   void *const *workspaces, size_t workspace_bytes, void *const *streams);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_BATCH_H */
