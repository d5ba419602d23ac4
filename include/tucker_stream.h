/*
 * tucker_stream.h -- Multislice Projection of a sparse third-order tensor
 * held in HOST memory, streamed through bounded device memory.
 *
 * The paper runs MP past the size of RAM by sorting the nonzeros once and
 * reading one slice file at a time in every sweep (Section 4.3, slice
 * construction; Section 5.1, varying tensor sizes). This entry point does the
 * same against device memory: the host sorts the nonzeros once into six
 * orderings (each leaf mode with each of the two other modes as the major
 * key), and every sweep uploads them slab by slab (consecutive values of the
 * major index) into two device buffers of `slab_bytes` each, while the
 * previous slab is projected and its share of the Gram accumulated. Results
 * equal tucker_mp's from the same start up to the grouping of the Gram's
 * sums (FP64 in FP64 mode). Conventions as tucker.h, except where marked.
 */
#ifndef TUCKER_STREAM_H
#define TUCKER_STREAM_H

#include <stddef.h>
#include <stdint.h>

#include "tucker.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of device workspace tucker_mp_streamed needs: the Grams, the
   eigensolver, factor copies, the core's intermediate (I2 x J1 x J3
   doubles) and two slab buffer sets of slab_bytes for the dense projection
   plus slab_bytes / 8 entries and their slot pointers. Host only.
   TK_ERR_ARG as tucker_mp_streamed. */
int tucker_mp_streamed_workspace(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                                 size_t slab_bytes, size_t *bytes);

/* MP (Figure 7) of X whose idx[n] and vals are HOST pointers (the tensor
   need not fit device memory: only the slabs, the Grams and the factors
   live there).
     slab_bytes  size of one dense slab buffer; one slice of every projection
                 (I_n rows of J_m padded to 16 bytes, for each pair n != m;
                 for the core's FP32 / FP64 projection, I1 rows of J3) must
                 fit, and no slice may hold more than slab_bytes / 8 entries
                 (else TK_ERR_ARG, before any device work)
     opt         precision TK_FP64, TK_FP32 or TK_MIXED_BF16; init
                 TK_INIT_RANDOM (Figure 5's random start, the same values
                 tucker_mp draws) or TK_INIT_GIVEN (factors[1], factors[2]);
                 no trace, no HO-SVD fit report (TK_ERR_ARG otherwise)
     core, factors, fit_history, iters_done, stats: as tucker_mp
                 (stats.streamed_bytes / streamed_slabs count the uploads).
   The host sort takes O(nnz) time and about 72 bytes of host memory per
   nonzero; the call creates one more HIP stream (default priority), two
   events pairs and two pinned host staging buffers, all released before it
   returns. TK_ERR_INDEX / TK_ERR_VALUE are detected on the host. */
int tucker_mp_streamed(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt, size_t slab_bytes,
                       double *core, double *const *factors, double *fit_history, int32_t *iters_done,
                       tk_stats *stats, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_STREAM_H */
