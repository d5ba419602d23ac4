/* Multislice Projection without explicit Grams, for tensors much sparser
 * than the squares of their mode sizes.
 *
 * Multislice Projection (Figure 7 of the paper, with the slice products
 * regrouped) takes each factor as the leading eigenvectors of
 *   M_n = sum over the two other modes m of T(m)_(n) T(m)_(n)^T,
 *   T(m) = X x_m A(m)^T.
 * tucker_mp forms every T(m) densely (one row per pair of coordinates of the
 * two other modes) and M_n (I_n x I_n) with a Gram kernel. This entry point
 * keeps T(m) only for the fibres that hold a nonzero and finds the leading
 * eigenvectors from products M_n Q = sum T_k (T_k^T Q) over the slices k of
 * the third mode, never forming M_n: memory and work grow with the number of
 * non-empty fibres instead of with I_n^2 and the product of two mode sizes.
 * Modes of at most 140 rows form M_n from products with the identity.
 *
 * The decomposition is the one tucker_mp computes (same start, sweep order,
 * eigensolver, core and fit, the paper's stopping rule); the products round
 * differently, so FP64 fits agree with tucker_mp's to about 1e-10.
 */
#ifndef TUCKER_IMPLICIT_H
#define TUCKER_IMPLICIT_H

#include "tucker.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes of tucker_mp_implicit for this problem (an upper bound:
 * it assumes every nonzero starts its own fibre). Returns TK_OK, or
 * TK_ERR_ARG for a problem or options that call rejects. */
int tucker_mp_implicit_workspace(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt, size_t *bytes);

/* Multislice Projection through implicit Gram products.
 * X: [dev] third-order COO as for tucker_mp (order 3; duplicates summed;
 *    I_a * I_b < 2^31 for every pair of modes; at most 2^31 - 3 nonzeros).
 * core_dims: [host] J_1..J_3, 1 <= J_n <= min(I_n, 128).
 * opt: precision TK_FP64 (FP64 projections and products), TK_FP32 (FP32
 *    projections, FP32 products summed per row in FP64) or TK_MIXED_BF16
 *    (BF16 projections from FP16 factor rows, FP32 products; the core from
 *    an FP32 projection); init TK_INIT_RANDOM (A(2), A(3) as tucker_mp's
 *    random start, from opt.seed) or TK_INIT_GIVEN (A(2), A(3) read from
 *    factors[1], factors[2]; orthonormal columns); max_iters >= 1; tol,
 *    eig_max_iters, eig_tol, timing and trace as for tucker_mp (the trace's
 *    TK_PHASE_GRAM events are the product kernels, one per Gram term and
 *    64-column slab); hosvd_fit must be 0; tune: the projection's fields.
 *    Other starts are TK_ERR_ARG.
 * core, factors, fit_history, iters_done, stats, workspace, stream: as for
 *    tucker_mp (device buffers; the workspace of
 *    tucker_mp_implicit_workspace bytes; stats.gram_ms / gram_calls count the
 *    product kernels).
 * Returns TK_OK, TK_WARN_NOCONV, or the errors of tucker_mp. */
int tucker_mp_implicit(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt, double *core,
                       double *const *factors, double *fit_history, int32_t *iters_done, tk_stats *stats,
                       void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif
