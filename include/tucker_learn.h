/*
 * tucker_learn.h -- learned warm start of the sparse Tucker library: the
 * pieces that compute it and train it on the GPU. The paper starts HOOI from
 * HO-SVD (Section 4.2) and MP from its pseudo HO-SVD (Section 4.4); this start
 * is an addition, used by tucker_hooi / tucker_mp with TK_INIT_LEARNED.
 * Conventions ([dev], [host], ownership, workspace, stream, status codes) are
 * those of tucker.h.
 *
 * For mode n (a = n+1, b = n+2 mod 3):
 *   S    = X_(n) Omega, In x 64 (FP32), Omega row of (i_a, i_b) generated
 *          from SplitMix64 outputs k = (n 2^40 + i_a I_b + i_b) 64 + 2q + h
 *          (h = 0, 1) of the given seed by the Box-Muller transform
 *          (u1 = 1 - k0/2^64 in 53 bits, u2 = k1/2^64 in 53 bits, entries
 *          2q, 2q+1 = sqrt(-2 ln u1) (cos, sin)(2 pi u2));
 *   F_i  = S_i / rho_i, rho_i = ||S_i||;
 *   R_i  = rho_i (W2^T relu(W1^T F_i + b1) + b2), weights rounded to BF16,
 *          FP32 accumulation;
 *   start factor = the leading Jn-dimensional subspace of H_n = X_(n) X_(n)^T
 *          within span(R[:, :K]), K = tucker_learn_test_width(Jn) = min(128,
 *          2 Jn) (Rayleigh-Ritz on an orthonormal basis of that span); the
 *          start is rejected (HO-SVD instead) when R[:, :K] is numerically
 *          rank-deficient or the start captures no more of ||X||^2 than
 *          Jn/In of it.
 * Parameters (FP32, this order, row-major): W1 64 x 128, b1 128,
 * W2 128 x 128, b2 128.
 */
#ifndef TUCKER_LEARN_H
#define TUCKER_LEARN_H

#include <stddef.h>
#include <stdint.h>

#include "tucker.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 network parameters (24,832). */
int tucker_learn_param_count(void);

/* Workspace bytes of tucker_learn_sketch for this tensor (TK_ERR_ARG on a
   bad tensor description). */
int tucker_learn_sketch_workspace(const tk_coo *X, size_t *bytes);

/* Features of mode `mode` (0..2): F [dev] In x 64 floats (rows of the sketch
   divided by their norms, zero rows stay zero) and rho [dev] In floats (the
   norms). Duplicates are summed first. Returns TK_OK, TK_ERR_ARG,
   TK_ERR_INDEX, TK_ERR_VALUE, TK_ERR_EMPTY, TK_ERR_WORKSPACE or
   TK_ERR_DEVICE. */
int tucker_learn_sketch(const tk_coo *X, int32_t mode, uint64_t seed, float *F, float *rho,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Network output R [dev] rows x 128 floats for features F [dev] rows x 64 and
   norms rho [dev] rows; Z1 [dev] rows x 128 floats receives the hidden
   pre-activations for the backward pass (NULL to skip). params [dev]. */
int tucker_learn_forward(const float *F, const float *rho, int64_t rows, const float *params, float *R,
                         float *Z1, void *stream);

/* Workspace bytes of tucker_learn_backward for `rows` rows. */
int tucker_learn_backward_workspace(int64_t rows, size_t *bytes);

/* grad [dev] param_count floats = gradient of a scalar with respect to the
   parameters, given dR [dev] rows x 128 (its gradient with respect to R) and
   the forward pass's Z1. Deterministic (fixed-order sums). */
int tucker_learn_backward(const float *F, const float *rho, int64_t rows, const float *params, const float *Z1,
                          const float *dR, float *grad, void *workspace, size_t workspace_bytes, void *stream);

/* K = min(128, 2J): the number of network outputs that span the test
   subspace of a rank-J start (TK_ERR_ARG unless 1 <= J <= 128). */
int tucker_learn_test_width(int32_t J);

/* Workspace bytes of tucker_learn_align for rows x K outputs and J targets. */
int tucker_learn_align_workspace(int64_t rows, int32_t K, int32_t J, size_t *bytes);

/* Subspace-alignment loss: how much of span(A) lies outside span(Rk), Rk the
   first K columns of R [dev] rows x 128 floats, A [dev] rows x J doubles with
   orthonormal columns: L = 1 - tr(B^T C^-1 B)/J with
   C = Rk^T Rk + shift tr(Rk^T Rk) I, B = Rk^T A, in FP64; *loss [host].
   dR [dev] rows x 128 floats receives dL/dR (the ridge held fixed; zero in
   columns >= K), or NULL for the loss alone. 1 <= K, J <= 128, J <= rows. */
int tucker_learn_align(const float *R, int64_t rows, int32_t K, const double *A, int32_t J, double shift,
                       double *loss, float *dR, void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (Kingma and Ba, 2015) on n FP32 parameters with first and
   second moments m, v [dev] (zero before step 1); step >= 1. */
int tucker_learn_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                      float beta2, float eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_LEARN_H */
