/*
 * tucker_steps.h -- step-level entry points of the sparse Tucker library, so
 * that each step of the HOOI / Multislice Projection path can be checked on
 * its own. Conventions ([dev], [host], ownership, workspace, stream, status
 * codes) are those of tucker.h.
 */
#ifndef TUCKER_STEPS_H
#define TUCKER_STEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes for tucker_step_lead_eig (TK_ERR_ARG if n < 1, J < 1,
   J > n or J > 128). */
int tucker_step_lead_eig_workspace(int32_t n, int32_t J, size_t *bytes);

/* "J leading eigenvectors" of a symmetric positive semi-definite matrix
   (every algorithm figure of Section 4; for SP and MP the figures name
   M M^T, whose leading eigenvectors are those of M).
     M        [dev]  n x n doubles, row-major, symmetric; not modified
     F        [dev]  n x J doubles (output), orthonormal columns in
                     descending eigenvalue order, largest-magnitude entry of
                     each column positive
     theta    [dev]  J doubles (output): the eigenvalues (Ritz values)
     matvecs  [host] output: products with M used (1 for the direct solver)
     tol      relative accuracy of the sum of the J leading Ritz values at
              which the iteration stops: the residual estimate
              sum_j r_j^2 / (theta_j - theta_{J+1}) (theta_{J+1}: the first
              Ritz value outside the J leading ones), or the
              change of the sum across a full-degree filter step, at most
              tol times the sum (used for n > 140; smaller matrices are
              diagonalised directly)
     warm     nonzero: start from the block that the previous call with the
              same n, J and workspace left in the workspace (as the sweeps
              of HOOI and MP do); zero: pseudo-random start
   Returns TK_OK, TK_WARN_NOCONV (cap of 400 products reached; outputs
   valid), TK_ERR_ARG, TK_ERR_WORKSPACE or TK_ERR_DEVICE. */
int tucker_step_lead_eig(const double *M, int32_t n, int32_t J, double *F, double *theta, int32_t *matvecs,
                         double tol, int32_t warm, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_STEPS_H */
