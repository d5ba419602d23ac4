/*
 * tucker.h -- C ABI of a GPU (gfx950) library for Tucker decompositions of
 * sparse third-order tensors by HOOI and Multislice Projection (MP).
 *
 * Problem (Turney 2007, Section 4, opening paragraph): given a tensor X of
 * size I1 x I2 x I3 and a core size J1 x J2 x J3, find a core G and factor
 * matrices A(n) of size In x Jn with orthonormal columns such that
 * X ~ [[G; A(1), A(2), A(3)]] (Tucker operator, Section 3). The input is a
 * list of nonzeros <i, j, k, x> (Section 4.3, slice construction).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * [dev]  = device pointer (memory of the current HIP device, allocated by the
 *          caller); [host] = host pointer.
 * Ownership: the caller owns every buffer. The library keeps no state
 *          between calls and allocates no device memory: all scratch space
 *          is carved from the caller's `workspace`, whose size is returned by
 *          tucker_workspace_bytes(). Calls with distinct workspaces and
 *          streams may run concurrently.
 * Stream:  `stream` is a hipStream_t passed as void* (NULL = the null
 *          stream). Work is enqueued on it; every entry point returns after
 *          its results are complete and visible to the host (the sweep loops
 *          read one fit value per sweep back to the host). With an HO-SVD or
 *          learned start, the start of mode 3 runs on a second stream that
 *          the call creates (default priority) and drives from a second host
 *          thread, beside mode 2's on `stream`; `stream` waits for it, and
 *          the stream is destroyed, before the sweeps begin.
 * Indices: 0-based int32 coordinates, structure of arrays: idx[n][p] is the
 *          mode-n coordinate of nonzero p. Duplicate coordinates are summed;
 *          explicit zeros are allowed.
 * Layouts: factor n is In x Jn row-major (row i contiguous). Columns are in
 *          descending order of the eigenvalue they belong to, and each
 *          column's largest-magnitude entry is positive. The core is
 *          J1 x J2 x J3 row-major: G[p][q][r] at (p*J2 + q)*J3 + r.
 * Errors:  every entry point returns a status code (TK_OK = 0, warnings > 0,
 *          errors < 0). TK_ERR_ARG is detected on the host before any device
 *          work is enqueued, and then no output is written. TK_ERR_INDEX and
 *          TK_ERR_VALUE are detected by the first kernels, before any output
 *          is written. tucker_strerror() gives a text.
 * Limits:  besides the conditions of the problem (Jn <= In), the library
 *          rejects with TK_ERR_ARG, before any device work:
 *          - Jn > 128 (the eigensolver keeps its Rayleigh-Ritz matrix of
 *            Jn + max(6, Jn/8) columns in one workgroup's LDS);
 *          - nnz >= 2^31 - 1, or any In >= 2^31 (32-bit coordinates);
 *          - I_a * I_b >= 2^31 for any pair of modes (the fibres of the third
 *            mode are the slots of a dense, 32-bit indexed layout);
 *          - with an HO-SVD start (TK_INIT_HOSVD, also as the fallback of
 *            TK_INIT_LEARNED, and opts.hosvd_fit), In > 8192 for a mode that
 *            needs its start Gram X_(n) X_(n)^T (modes 2 and 3; all three for
 *            tucker_hosvd and opts.hosvd_fit): one Gram row is kept in a
 *            workgroup's LDS. TK_INIT_GIVEN and TK_INIT_RANDOM have no such
 *            limit.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define TK_OK              0
#define TK_WARN_NOCONV     1  /* an eigensolve hit its iteration cap; outputs are valid */
#define TK_ERR_ARG        -1  /* null pointer, order != 3, nnz < 0 or >= 2^31, In < 1,
                                 Jn < 1 or Jn > In, max_iters < 0, bad precision/init,
                                 a launch choice out of its range */
#define TK_ERR_INDEX      -2  /* a coordinate outside [0, In) */
#define TK_ERR_VALUE      -3  /* a NaN or infinite value */
#define TK_ERR_EMPTY      -4  /* ||X|| = 0: the fit is undefined */
#define TK_ERR_WORKSPACE  -5  /* workspace NULL or smaller than tucker_workspace_bytes() */
#define TK_ERR_DEVICE     -6  /* a HIP call failed; tucker_strerror() has the HIP text */
#define TK_ERR_SIZE       -7  /* tucker_fit_static: the problem needs more scratch than
                                 TK_STATIC_SCRATCH_BYTES */

/* ---- precision of the projection / Gram / TTMc path ------------------- */
#define TK_FP64        0  /* FP64 everywhere */
#define TK_FP32        1  /* FP32 projections, FP32 MFMA Grams; eigensolve, core, fit FP64 */
#define TK_MIXED_BF16  2  /* BF16 projections for the Grams (MP: FP32 sums of FP16
                             factor rows), BF16 MFMA with FP32 accumulation;
                             eigensolve, core and fit FP64 */
#define TK_MIXED_BF16X3 3 /* MP only: each projection for the Grams as a BF16 pair
                             (rounded value + rounded remainder, from FP32 factors),
                             Grams as hi hi^T + hi lo^T + lo hi^T on BF16 MFMA with
                             FP32 accumulation (about FP32 accuracy, three times the
                             MFMA work of TK_MIXED_BF16); TK_ERR_ARG for HOOI */

/* ---- initialisation --------------------------------------------------- */
#define TK_INIT_HOSVD  0  /* B, C from the leading eigenvectors of X_(n) X_(n)^T */
#define TK_INIT_GIVEN  1  /* B, C read from factors[1], factors[2] (resume) */
#define TK_INIT_LEARNED 2 /* B, C from the learned start of tucker_learn.h (opts.model,
                             opts.seed); a mode whose start is rank-deficient or
                             captures no more of ||X||^2 than a random subspace
                             would on average (Jn/In of it) falls back to HO-SVD */
#define TK_INIT_RANDOM  3 /* Slice Projection's start (Section 4.3, Figure 5): a
                             random matrix with entries uniform on [0, 1) and
                             columns normalised to unit length, for C (SP) or B
                             and C (HOOI, MP). Entry (i, r) of mode n (0-based n)
                             is the top 53 bits, scaled by 2^-53, of output number
                             n * 2^40 + i * Jn + r of SplitMix64 (Steele, Lea and
                             Flood, OOPSLA 2014) seeded with opts.seed. */

/* ---- algorithm selector of the workspace query ------------------------ */
#define TK_ALGO_HOOI   0
#define TK_ALGO_MP     1
#define TK_ALGO_FIT    2
#define TK_ALGO_SP     3
#define TK_ALGO_HOSVD  4

/* Sparse tensor in coordinate form: third order everywhere; fourth order
   for tucker_hooi, tucker_mp, tucker_hosvd and their workspace query
   (TK_ERR_ARG elsewhere). */
#define TK_MAX_ORDER 4
typedef struct tk_coo {
    int32_t        order;   /* 3, or 4 (see above) */
    int64_t        nnz;     /* number of listed entries, 0 <= nnz < 2^31 */
    const int64_t *dims;    /* [host] order entries: I1, ..., IN (each >= 1, < 2^31) */
    const int32_t *idx[TK_MAX_ORDER];  /* [dev] nnz coordinates per mode, 0-based; the
                                          first `order` are read */
    const double  *vals;    /* [dev] nnz values */
} tk_coo;

/* Per-launch trace (opts.trace): one event per timed kernel or phase of the
   sweeps, measured with HIP events on the call's stream. */
#define TK_PHASE_PROJECT 0  /* a projection T(m) = X x_m A(m)^T (one kernel) */
#define TK_PHASE_TTMC2   1  /* a HOOI second-stage product Y = T x_o A(o)^T */
#define TK_PHASE_GRAM    2  /* a Gram (SYRK kernel and its FP64 partial-sum pass) */
#define TK_PHASE_EIG     3  /* one leading-eigenvector solve (with its host round trips) */
#define TK_PHASE_CORE    4  /* the core contractions of a sweep */
typedef struct tk_event {
    int32_t phase;      /* TK_PHASE_* */
    int32_t mode;       /* 0-based: the leaf mode m of a projection T(m), the mode
                           n a Gram or eigensolve serves, the mode of the Gram a
                           second-stage product feeds; -1 for the core */
    int32_t precision;  /* element type of the output (projection) or of the
                           operands (products, Grams): TK_FP64, TK_FP32,
                           TK_MIXED_BF16; the eigensolve is always TK_FP64 */
    int32_t sweep;      /* 1-based sweep it belongs to */
    double  ms;         /* duration in milliseconds */
} tk_event;
typedef struct tk_trace {
    tk_event *events;   /* [host] room for `capacity` events, filled in launch order */
    int32_t   capacity;
    int32_t   count;    /* out: events written; the caller sets it to 0 first */
    int64_t   dropped;  /* out: events that did not fit; the caller sets it to 0 first */
} tk_trace;

/* Launch choices: 0 in a field = the built-in choice. The projection's
   choices change no result bit (each output sums its nonzeros in the same
   order whatever the run length). The Gram's choices set its split over the
   summed dimension: results stay deterministic for a given choice but the
   FP32 partial sums (BF16/FP32 Grams) round differently, within the same
   bound. A tuner (paper_0711_2023_amd.autotune) measures them per tensor
   shape and caches them as JSON. */
typedef struct tk_tune {
    int32_t proj_elems;       /* output elements per projection workgroup, at most
                                 (1024 .. 65536; built-in 32768) */
    int32_t proj_min_blocks;  /* projection workgroups wanted before runs of slots
                                 grow (64 .. 16384; built-in 1536) */
    int32_t gram_items;       /* Gram workgroups (tile pairs x K splits) wanted
                                 (64 .. 16384; built-in 1024) */
    int32_t gram_min_stages;  /* K stages per Gram workgroup, at least (1 .. 64;
                                 built-in 4) */
} tk_tune;

/* Options; tucker_default_opts() fills the paper's values. */
typedef struct tk_opts {
    int32_t precision;      /* TK_FP64 | TK_FP32 | TK_MIXED_BF16 | TK_MIXED_BF16X3 */
    int32_t init;           /* TK_INIT_HOSVD | TK_INIT_GIVEN | TK_INIT_LEARNED */
    int32_t max_iters;      /* sweep cap; the paper uses 50 */
    double  tol;            /* stop after sweep t when fit(t) - fit(t-1) < tol,
                               with fit(0) = 0 (paper: 1e-4); tol <= 0 runs
                               exactly max_iters sweeps */
    int32_t eig_max_iters;  /* cap on filtered subspace iterations per eigensolve */
    double  eig_tol;        /* relative accuracy of the sum of the J leading Ritz values
                               at which an eigensolve stops (residual estimate, or
                               change across a full-degree filter step); 0 = by
                               precision (1e-12 for FP64, 1e-8 for FP32 and split
                               BF16, 1e-4 for mixed BF16: a tenth of the relative
                               accuracy of the Gram at that precision) */
    int32_t timing;         /* 1: record HIP events around the kernels and phases of
                               the sweeps and report their sums in tk_stats */
    const float *model;     /* [dev] TK_INIT_LEARNED: the network parameters
                               (tucker_learn_param_count() floats, layout in
                               tucker_learn.h); NULL otherwise */
    uint64_t seed;          /* TK_INIT_LEARNED: seed of the sketch generator;
                               TK_INIT_RANDOM: seed of the start */
    const tk_tune *tune;    /* [host] launch choices, or NULL for the built-in ones */
    int32_t hosvd_fit;      /* 1: HOOI, MP and SP also compute the fit of the HO-SVD
                               (Figure 1: all three factors from X_(n) X_(n)^T, then
                               the core) before the sweeps and report it in
                               stats.hosvd_fit; costs the mode-1 start Gram and
                               eigensolve (and modes 2, 3 for SP or a non-HO-SVD
                               start), one FP64 projection and the core. The
                               decomposition itself is unchanged. Only with
                               TK_INIT_HOSVD or TK_INIT_RANDOM (TK_ERR_ARG
                               otherwise): the report uses the factor buffers
                               as scratch before the sweeps. */
    tk_trace *trace;        /* [host] per-launch trace of the sweeps, or NULL; a
                               trace implies timing = 1 */
} tk_opts;

/* Optional statistics (pass NULL to skip). Times in milliseconds. */
typedef struct tk_stats {
    double  prep_ms;        /* validation, duplicate summing, three orderings, ||X||^2 */
    double  init_ms;        /* initial Grams and eigensolves */
    double  sweeps_ms;      /* all sweeps, including the per-sweep fit read-back */
    /* With opts.timing = 1, HIP events recorded on `stream` around each
       phase of the sweeps give these sums (milliseconds over all sweeps): */
    double  ttmc_ms;        /* projections + HOOI second-stage GEMMs (the TTMc phase) */
    double  project_ms;     /* projection kernels alone */
    int64_t project_calls;  /* number of projection launches in the sweeps */
    double  gram_ms;        /* Gram (SYRK) kernels, including their FP64 partial-sum pass */
    int64_t gram_calls;
    double  eig_ms;         /* leading-eigenvector solves (including their host round trips) */
    double  core_ms;        /* core contractions */
    int64_t nnz_unique;     /* nonzeros after duplicate summing */
    int32_t eig_iters;      /* total filtered subspace iterations */
    int32_t eig_noconv;     /* eigensolves that hit eig_max_iters */
    double  norm_x;         /* ||X||_F */
    int32_t init_fallbacks; /* TK_INIT_LEARNED: modes that fell back to HO-SVD */
    double  hosvd_fit;      /* opts.hosvd_fit = 1 (and tucker_hosvd): the HO-SVD fit;
                               otherwise 0 */
    double  core_norm;      /* ||G||_F of the returned core */
    double  ttmc_sweep_ms[64]; /* opts.timing = 1: the TTMc phase's time in sweep t
                               (t < 64; its share of ttmc_ms), 0 beyond */
    int64_t streamed_bytes; /* tucker_mp_streamed: bytes uploaded from host memory */
    int64_t streamed_slabs; /* tucker_mp_streamed: slabs uploaded */
    int64_t product_fibres; /* tucker_mp_implicit: sum over its product kernel launches of the
                               fibres each launch visits (each reads its row twice) */
    int64_t product_pairs;  /* tucker_mp_implicit: sum over the same launches of fibres x
                               columns (one gathered Q element and one written row element
                               per pair, 4 J flops) */
} tk_stats;

/* Fill *opt with: FP32, HO-SVD init, 50 sweeps, tol 1e-4, eig cap 400
   products, eig tol 0 (by precision), no timing, no model, seed 0x5eed,
   built-in launch choices, no HO-SVD fit, no trace. */
void tucker_default_opts(tk_opts *opt);

/* Bytes of device workspace that tucker_hooi (algo TK_ALGO_HOOI),
   tucker_mp (TK_ALGO_MP), tucker_sp (TK_ALGO_SP), tucker_hosvd
   (TK_ALGO_HOSVD) or tucker_fit (TK_ALGO_FIT) needs for this tensor shape,
   nnz, core size and options. Host only; enqueues nothing. Returns TK_OK
   and writes *bytes, or TK_ERR_ARG. */
int tucker_workspace_bytes(int32_t algo, const tk_coo *X, const int32_t *core_dims,
                           const tk_opts *opt, size_t *bytes);

/* HOOI (Section 4.2, Figure 3): B and C from the HO-SVD Grams X_(n)X_(n)^T
   (mode 1 needs no start), then per sweep A, B, C in turn from the leading
   eigenvectors of Z_(n) Z_(n)^T with Z = X projected on the two other
   factors; core G = [[X; A^T, B^T, C^T]] and the fit after every sweep.
     core_dims   [host] J1, J2, J3
     core        [dev]  J1*J2*J3 doubles (output)
     factors     [host] array of 3 [dev] pointers to In x Jn doubles (output;
                 with TK_INIT_GIVEN factors[1] and factors[2] are also read)
     fit_history [host] max_iters doubles; entry t-1 = fit after sweep t
     iters_done  [host] number of sweeps run
     stats       [host] optional, may be NULL                                */
int tucker_hooi(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                double *core, double *const *factors, double *fit_history,
                int32_t *iters_done, tk_stats *stats,
                void *workspace, size_t workspace_bytes, void *stream);

/* Multislice Projection (Section 4.4, Figure 7): pseudo HO-SVD start of B
   and C, then per sweep
     M1 = sum_k X_::k B B^T X_::k^T + sum_j X_:j: C C^T X_:j:^T  -> A
     M2 = sum_k X_::k^T A A^T X_::k + sum_i X_i:: C C^T X_i::^T  -> B
     M3 = sum_j X_:j:^T A A^T X_:j: + sum_i X_i::^T B B^T X_i::  -> C
   (leading eigenvectors), the core and the fit. Arguments as tucker_hooi. */
int tucker_mp(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
              double *core, double *const *factors, double *fit_history,
              int32_t *iters_done, tk_stats *stats,
              void *workspace, size_t workspace_bytes, void *stream);

/* Slice Projection (Section 4.3, Figure 5): C from the start (TK_INIT_RANDOM,
   the paper's; TK_INIT_GIVEN reads factors[2]; TK_INIT_HOSVD; columns are
   normalised to unit length either way), then per sweep
     M13 = sum_j X_:j: C C^T X_:j:^T -> A
     M21 = sum_k X_::k^T A A^T X_::k -> B
     M32 = sum_i X_i::^T B B^T X_i:: -> C
   (leading eigenvectors; each Gram uses one other factor), the core and
   Delta_G(t) = 1 - ||G(t-1)|| / ||G(t)|| with ||G(0)|| = 0: stop after sweep
   t when Delta_G(t) < tol (tol <= 0: exactly max_iters sweeps).
   fit_history holds the fit after every sweep (as for HOOI and MP).
   TK_INIT_LEARNED is rejected (TK_ERR_ARG). Arguments as tucker_hooi. */
int tucker_sp(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
              double *core, double *const *factors, double *fit_history,
              int32_t *iters_done, tk_stats *stats,
              void *workspace, size_t workspace_bytes, void *stream);

/* HO-SVD (Section 4.1, Figure 1): A(n) = Jn leading eigenvectors of
   X_(n) X_(n)^T for n = 1, 2, 3 (FP64 Grams; the eigensolver's tolerance
   follows opt->precision as for the other algorithms), then
   G = [[X; A^T, B^T, C^T]] from an FP64 projection and the fit.
   opt->init, max_iters and tol are not used.
     core    [dev]  J1*J2*J3 doubles (output)
     factors [host] array of 3 [dev] pointers to In x Jn doubles (output)
     fit     [host] output
     stats   [host] optional                                                 */
int tucker_hosvd(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                 double *core, double *const *factors, double *fit, tk_stats *stats,
                 void *workspace, size_t workspace_bytes, void *stream);

/* fit(X, Xhat) = 1 - ||X - Xhat||_F / ||X||_F (Section 3, fit equation) of
   Xhat = [[G; A(1), A(2), A(3)]] for ANY core and factors (orthonormality
   is not assumed): ||X - Xhat||^2 = ||X||^2 - 2<X, Xhat> + ||Xhat||^2 with
   <X, Xhat> = <X x_n A(n)^T, G> and ||Xhat||^2 = <G, G x_n A(n)^T A(n)>,
   all in FP64.
     core    [dev]  J1*J2*J3 doubles, row-major
     factors [host] array of 3 [dev] pointers, In x Jn row-major doubles
     fit     [host] output                                                   */
int tucker_fit(const tk_coo *X, const int32_t *core_dims, const double *core,
               const double *const *factors, double *fit,
               void *workspace, size_t workspace_bytes, void *stream);

/* The fit of tucker_fit for callers that cannot allocate device memory
   (code under stream capture, serving loops that must not call the
   allocator): the same arguments and result, without a workspace. Its scratch
   space is a static device array of TK_STATIC_SCRATCH_BYTES (64 MiB) inside
   the library, of which every device the library runs on holds one copy from
   the library's load until the process ends. The first call on a device,
   with that device current, looks up the array's device address once
   (hipGetSymbolAddress); no call allocates or frees device memory.
   Limit: TK_ERR_SIZE, before any device work, when the problem needs more
   than TK_STATIC_SCRATCH_BYTES, i.e. when tucker_workspace_bytes(TK_ALGO_FIT,
   ...) exceeds it (about 72 bytes per nonzero, 4 bytes per fibre slot of each
   mode (I2*I3 + I3*I1 + I1*I2 slots) plus 8 per slot of the largest family,
   8*J3 bytes per mode-3 fibre slot (I1*I2 of them, the FP64 projection), and
   terms of the core's size). Other errors as tucker_fit.
   Every call on one device shares that device's array: calls that overlap on
   one device (from several host threads, or on several streams without
   ordering between them) race and give wrong results; calls in sequence on
   one stream, or on streams the caller orders, are safe. The call returns
   after the fit has been read back (host-blocking, as tucker_fit).
     core    [dev]  J1*J2*J3 doubles, row-major
     factors [host] array of 3 [dev] pointers, In x Jn row-major doubles
     fit     [host] output
     stream  hipStream_t as void* (NULL = the null stream) of the current
             device                                                        */
#define TK_STATIC_SCRATCH_BYTES (64u << 20)
int tucker_fit_static(const tk_coo *X, const int32_t *core_dims, const double *core,
                      const double *const *factors, double *fit, void *stream);

/* Static text for a status code (for TK_ERR_DEVICE, the last HIP error text
   seen by the calling thread). */
const char *tucker_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_H */
