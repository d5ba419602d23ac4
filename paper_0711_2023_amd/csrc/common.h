// Internal declarations shared by the HIP sources of the sparse Tucker library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct tk_coo;
struct tk_opts;
struct tk_stats;

namespace tk {

typedef __bf16 bf16;
typedef _Float16 f16;
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum Prec { P64 = 0, P32 = 1, PBF16 = 2 };

// Raise kernel fn's dynamic LDS limit to at least `bytes` (one runtime call
// the first time a kernel needs more than it was given before; thread safe).
void lds_limit(const void *fn, size_t bytes);

// Records the first failing HIP call of the current thread; returned as text
// by tucker_strerror(TK_ERR_DEVICE).
void set_hip_error(hipError_t e, const char *where);
// Forget the calling thread's recorded HIP error (at the start of a call).
void g_err_clear();

#define TK_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) {                        \
            ::tk::set_hip_error(e_, #call);            \
            return e_;                                 \
        }                                              \
    } while (0)

#define TK_LAUNCHED()                                  \
    do {                                               \
        hipError_t e_ = hipGetLastError();             \
        if (e_ != hipSuccess) {                        \
            ::tk::set_hip_error(e_, __func__);         \
            return e_;                                 \
        }                                              \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace. With base == nullptr it only
// counts bytes (used by the size query and by the carve-out, so both agree).
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    template <class T>
    T *take(int64_t count) {
        size_t off = align_up(used, 256);
        used = off + sizeof(T) * (size_t)(count > 0 ? count : 1);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

// ---------------------------------------------------------------- prep.hip
// Exclusive scan of n int32 counts into out[0..n]; out[n] = total.
// scratch: at least scan_scratch_ints(n) ints.
int64_t scan_scratch_ints(int64_t n);
hipError_t scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s);

hipError_t fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t fill_f64(double *p, int64_t n, double v, hipStream_t s);

// One ordering of the nonzeros: slots are the mode-m fibres (i_hi, i_lo)
// with hi = (m+2)%3, lo = (m+1)%3, slot = i_hi*I_lo + i_lo; within a slot the
// entries are sorted by (i_m, input position). perm[q] = input position of
// the q-th sorted entry. Needs slot_count(m)+1 ints in ptr and the scratch
// buffers described at the definition.
struct OrderScratch {
    int32_t *counts;   // nslots
    int32_t *cursor;   // nslots
    int32_t *tmp;      // nnz
    int32_t *scan;     // scan_scratch_ints(nslots)
};
// Positions are range-checked (guards.h): a failed check sets
// kFlagOrderCheck in *flags and leaves perm unwritten.
hipError_t build_order(const int32_t *const idx[3], int64_t nnz, const int64_t dims[3], int m,
                       int32_t *ptr, int32_t *perm, OrderScratch sc, int32_t *flags, hipStream_t s);

// The non-empty fibres of an ordering with slot pointers ptr[0..nslots]:
// fib[f] = slot of the f-th non-empty fibre (ascending), fptr[f] = its first
// entry, fptr[F] = ptr[nslots], where F = pos_tmp[nslots] (device) is their
// number. fib has room for cap entries, fptr for cap + 1; a count beyond cap
// sets kFlagOrderCheck in *flags and writes nothing out of range.
// flag_tmp: nslots ints; pos_tmp: nslots + 1 ints; scan_scratch as scan.
hipError_t fibre_list(const int32_t *ptr, int64_t nslots, int64_t cap, int32_t *fib, int32_t *fptr, int32_t *flag_tmp,
                      int32_t *pos_tmp, int32_t *scan_scratch, int32_t *flags, hipStream_t s);

// The fibres of a fibre list (fptr[0..n]) with more than maxlen nonzeros:
// lf[k] = index of the k-th of them (ascending), their number at
// pos_tmp[n] (device). lf has room for cap entries; a count beyond cap sets
// kFlagOrderCheck in *flags and writes nothing out of range.
// flag_tmp: n ints; pos_tmp: n + 1 ints; scan_scratch as scan.
hipError_t long_fibres(const int32_t *fptr, int64_t n, int32_t maxlen, int64_t cap, int32_t *lf, int32_t *flag_tmp,
                       int32_t *pos_tmp, int32_t *scan_scratch, int32_t *flags, hipStream_t s);

// The counting sort of build_order on explicit key digits: slot =
// ihi[p] * Ilo + ilo[p] (nslots of them), within a slot by (im[p], p).
hipError_t build_order_keys(const int32_t *ihi, const int32_t *ilo, const int32_t *im, int64_t nnz, int32_t Ilo,
                            int64_t nslots, int32_t *ptr, int32_t *perm, OrderScratch sc, int32_t *flags,
                            hipStream_t s);

// ---- tensors of order N (at most 4 modes)
constexpr int kMaxOrder = 4;
struct CoordsN {
    const int32_t *i[kMaxOrder];
    int32_t dim[kMaxOrder];
    int n;
};
struct CoordsOut {
    int32_t *i[kMaxOrder];
};
// out[p] = a[p] * Ib + b[p] (two coordinates merged into one key digit).
hipError_t merge_keys(const int32_t *a, const int32_t *b, int64_t nnz, int32_t Ib, int32_t *out, hipStream_t s);
// flags |= 1 (a coordinate outside its mode), 2 (a non-finite value).
hipError_t validate_n(CoordsN c, const double *vals, int64_t nnz, int32_t *flags, hipStream_t s);
// Duplicate summing over an ordering whose sort key is the full coordinate
// (perm), as dedup.
hipError_t dedup_n(CoordsN c, const double *vals, int64_t nnz, const int32_t *perm, int32_t *heads, int32_t *pos,
                   int32_t *scan_scratch, CoordsOut out, double *cval, int32_t *nu_dev, hipStream_t s);

// Validation: flags |= 1 (index out of range), 2 (non-finite value).
hipError_t validate(const int32_t *const idx[3], const double *vals, int64_t nnz, const int64_t dims[3],
                    int32_t *flags, hipStream_t s);

// Duplicate summing over a leaf-2 ordering. heads/scan scratch of nnz+1 ints.
// Writes unique coordinates cidx[3][u] and values cval[u] in sorted order and
// u to *nu_dev.
hipError_t dedup(const int32_t *const idx[3], const double *vals, int64_t nnz, const int32_t *perm,
                 int32_t *heads, int32_t *pos, int32_t *scan_scratch, int32_t *const cidx[3], double *cval,
                 int32_t *nu_dev, hipStream_t s);

// Gather the leaf index and value of an ordering: lidx[q] = idx_m[perm[q]],
// lval[q] = (T)vals[perm[q]]; nothing when *flags has kFlagOrderCheck.
template <class T>
hipError_t gather_leaf(const int32_t *idx_m, const double *vals, const int32_t *perm, int64_t n, int32_t *lidx,
                       T *lval, const int32_t *flags, hipStream_t s);

// Deterministic sum of squares (FP64) into *out.
hipError_t sumsq(const double *v, int64_t n, double *partials, double *out, hipStream_t s);
constexpr int kReduceBlocks = 512;

// Unfolding Gram H_n = X_(n) X_(n)^T (FP64, In x In, full). Uses the leaf-n
// ordering (fibres) and the leaf-(n+1) ordering (slices of mode n).
hipError_t hosvd_gram(int n, const int64_t dims[3], const int32_t *ptr_n, const int32_t *lidx_n,
                      const double *lval_n, const int32_t *ptr_s, const int32_t *lidx_s, const double *lval_s,
                      double *H, hipStream_t s);
// The same with explicit sizes, for any order: In = I_n rows; the slice of
// row i is slots [i * In2, (i + 1) * In2) of ordering s (leaf index i_{n+1});
// the entry at sub-slot j with leaf index k lies on fibre j * In1 + k of
// ordering n (In1 = I_{n+1}).
hipError_t hosvd_gram_sized(int32_t In, int32_t In1, int32_t In2, const int32_t *ptr_n, const int32_t *lidx_n,
                            const double *lval_n, const int32_t *ptr_s, const int32_t *lidx_s, const double *lval_s,
                            double *H, hipStream_t s);

// Launch choices that do not change results (run lengths of the projection,
// split-K items of the Gram); the defaults are the built-in ones, a tuned
// table can replace them per tensor shape.
struct Tune {
    int proj_elems = 32768;     // output elements per projection workgroup, at most
    int proj_min_blocks = 1536; // projection workgroups wanted before runs grow
    int gram_items = 1024;      // Gram workgroups (tile pairs x K splits) wanted
    int gram_min_stages = 4;    // K stages per Gram workgroup, at least
};

// Events a kernel launch records itself at the kernel's start and end (both
// null: an ordinary launch).
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// ---------------------------------------------------------------- project.hip
// The non-empty fibres of an ordering (fibre_list): n fibres, fib[f] their
// slots, fptr[f] their first entries. Empty (fib == nullptr) = not given.
// Long fibres (more than maxlen nonzeros) listed in lf (nlong of them, as
// indices into the list) are skipped by the per-thread walk of the vector
// projection and projected by one workgroup each; the same for long slots
// (ls) when a projection writes every slot.
struct FibreList {
    const int32_t *fib = nullptr, *fptr = nullptr;
    int64_t n = 0;
    const int32_t *lf = nullptr;
    int64_t nlong = 0;
    int32_t maxlen = 0x7fffffff;
    // Projections that write every slot (no list): the slots with more than
    // slot_maxlen nonzeros (ls, nls of them), projected by one workgroup each.
    const int32_t *ls = nullptr;
    int64_t nls = 0;
    int32_t slot_maxlen = 0x7fffffff;
};
// Fibres with more nonzeros than a limit go to the one-workgroup-per-fibre
// projection (one thread walking them would hold its workgroup back). The
// limit depends on the output row: BF16 rows (8 chunks of 16 bytes at J = 50,
// so 32 nonzero groups per long-fibre workgroup) keep fibres up to 12 in the
// per-thread walk, FP32 and FP64 rows (13 or 25 chunks, fewer groups) up to
// 8. On a Zipf-skewed 1000^3 tensor with 1M nonzeros, BF16 projections took
// 54, 45, 40 and 42 us at limits 8, 10, 12 and 16 (50 us at 24), FP32 ones
// 40, 48-51 and 55-57 us at 8, 12 and 16; uniform tensors were unchanged at
// every limit.
constexpr int32_t kLongFibreBf16 = 12;
constexpr int32_t kLongFibreWide = 8;
// T[slot * ldT + r] = sum over the slot's entries of lval * F[lidx * ldF + r]
// for r < J, zero for J <= r < ldT; slots = I_hi * I_lo, dense and
// zero-filled; F has rowsF rows (the leaf mode's size) and the ordering at
// most nnz nonzeros. With ldF == ldT,
// 16-byte rows and F's padding columns zero (as pad_rows leaves them), whole
// 16-byte chunks are computed at once. With a fibre list as well (and the
// whole output below 2 GiB), only the rows of non-empty fibres are written:
// the rows of empty fibres must hold zeros already (the caller zeroes the
// buffer once before the first such projection into it); the values written
// are bitwise those of the dense form.
template <class TV, class TF, class TO>
hipError_t project(const int32_t *ptr, const int32_t *lidx, const TV *lval, const TF *F, int64_t rowsF, int ldF,
                   int J, int ldT, int64_t nslots, int64_t nnz, TO *T, hipStream_t s, const Tune &tn = Tune(),
                   KernelEvents ke = KernelEvents(), FibreList fl = FibreList());
// Projection into a BF16 pair (hi = rounded value, lo = rounded remainder)
// from FP32 factor rows padded to ld (a multiple of 8), for split-BF16 Grams;
// a fibre list as for project.
hipError_t project_split(const int32_t *ptr, const int32_t *lidx, const float *lval, const float *F, int64_t rowsF,
                         int ld, int J, int64_t nslots, int64_t nnz, bf16 *Thi, bf16 *Tlo, hipStream_t s,
                         const Tune &tn = Tune(), KernelEvents ke = KernelEvents(), FibreList fl = FibreList());
// FP32 projection into T over the fibre list fl (rows of ld, a multiple of
// 4, as the factor rows F) that also writes each output rounded to BF16 into
// T2 (rows of ld2 = ld or ld + 4 + 8k, a multiple of 8; columns from ld on are
// written as zeros, the rows of empty fibres keep what T2 holds), in one pass
// over the nonzeros. Only where
// project_dual_ok holds (the fibre-list vector form with 32-bit offsets for
// both outputs); else hipErrorInvalidValue and nothing is launched.
bool project_dual_ok(const float *F, int64_t rowsF, int ld, const float *T, const bf16 *T2, int ld2,
                     int64_t nslots, int64_t nnz, const Tune &tn, const FibreList &fl);
hipError_t project_dual(const int32_t *ptr, const int32_t *lidx, const float *lval, const float *F, int64_t rowsF,
                        int ld, int J, int64_t nslots, int64_t nnz, float *T, bf16 *T2, int ld2, hipStream_t s,
                        const Tune &tn, KernelEvents ke, FibreList fl);
// out[i * ld + r] = in[i * J + r] for r < J, zero for J <= r < ld.
template <class TO>
hipError_t pad_rows(const double *in, int64_t rows, int J, int ld, TO *out, hipStream_t s);

// ---------------------------------------------------------------- mfma.hip
// One operand of a Gram: row i, column k = (kc, kr) with kr < chunk_len,
// element at base + i*s_row + kc*s_chunk + kr.
// A term may pair two operands of the same layout: base_b (NULL = base) holds
// the right-hand rows, for the cross products of split operands.
struct GramTerm {
    const void *base;
    int64_t s_row;
    int64_t s_chunk;
    int64_t chunk_len;
    int64_t nchunks;
    const void *base_b = nullptr;
};
constexpr int kGramMaxTerms = 6;
// M (FP64, n x n, symmetric, full) = sum over terms of T_t U_t^T (U_t = T_t
// unless base_b is set; the sum must be symmetric, as the lower triangle is
// computed and mirrored). At most kGramMaxTerms terms.
// Element type by precision: P64 double, P32 float, PBF16 bf16.
size_t gram_scratch_bytes(int n, int prec, int nterms, const int64_t *K, const Tune &tn = Tune());
hipError_t gram(int n, int prec, int nterms, const GramTerm *terms, double *M, void *scratch, hipStream_t s,
                const Tune &tn = Tune());

// General batched GEMM out[b][i][j] = alpha * sum_k A(i,k) B[b](k,j) (+ epilogue)
// A(i,k) = a_trans ? A[k*lda + i] : A[i*lda + k]; B[b](k,j) = B[b*sB + k*ldb + j].
struct GemmArgs {
    int M, N, K, batch;
    const void *A;  int64_t lda; bool a_trans;
    const void *B;  int64_t ldb, sB;
    void *C;        int64_t ldc, sC;
    int prec;       // element type of A and B (and MFMA kind)
    int out_type;   // element type of C: P64 double, P32 float, PBF16 bf16
    // epilogue (FP64 outputs only): C = alpha*acc + beta*E1 + gamma*E2
    double alpha = 1.0, beta = 0.0, gamma = 0.0;
    const double *E1 = nullptr, *E2 = nullptr;  // same layout as C
    int splitk = 1;                   // >1: partial sums to scratch, then reduced
    double *split_scratch = nullptr;  // splitk * batch * M * N doubles
};
hipError_t gemm(const GemmArgs &g, hipStream_t s);

// ---------------------------------------------------------------- eig.hip
struct EigWork;  // opaque, carved from the workspace
size_t eig_work_bytes(int n, int b);
int eig_block_width(int n, int J);
// Leading J eigenvectors of the symmetric PSD matrix M (FP64 n x n). M is
// overwritten (converged pairs are deflated out of it).
// X (n x b, b = eig_block_width) holds the start block on entry when warm,
// and the converged block on exit. F receives the J leading eigenvectors
// (n x J row-major, sign-canonical); theta (device, b) the Ritz values.
// Returns 0 or a hip error; *iters / *noconv report convergence.
// The matrix of a solve given as an operator instead of explicitly: apply
// writes Y (n x w, row stride ldy) = A X for X (n x w, row stride ldx), A
// symmetric PSD, on stream s. Solves with n <= 140 need A explicitly.
struct EigOp {
    hipError_t (*apply)(const void *ctx, const double *X, int64_t ldx, int w, double *Y, int64_t ldy, hipStream_t s);
    const void *ctx;
};
struct EigOpts {
    const EigOp *op = nullptr;  // set: M is not read (may be null), products go through op
    int max_iters = 400;
    double tol = 1e-10;
    int degree = 60;
    int warm_degree = 16;  // first filter degree of a warm start (doubles per step)
    bool warm = false;
    uint64_t seed = 1234;
    int direct_sweeps = 30;  // Jacobi sweep cap when the matrix is diagonalised directly
};
hipError_t lead_eig(double *M, int n, int J, double *X, double *F, double *theta_dev, void *work,
                    const EigOpts &o, int *iters, int *noconv, hipStream_t s);
// Skinny FP64 products C (M x N, N <= 144) = alpha op(A) B + beta E1 with
// split-K partial strips in `part` (at most skinny_part_bound(N) doubles).
hipError_t skinny_gemm(int M, int N, int K, const double *A, int64_t lda, bool at, const double *B, int64_t ldb,
                       double *C, int64_t ldc, double alpha, double beta, const double *E1, double *part,
                       int64_t part_elems, hipStream_t s);
int64_t skinny_part_bound(int max_n);
// Upper Cholesky factor of S + shift * trace(S) * I (w x w, w <= 140) and its
// inverse (one workgroup).
hipError_t chol_inv_upper(const double *S, int w, double shift, double *Rinv, hipStream_t s);
// F (n x J) = columns of X (leading dimension ldx) with the sign that makes
// each column's largest-magnitude entry positive.
hipError_t canonical_cols(const double *X, int64_t n, int ldx, int J, double *F, hipStream_t s);
// Start block of the eigensolver (n x eig_block_width(n, J)) from J
// orthonormal columns U plus pseudo-random columns orthonormalised against
// them; `work` is an eigensolver workspace of eig_work_bytes.
hipError_t eig_seed_block(double *X, int n, int J, const double *U, void *work, uint64_t seed, hipStream_t s);

// ---------------------------------------------------------------- small helpers (eig.hip)
template <class TO>
hipError_t convert_f64(const double *in, TO *out, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- learn.hip
// Learned start: sketch features of mode n from the ordering whose slots are
// the mode-n slices (I_lo = size of mode n+2), the row-wise network, its
// backward pass (scratch learn_backward_scratch(rows) bytes), Adam, the
// subspace-alignment loss (scratch learn_align_scratch_doubles doubles) and
// the start factor.
int learn_param_count();
template <class TV>
hipError_t learn_sketch(const int32_t *ptr, const int32_t *lidx, const TV *lval, int64_t In, int64_t Ilo, int n,
                        uint64_t seed, float *F, float *rho, hipStream_t s);
hipError_t learn_forward(const float *F, const float *rho, int64_t rows, const float *P, float *R, float *Z1,
                         hipStream_t s);
size_t learn_backward_scratch(int64_t rows);
hipError_t learn_backward(const float *F, const float *rho, int64_t rows, const float *P, const float *Z1,
                          const float *dR, float *grad, float *part, hipStream_t s);
hipError_t learn_adam(float *P, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                      float eps, int step, hipStream_t s);
int64_t learn_align_scratch_doubles(int64_t rows, int K, int J);
hipError_t learn_align(const float *R, int64_t rows, int K, const double *A, int J, double shift, double *loss_dev,
                       float *dR, double *scratch, hipStream_t s);
int learn_test_width(int J);
hipError_t learn_start(const float *R, int64_t rows, int J, const double *H, double *F, double *theta, double *gC,
                       double *Q, double *HQ, double *C, double *V, void *eigw, double *part, int64_t part_elems,
                       hipStream_t s);

// ---------------------------------------------------------------- api.hip
// The random start of TK_INIT_RANDOM: F (I x J) with entries uniform on
// [0, 1) from SplitMix64 output n * 2^40 + i * J + r, columns normalised.
hipError_t random_start_fill(double *F, int64_t I, int J, int n, uint64_t seed, hipStream_t s);

// ---------------------------------------------------------------- stream.hip
// Multislice Projection streamed from host memory (tucker_mp_streamed).
int mp_streamed_workspace(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t slab_bytes, size_t *bytes);
int mp_streamed(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t slab_bytes, double *core,
                double *const *F, double *hist, int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb,
                void *stream);

// ---------------------------------------------------------------- implicit.hip
// Multislice Projection through implicit Gram products (tucker_mp_implicit).
int mp_implicit_workspace(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t *bytes);
int mp_implicit(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
                int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream);

// ---------------------------------------------------------------- order_n.hip
// Fourth-order HO-SVD, HOOI and MP behind tucker_hosvd, tucker_hooi and
// tucker_mp (tk_coo.order == 4); the same arguments as those entry points.
size_t order_n_workspace(int algo, const tk_coo *X, const int32_t *J, const tk_opts *o, int *status);
int order_n_mp(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
               int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream);
int order_n_hooi(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
                 int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream);
int order_n_hosvd(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *fit,
                  tk_stats *stats, void *ws, size_t wsb, void *stream);

}  // namespace tk
