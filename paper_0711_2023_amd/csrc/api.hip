// C ABI of the library (include/tucker.h) and the host drivers of HOOI
// (Section 4.2, Figure 3) and Multislice Projection (Section 4.4, Figure 7).
//
// The host only validates arguments, carves the caller's workspace and
// sequences kernels; all arithmetic on tensor data runs on the GPU. The only
// device-to-host traffic is a few status words during preparation, the
// Ritz values of the eigensolver's Rayleigh-Ritz steps, and one fit value
// per sweep.
#include "../../include/tucker.h"
#include "../../include/tucker_stream.h"
#include "../../include/tucker_implicit.h"
#include "common.h"
#include "guards.h"
#include "timer.h"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

namespace tk {

static thread_local char g_err[320];

void g_err_clear() { g_err[0] = 0; }

void set_hip_error(hipError_t e, const char *where) {
    if (g_err[0]) return;
    snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
}

constexpr int kMaxJ = 128;
constexpr int64_t kMaxHosvdDim = 8192;

// Buffers of one learned start: features, norms, network output, FP64
// leading columns / H U, K x K Gram and eigenvectors, eigenvalues, pivots,
// skinny partial strips, eigensolver workspace.
struct LearnBufs {
    float *LF = nullptr, *Lrho = nullptr, *LR = nullptr;
    double *LQ = nullptr, *LHQ = nullptr, *LC = nullptr, *LV = nullptr, *Ltheta = nullptr, *Lg = nullptr;
    double *Lpart = nullptr;
    int64_t Lpart_elems = 0;
    void *Leigw = nullptr;
};

// ------------------------------------------------------------------ small kernels
__global__ void k_fit(const double *normx2, const double *g2, const double *xhx, const double *xh2, double *fit,
                      int general) {
    double nx2 = *normx2;
    double r2 = general ? (nx2 - 2.0 * (*xhx) + (*xh2)) : (nx2 - *g2);
    if (r2 < 0) r2 = 0;
    *fit = 1.0 - sqrt(r2) / sqrt(nx2);
}

// out[p][q][r] = in[perm...]: in is laid out [a][b][c] with (a,b,c) a
// permutation of (p,q,r) given by where[3] (position of p, q, r in the input).
__global__ void k_permute3(const double *in, double *out, int J0, int J1, int J2, int d0, int d1, int d2, int w0,
                           int w1, int w2) {
    const int64_t tot = (int64_t)J0 * J1 * J2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int p = (int)(t / ((int64_t)J1 * J2));
        int rem = (int)(t - (int64_t)p * J1 * J2);
        int q = rem / J2, r = rem - q * J2;
        int c[3];
        c[w0] = p;
        c[w1] = q;
        c[w2] = r;
        out[t] = in[((int64_t)c[0] * d1 + c[1]) * d2 + c[2]];
    }
}

__global__ void k_dot_partial(const double *a, const double *b, int64_t n, double *partials) {
    double acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    __shared__ double ws[16];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i];
        partials[blockIdx.x] = t;
    }
}
__global__ void k_sum_parts(const double *partials, int np, double *out) {
    double acc = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
    __shared__ double ws[16];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i];
        *out = t;
    }
}
static hipError_t dot(const double *a, const double *b, int64_t n, double *partials, double *out, hipStream_t s) {
    k_dot_partial<<<kReduceBlocks, 256, 0, s>>>(a, b, n, partials);
    TK_LAUNCHED();
    k_sum_parts<<<1, 256, 0, s>>>(partials, kReduceBlocks, out);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ plan
static inline int hi_of(int m) { return (m + 2) % 3; }
static inline int lo_of(int m) { return (m + 1) % 3; }

struct Plan {
    int algo, prec, init = TK_INIT_HOSVD;
    int eprec = P64;    // precision whose accuracy sets the eigensolver tolerance
    bool hfit = false;  // also the HO-SVD fit (opts.hosvd_fit): FP64 projection buffer Th
    Tune tune;
    int64_t I[3], nnz;
    int J[3];
    int64_t nslots[3];
    int ldT[3];  // row stride of the projections T(m) (MP pads rows to 16 bytes, BF16 rows to 128 when cheap)
    int ldG[3];  // columns of a T(m) row that the Grams read (J_m rounded to 16 bytes)
    int b[3];
    // device buffers
    int32_t *flags, *nu;
    double *scal;  // [0] normx2 [1] g2 [2] fit [3] xhx [4] xh2
    double *partials;
    int32_t *perm, *tmp, *heads, *pos, *counts, *cursor, *scan;
    int32_t *cidx[3];
    double *cval;
    int32_t *ptr[3], *lidx[3];
    double *lval64[3];
    float *lval32[3];
    void *T[3];        // projections for the Grams (type by precision)
    float *Tcore;      // mixed MP: FP32 copy of the last projection, for the core (rows of ldc)
    float *Fc = nullptr;  // mixed MP: mode-3 factor rows in FP32 padded to ldc, for that projection
    int ldc = 0;
    float *T0f;        // mixed HOOI: FP32 T(0) for mode 3 and the core
    void *Y;           // HOOI second-stage output for the Gram
    float *Y2f;        // mixed HOOI: FP32 Y2 (core input)
    double *Mg;        // Gram (max In^2)
    // HO-SVD start: Gram, eigensolver workspace and Ritz values of mode 3,
    // whose start solve runs beside mode 2's
    double *Mg2 = nullptr, *theta2 = nullptr;
    char *eigw2 = nullptr;
    void *gram_scratch;
    double *Xblk[3];
    void *eigw;
    double *theta;
    float *F32[3] = {nullptr, nullptr, nullptr};
    bf16 *Fbf[3] = {nullptr, nullptr, nullptr};  // BF16 factor copies (rows of J), MFMA operands of the TTMc
    void *Fp[3] = {nullptr, nullptr, nullptr};  // MP: factor rows padded to ldT, zero padding
                                                //     (FP64 / FP32; FP16 for BF16 T)
    double *Th = nullptr;  // FP64 T(2) = X x_3 C^T (J3 columns) for the HO-SVD core
    double *Z, *Gp, *core_split;
    int64_t core_split_elems;
    double *Gx, *Pn[3], *W1, *W2;
    // learned start: one buffer set per start slot (slot 1 serves mode 3,
    // whose start runs beside mode 2's)
    LearnBufs L[2];
    bool blk_ok[3] = {false, false, false};  // Xblk[n] holds a previous block
    bool split = false;                      // MP with split-BF16 Grams (hi and lo parts)
    void *Tlo[3] = {nullptr, nullptr, nullptr};  // lo parts of the projections
    int sweep_solves[3] = {0, 0, 0};         // warm (sweep) eigensolves done per mode
    // MP / SP: the non-empty fibres of each ordering; the projections for
    // the Grams (and the core's FP32 one) write only their rows, into
    // buffers zeroed once per call (zero_projections)
    int32_t *fib[3] = {nullptr, nullptr, nullptr}, *fptr[3] = {nullptr, nullptr, nullptr};
    int64_t nfib[3] = {0, 0, 0};
    // the fibres of each list with more than maxlen[m] nonzeros (the limit
    // of the output type of that ordering's sweep projections)
    int32_t *lf[3] = {nullptr, nullptr, nullptr};
    int64_t nlong[3] = {0, 0, 0};
    int32_t maxlen[3] = {kLongFibreWide, kLongFibreWide, kLongFibreWide};
    // HOOI (projections that write every slot): the slots of each ordering
    // with more than kLongFibreWide nonzeros (on the Zipf-skewed 1000^3
    // tensor 8 beat 16: 214 against 358 us per projection, 91 us uniform)
    int32_t *ls[3] = {nullptr, nullptr, nullptr};
    int64_t nls[3] = {0, 0, 0};
};

static size_t elem_size(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// MP and SP share their buffers (three projections with padded rows).
static inline bool slice_algo(int algo) { return algo == TK_ALGO_MP || algo == TK_ALGO_SP; }

static GramTerm term_of(const Plan &p, int m, int n, const void *base) {
    // T(m) is [i_hi][i_lo][r < ldT]; rows of the mode-n unfolding are i_n.
    // Padding columns are zero and only add zero products.
    GramTerm t;
    t.base = base;
    // Columns from ldG on (the padding of rows to whole 128-byte lines) are
    // skipped: chunks of ldG at a stride of ldT.
    const int64_t Jm = p.ldT[m], Jg = p.ldG[m], Ilo = p.I[lo_of(m)], Ihi = p.I[hi_of(m)];
    if (hi_of(m) == n) {
        t.s_row = Ilo * Jm;
        t.chunk_len = Jg == Jm ? Ilo * Jm : Jg;
        t.nchunks = Jg == Jm ? 1 : Ilo;
        t.s_chunk = Jg == Jm ? 0 : Jm;
    } else {
        t.s_row = Jm;
        t.chunk_len = Jg;
        t.nchunks = Ihi;
        t.s_chunk = Ilo * Jm;
    }
    return t;
}

// M_n from the projections T(ma), T(mb): two terms, or six for split-BF16
// (hi hi^T + hi lo^T + lo hi^T of each; the dropped lo lo^T is below the
// rounding of the others)
static hipError_t mp_gram(Plan &p, int n, int ma, int mb, hipStream_t s) {
    GramTerm g[kGramMaxTerms];
    int nt = 0;
    for (int m : {ma, mb}) {
        g[nt++] = term_of(p, m, n, p.T[m]);
        if (p.split) {
            GramTerm hl = term_of(p, m, n, p.T[m]);
            hl.base_b = p.Tlo[m];
            GramTerm lh = term_of(p, m, n, p.Tlo[m]);
            lh.base_b = p.T[m];
            g[nt++] = hl;
            g[nt++] = lh;
        }
    }
    return gram((int)p.I[n], p.prec, nt, g, p.Mg, p.gram_scratch, s, p.tune);
}

static void carve(Plan &p, Arena &ar) {
    const int64_t nnz = p.nnz > 0 ? p.nnz : 1;
    const int prec = p.prec;
    int64_t maxslots = 1, maxI = 1;
    for (int m = 0; m < 3; ++m) {
        maxslots = std::max(maxslots, p.nslots[m]);
        maxI = std::max(maxI, p.I[m]);
    }
    p.flags = ar.take<int32_t>(4);
    p.nu = ar.take<int32_t>(4);
    p.scal = ar.take<double>(8);
    p.partials = ar.take<double>(kReduceBlocks);
    p.perm = ar.take<int32_t>(nnz);
    p.tmp = ar.take<int32_t>(nnz);
    p.heads = ar.take<int32_t>(nnz + 1);
    p.pos = ar.take<int32_t>(nnz + 1);
    p.counts = ar.take<int32_t>(maxslots);
    p.cursor = ar.take<int32_t>(maxslots + 1);
    p.scan = ar.take<int32_t>(std::max(scan_scratch_ints(maxslots), scan_scratch_ints(nnz + 1)));
    for (int n = 0; n < 3; ++n) p.cidx[n] = ar.take<int32_t>(nnz);
    p.cval = ar.take<double>(nnz);
    for (int m = 0; m < 3; ++m) {
        p.ptr[m] = ar.take<int32_t>(p.nslots[m] + 1);
        p.lidx[m] = ar.take<int32_t>(nnz);
        p.lval64[m] = ar.take<double>(nnz);
        p.lval32[m] = prec != P64 ? ar.take<float>(nnz) : nullptr;
    }
    p.Tcore = nullptr;
    p.T0f = nullptr;
    p.Y = nullptr;
    p.Y2f = nullptr;
    for (int m = 0; m < 3; ++m) p.T[m] = nullptr;
    const size_t es = elem_size(prec);
    if (slice_algo(p.algo)) {
        for (int m = 0; m < 3; ++m) {
            const int64_t cap = std::min(p.nslots[m], nnz);
            p.fib[m] = ar.take<int32_t>(cap);
            p.fptr[m] = ar.take<int32_t>(cap + 1);
            p.lf[m] = ar.take<int32_t>(nnz / (kLongFibreWide + 1) + 1);
        }
        for (int m = 0; m < 3; ++m) p.T[m] = ar.take<char>((int64_t)(p.nslots[m] * p.ldT[m] * es));
        if (p.split)
            for (int m = 0; m < 3; ++m) p.Tlo[m] = ar.take<char>((int64_t)(p.nslots[m] * p.ldT[m] * es));
        if (prec == PBF16) {
            p.ldc = (int)ceil_div(p.J[2], 4) * 4;  // 16-byte rows: the vector projection
            p.Tcore = ar.take<float>(p.nslots[2] * p.ldc);
            p.Fc = ar.take<float>(p.I[2] * p.ldc);
        }
    } else if (p.algo == TK_ALGO_HOOI) {
        for (int m = 0; m < 3; ++m) p.ls[m] = ar.take<int32_t>(nnz / (kLongFibreWide + 1) + 1);
        p.T[2] = ar.take<char>((int64_t)(p.nslots[2] * p.J[2] * es));
        if (prec == PBF16)
            p.T0f = ar.take<float>(p.nslots[0] * p.J[0]);
        else
            p.T[0] = ar.take<char>((int64_t)(p.nslots[0] * p.J[0] * es));
        int64_t ymax = 0;
        for (int n = 0; n < 3; ++n)
            ymax = std::max(ymax, p.I[n] * (int64_t)p.J[(n + 1) % 3] * p.J[(n + 2) % 3]);
        p.Y = ar.take<char>(ymax * (prec == P64 ? 8 : 4));
        if (prec == PBF16) p.Y2f = nullptr;
    } else {  // fit, HO-SVD: FP64 T(2) for the core
        p.T[2] = ar.take<double>(p.nslots[2] * p.J[2]);
    }
    p.Th = p.algo == TK_ALGO_FIT || p.algo == TK_ALGO_HOSVD ? (double *)p.T[2]
           : p.hfit ? ar.take<double>(p.nslots[2] * p.J[2]) : nullptr;
    if (p.algo != TK_ALGO_FIT) {
        p.Mg = ar.take<double>(maxI * maxI);
        size_t gs = 0;
        for (int n = 0; n < 3 && p.algo != TK_ALGO_HOSVD; ++n) {
            int64_t K[kGramMaxTerms];
            int gprec = prec;
            if (p.algo == TK_ALGO_SP) {
                // SP: one projection per Gram, T((n+2)%3) (Figure 5)
                const int m = (n + 2) % 3;
                const int per = p.split ? 3 : 1;
                for (int q = 0; q < per; ++q) K[q] = p.nslots[m] / p.I[n] * p.ldG[m];
                gs = std::max(gs, gram_scratch_bytes((int)p.I[n], gprec, per, K, p.tune));
            } else if (slice_algo(p.algo)) {
                int m1 = (n + 1) % 3, m2 = (n + 2) % 3;
                const int64_t K1 = p.nslots[m1] / p.I[n] * p.ldG[m1], K2 = p.nslots[m2] / p.I[n] * p.ldG[m2];
                const int per = p.split ? 3 : 1;  // hi.hi (+ hi.lo, lo.hi)
                for (int q = 0; q < per; ++q) {
                    K[q] = K1;
                    K[per + q] = K2;
                }
                gs = std::max(gs, gram_scratch_bytes((int)p.I[n], gprec, 2 * per, K, p.tune));
            } else if (p.algo == TK_ALGO_HOOI) {
                K[0] = (int64_t)p.J[(n + 1) % 3] * p.J[(n + 2) % 3];
                gprec = prec == P64 ? P64 : P32;
                gs = std::max(gs, gram_scratch_bytes((int)p.I[n], gprec, 1, K, p.tune));
            }
        }
        p.gram_scratch = ar.take<char>((int64_t)gs);
        size_t ew = 0;
        int bmax = 1;
        for (int n = 0; n < 3; ++n) {
            p.b[n] = eig_block_width((int)p.I[n], p.J[n]);
            bmax = std::max(bmax, p.b[n]);
            p.Xblk[n] = ar.take<double>(p.I[n] * p.b[n]);
            ew = std::max(ew, eig_work_bytes((int)p.I[n], p.b[n]));
        }
        p.eigw = ar.take<char>((int64_t)ew);
        p.theta = ar.take<double>(std::max<int64_t>(bmax, maxI));
        if (p.init == TK_INIT_HOSVD || p.init == TK_INIT_LEARNED) {
            p.Mg2 = ar.take<double>(p.I[2] * p.I[2]);
            p.eigw2 = ar.take<char>((int64_t)eig_work_bytes((int)p.I[2], p.b[2]));
            p.theta2 = ar.take<double>(std::max<int64_t>(p.b[2], p.I[2]));
        }
        for (int n = 0; n < 3; ++n) {
            p.F32[n] = prec != P64 ? ar.take<float>(p.I[n] * p.J[n]) : nullptr;
            p.Fbf[n] = prec == PBF16 ? ar.take<bf16>(p.I[n] * p.J[n]) : nullptr;
            // padded factor rows for the projections: FP16 for BF16 T (more
            // significand than BF16 for entries of orthonormal columns, and
            // the projection's FMA takes FP16 operands directly), FP32 for
            // split Grams (their lo parts need more than 16-bit factors)
            p.Fp[n] = slice_algo(p.algo)
                          ? ar.take<char>(p.I[n] * p.ldT[n] * (int64_t)(p.split ? 4 : elem_size(prec)))
                          : nullptr;
        }
    }
    const int64_t J0 = p.J[0], J1 = p.J[1], J2 = p.J[2];
    // core / fit contractions
    p.Z = ar.take<double>(std::max(p.I[1] * J0 * J2, (int64_t)1));
    p.Gp = ar.take<double>(J0 * J1 * J2);
    p.core_split_elems = 8 * J0 * J1 * J2;
    p.core_split = ar.take<double>(p.core_split_elems);
    if (p.algo == TK_ALGO_FIT) {
        p.Gx = ar.take<double>(J0 * J1 * J2);
        for (int n = 0; n < 3; ++n) p.Pn[n] = ar.take<double>((int64_t)p.J[n] * p.J[n]);
        p.W1 = ar.take<double>(J0 * J1 * J2);
        p.W2 = ar.take<double>(J0 * J1 * J2);
    }
    if (p.init == TK_INIT_LEARNED && p.algo != TK_ALGO_FIT && p.algo != TK_ALGO_HOSVD) {
        int64_t In = std::max({p.I[0], p.I[1], p.I[2]});
        int Km = learn_test_width(std::max({p.J[0], p.J[1], p.J[2]}));
        for (int k = 0; k < 2; ++k) {
            LearnBufs &b = p.L[k];
            const int64_t Ik = k == 0 ? In : p.I[2];
            const int Kk = k == 0 ? Km : learn_test_width(p.J[2]);
            b.LF = ar.take<float>(Ik * 64);
            b.Lrho = ar.take<float>(Ik);
            b.LR = ar.take<float>(Ik * 128);
            b.LQ = ar.take<double>(Ik * Kk);
            b.LHQ = ar.take<double>(Ik * Kk);
            b.LC = ar.take<double>((int64_t)Kk * Kk);
            b.LV = ar.take<double>((int64_t)Kk * Kk);
            b.Ltheta = ar.take<double>(Kk);
            b.Lg = ar.take<double>(Kk);
            b.Lpart_elems = skinny_part_bound(Kk);
            b.Lpart = ar.take<double>(b.Lpart_elems);
            b.Leigw = ar.take<char>((int64_t)eig_work_bytes(Kk, Kk));
        }
    }
}

static int check_coo(const tk_coo *X, const int32_t *J) {
    if (!X || !J || !X->dims || X->order != 3) return TK_ERR_ARG;
    if (X->nnz < 0 || X->nnz >= (int64_t)INT32_MAX - 1) return TK_ERR_ARG;
    if (X->nnz > 0 && (!X->idx[0] || !X->idx[1] || !X->idx[2] || !X->vals)) return TK_ERR_ARG;
    for (int n = 0; n < 3; ++n) {
        if (X->dims[n] < 1 || X->dims[n] >= INT32_MAX) return TK_ERR_ARG;
        if (J[n] < 1 || J[n] > X->dims[n] || J[n] > kMaxJ) return TK_ERR_ARG;
    }
    for (int m = 0; m < 3; ++m)
        if (X->dims[hi_of(m)] * X->dims[lo_of(m)] >= (int64_t)INT32_MAX) return TK_ERR_ARG;
    return TK_OK;
}

static int check_opts(const tk_opts *o, const tk_coo *X, int algo) {
    if (!o) return TK_ERR_ARG;
    if (o->precision < 0 || o->precision > 3) return TK_ERR_ARG;
    if (o->precision == TK_MIXED_BF16X3 && !slice_algo(algo)) return TK_ERR_ARG;
    if (algo == TK_ALGO_HOSVD) {
        if (o->eig_max_iters < 1 || !(o->eig_tol >= 0.0)) return TK_ERR_ARG;
        for (int n = 0; n < 3; ++n)
            if (X->dims[n] > kMaxHosvdDim) return TK_ERR_ARG;
        return TK_OK;
    }
    if (o->init != TK_INIT_HOSVD && o->init != TK_INIT_GIVEN && o->init != TK_INIT_LEARNED &&
        o->init != TK_INIT_RANDOM)
        return TK_ERR_ARG;
    if (o->init == TK_INIT_LEARNED && (!o->model || algo == TK_ALGO_SP)) return TK_ERR_ARG;
    if (o->hosvd_fit != 0 && o->hosvd_fit != 1) return TK_ERR_ARG;
    // the report uses the factor buffers as scratch: not with a start read
    // from them or one that replaces the HO-SVD
    if (o->hosvd_fit && (o->init == TK_INIT_GIVEN || o->init == TK_INIT_LEARNED)) return TK_ERR_ARG;
    if (o->tune) {
        const tk_tune *t = o->tune;
        auto in = [](int32_t v, int32_t lo, int32_t hi) { return v == 0 || (v >= lo && v <= hi); };
        if (!in(t->proj_elems, 1024, 65536) || !in(t->proj_min_blocks, 64, 16384) ||
            !in(t->gram_items, 64, 16384) || !in(t->gram_min_stages, 1, 64))
            return TK_ERR_ARG;
    }
    if (o->max_iters < 0 || o->eig_max_iters < 1) return TK_ERR_ARG;
    if (!(o->eig_tol >= 0.0) || std::isnan(o->tol)) return TK_ERR_ARG;
    // start Grams X_(n) X_(n)^T: modes 2 and 3 for an HO-SVD start (or the
    // learned start's fallback), mode 3 alone for SP's; all three for the
    // HO-SVD fit
    const bool hs = o->init == TK_INIT_HOSVD || o->init == TK_INIT_LEARNED;
    for (int n = 0; n < 3; ++n) {
        const bool needs = o->hosvd_fit || (hs && (algo == TK_ALGO_SP ? n == 2 : n >= 1));
        if (needs && X->dims[n] > kMaxHosvdDim) return TK_ERR_ARG;
    }
    return TK_OK;
}

static Tune tune_of(const tk_tune *t) {
    Tune tn;
    if (t) {
        if (t->proj_elems) tn.proj_elems = t->proj_elems;
        if (t->proj_min_blocks) tn.proj_min_blocks = t->proj_min_blocks;
        if (t->gram_items) tn.gram_items = t->gram_items;
        if (t->gram_min_stages) tn.gram_min_stages = t->gram_min_stages;
    }
    return tn;
}

static void plan_init(Plan &p, int algo, int prec, const tk_coo *X, const int32_t *J, int init = TK_INIT_HOSVD,
                      const tk_tune *tune = nullptr, bool hfit = false) {
    p.algo = algo;
    p.hfit = hfit && algo != TK_ALGO_FIT && algo != TK_ALGO_HOSVD;
    p.split = prec == TK_MIXED_BF16X3;
    p.eprec = p.split ? P32 : prec;
    if (p.split) prec = PBF16;  // BF16 storage, two parts
    p.prec = prec;
    p.init = init;
    p.tune = tune_of(tune);
    p.nnz = X->nnz;
    for (int n = 0; n < 3; ++n) {
        p.I[n] = X->dims[n];
        p.J[n] = J[n];
    }
    for (int m = 0; m < 3; ++m) p.nslots[m] = p.I[hi_of(m)] * p.I[lo_of(m)];
    const int vec = prec == P64 ? 2 : (prec == P32 ? 4 : 8);  // elements per 16 bytes
    for (int m = 0; m < 3; ++m) {
        p.ldG[m] = slice_algo(algo) ? (int)ceil_div(p.J[m], vec) * vec : p.J[m];
        p.ldT[m] = p.ldG[m];
        // BF16 rows padded on to whole 128-byte lines where that adds at most
        // a sixth to the row: the projection then stores whole lines (at
        // J = 50, rows of 64 instead of 56: 24.8 -> 22.0 us per launch at
        // 1000^3), and the Grams skip the extra columns
        const int64_t line = ceil_div((int64_t)p.ldG[m] * 2, 128) * 64;
        if (slice_algo(algo) && prec == PBF16 && 6 * line <= 7 * (int64_t)p.ldG[m]) p.ldT[m] = (int)line;
    }
}

}  // namespace tk

using namespace tk;

extern "C" {

void tucker_default_opts(tk_opts *o) {
    if (!o) return;
    o->precision = TK_FP32;
    o->init = TK_INIT_HOSVD;
    o->max_iters = 50;
    o->tol = 1e-4;
    o->eig_max_iters = 400;
    o->eig_tol = 0.0;
    o->timing = 0;
    o->model = nullptr;
    o->seed = 0x5eedull;
    o->tune = nullptr;
    o->hosvd_fit = 0;
    o->trace = nullptr;
}

const char *tucker_strerror(int st) {
    switch (st) {
        case TK_OK: return "success";
        case TK_WARN_NOCONV: return "an eigensolve reached its iteration cap (outputs are valid)";
        case TK_ERR_ARG: return "invalid argument";
        case TK_ERR_INDEX: return "a coordinate is outside its mode's range";
        case TK_ERR_VALUE: return "a value is NaN or infinite";
        case TK_ERR_EMPTY: return "the tensor has zero norm; the fit is undefined";
        case TK_ERR_WORKSPACE: return "workspace missing or too small";
        case TK_ERR_DEVICE: return g_err[0] ? g_err : "HIP error";
        case TK_ERR_SIZE:
            return "the problem needs more scratch than the static buffer of tucker_fit_static holds "
                   "(TK_STATIC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

int tucker_workspace_bytes(int32_t algo, const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                           size_t *bytes) {
    if (!bytes) return TK_ERR_ARG;
    if (X && X->order == 4) {  // fourth order: HOOI, MP, HO-SVD
        if (algo != TK_ALGO_HOOI && algo != TK_ALGO_MP && algo != TK_ALGO_HOSVD) return TK_ERR_ARG;
        int st4 = TK_OK;
        const size_t b = order_n_workspace(algo, X, core_dims, opt, &st4);
        if (st4) return st4;
        *bytes = b;
        return TK_OK;
    }
    int st = check_coo(X, core_dims);
    if (st) return st;
    if (algo < TK_ALGO_HOOI || algo > TK_ALGO_HOSVD) return TK_ERR_ARG;
    int prec = P64;
    if (algo != TK_ALGO_FIT) {
        if ((st = check_opts(opt, X, algo))) return st;
        prec = algo == TK_ALGO_HOSVD ? P64 : opt->precision;
    }
    const bool dec = algo != TK_ALGO_FIT && algo != TK_ALGO_HOSVD;
    Plan p;
    plan_init(p, algo, prec, X, core_dims, dec ? opt->init : TK_INIT_HOSVD, dec ? opt->tune : nullptr,
              dec && opt->hosvd_fit);
    Arena ar;
    carve(p, ar);
    *bytes = ar.used + 256;
    return TK_OK;
}

}  // extern "C"

namespace tk {

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define ST(call)                          \
    do {                                  \
        hipError_t e_ = (call);           \
        if (e_ != hipSuccess) {           \
            set_hip_error(e_, #call);     \
            return TK_ERR_DEVICE;         \
        }                                 \
    } while (0)

// An ordering failed its range checks (guards.h): nothing was written out
// of bounds, but the decomposition cannot go on.
static int order_failed(int r) {
    if (r == TK_ERR_DEVICE && !g_err[0])
        snprintf(g_err, sizeof(g_err), "fibre ordering failed its range checks (scan total or slot position)");
    return r;
}

// The fibre list of ordering m when it exists and `zeroed_target` (the
// projection goes to a buffer zeroed by zero_projections), else none.
static FibreList fibres_of(const Plan &p, int m, bool zeroed_target) {
    FibreList fl;
    if (p.ls[m] && p.nls[m] > 0) {  // every slot written: no zeroed target needed
        fl.ls = p.ls[m];
        fl.nls = p.nls[m];
        fl.slot_maxlen = kLongFibreWide;
    }
    if (p.fib[m] && zeroed_target) {
        fl.fib = p.fib[m];
        fl.fptr = p.fptr[m];
        fl.n = p.nfib[m];
        if (p.nlong[m] > 0) {
            fl.lf = p.lf[m];
            fl.nlong = p.nlong[m];
            fl.maxlen = p.maxlen[m];
        }
    }
    return fl;
}

// Zero the buffers whose empty-fibre rows the fibre-list projections leave
// untouched: T(m) (and their lo parts) and the core's FP32 projection.
static hipError_t zero_projections(Plan &p, hipStream_t s) {
    if (!p.fib[0]) return hipSuccess;
    const size_t es = elem_size(p.prec);
    for (int m = 0; m < 3; ++m) {
        const int64_t words = p.nslots[m] * p.ldT[m] * (int64_t)es / 4;  // rows are whole 16-byte chunks
        TK_HIP(fill_i32((int32_t *)p.T[m], words, 0, s));
        if (p.Tlo[m]) TK_HIP(fill_i32((int32_t *)p.Tlo[m], words, 0, s));
    }
    if (p.Tcore) TK_HIP(fill_i32((int32_t *)p.Tcore, p.nslots[2] * (int64_t)p.ldc, 0, s));
    return hipSuccess;
}

// Validation, duplicate summing, orderings, ||X||^2.
static int prep(Plan &p, const tk_coo *X, hipStream_t s, int64_t *nu_out, double *normx2_out) {
    const int64_t dims[3] = {p.I[0], p.I[1], p.I[2]};
    ST(validate(X->idx, X->vals, p.nnz, dims, p.flags, s));
    int32_t flags = 0;
    ST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    OrderScratch sc{p.counts, p.cursor, p.tmp, p.scan};
    ST(build_order(X->idx, p.nnz, dims, 2, p.ptr[2], p.perm, sc, p.flags, s));
    // the duplicate pass reads through perm: the ordering must have passed
    // its range checks first
    ST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return order_failed(r);
    int32_t *cidx[3] = {p.cidx[0], p.cidx[1], p.cidx[2]};
    ST(dedup(X->idx, X->vals, p.nnz, p.perm, p.heads, p.pos, p.scan, cidx, p.cval, p.nu, s));
    int32_t nu = 0;
    ST(hipMemcpyAsync(&nu, p.nu, 4, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    ST(sumsq(p.cval, nu, p.partials, p.scal + 0, s));
    const int32_t *cid[3] = {p.cidx[0], p.cidx[1], p.cidx[2]};
    for (int m = 0; m < 3; ++m) {
        ST(build_order(cid, nu, dims, m, p.ptr[m], p.perm, sc, p.flags, s));
        ST(gather_leaf<double>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval64[m], p.flags, s));
        if (p.lval32[m])
            ST(gather_leaf<float>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval32[m], p.flags, s));
    }
    // MP / SP: non-empty fibre lists of the three orderings
    int32_t nfib[3] = {0, 0, 0};
    if (p.fib[0])
        for (int m = 0; m < 3; ++m) {
            ST(fibre_list(p.ptr[m], p.nslots[m], std::min<int64_t>(p.nslots[m], std::max<int64_t>(p.nnz, 1)),
                          p.fib[m], p.fptr[m], p.counts, p.cursor, p.scan, p.flags, s));
            ST(hipMemcpyAsync(&nfib[m], p.cursor + p.nslots[m], 4, hipMemcpyDeviceToHost, s));
        }
    double nx2 = 0;
    ST(hipMemcpyAsync(&nx2, p.scal + 0, 8, hipMemcpyDeviceToHost, s));
    ST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return order_failed(r);
    for (int m = 0; m < 3; ++m) p.nfib[m] = nfib[m];
    // HOOI: the long slots of each ordering
    if (p.ls[0]) {
        int32_t nls[3] = {0, 0, 0};
        for (int m = 0; m < 3; ++m) {
            ST(long_fibres(p.ptr[m], p.nslots[m], kLongFibreWide, p.nnz / (kLongFibreWide + 1) + 1, p.ls[m],
                           p.counts, p.cursor, p.scan, p.flags, s));
            ST(hipMemcpyAsync(&nls[m], p.cursor + p.nslots[m], 4, hipMemcpyDeviceToHost, s));
            ST(hipStreamSynchronize(s));  // the next list reuses the scan buffers
        }
        ST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
        ST(hipStreamSynchronize(s));
        if (int r = prep_status(flags)) return order_failed(r);
        for (int m = 0; m < 3; ++m) p.nls[m] = nls[m];
    }
    // the long fibres of each list (their own workgroups in the projection launch)
    if (p.fib[0]) {
        int32_t nlong[3] = {0, 0, 0};
        for (int m = 0; m < 3; ++m) {
            // BF16 rows, except mode 3's in mixed precision, which come from
            // the FP32 projection for the core (project_dual)
            const bool bf16_rows = p.prec == PBF16 && (m < 2 || p.split);
            p.maxlen[m] = bf16_rows ? kLongFibreBf16 : kLongFibreWide;
            ST(long_fibres(p.fptr[m], nfib[m], p.maxlen[m], p.nnz / (kLongFibreWide + 1) + 1, p.lf[m], p.counts,
                           p.cursor, p.scan, p.flags, s));
            ST(hipMemcpyAsync(&nlong[m], p.cursor + nfib[m], 4, hipMemcpyDeviceToHost, s));
            ST(hipStreamSynchronize(s));  // the next list reuses the scan buffers
        }
        ST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
        ST(hipStreamSynchronize(s));
        if (int r = prep_status(flags)) return order_failed(r);
        for (int m = 0; m < 3; ++m) p.nlong[m] = nlong[m];
    }
    *nu_out = nu;
    *normx2_out = nx2;
    if (!(nx2 > 0.0)) return TK_ERR_EMPTY;
    ST(zero_projections(p, s));
    return TK_OK;
}

// T(m) = X x_m F^T for the given output precision. F64 is the FP64 factor;
// its FP32 copy must be current for FP32 / BF16 outputs.
static hipError_t project_m(Plan &p, int m, const double *F64, void *T, int out_prec, hipStream_t s, int ld = 0,
                            KernelEvents ke = KernelEvents()) {
    const int J = p.J[m];
    if (ld <= 0) ld = p.ldT[m];
    const int32_t *ptr = p.ptr[m], *lidx = p.lidx[m];
    const int64_t I = p.I[m], ns = p.nslots[m];
    // the Gram buffers T(m) were zeroed once (zero_projections): only the
    // rows of non-empty fibres are written
    const FibreList fl = fibres_of(p, m, T == p.T[m] && ld == p.ldT[m]);
    if (p.split && T == p.T[m] && out_prec == PBF16 && ld == p.ldT[m])  // the Gram copy: hi and lo parts
        return project_split(ptr, lidx, p.lval32[m], (const float *)p.Fp[m], I, ld, J, ns, p.nnz, (bf16 *)T,
                             (bf16 *)p.Tlo[m], s, p.tune, ke, fl);
    // the padded copy (rows of ldT) when T has that stride and type, else
    // rows of J
    const bool padded = p.Fp[m] && ld == p.ldT[m] && out_prec == p.prec;
    if (padded) {
        if (out_prec == P64)
            return project<double, double, double>(ptr, lidx, p.lval64[m], (const double *)p.Fp[m], I, ld, J, ld, ns,
                                                   p.nnz, (double *)T, s, p.tune, ke, fl);
        if (out_prec == P32)
            return project<float, float, float>(ptr, lidx, p.lval32[m], (const float *)p.Fp[m], I, ld, J, ld, ns,
                                                p.nnz, (float *)T, s, p.tune, ke, fl);
        return project<float, f16, bf16>(ptr, lidx, p.lval32[m], (const f16 *)p.Fp[m], I, ld, J, ld, ns, p.nnz,
                                         (bf16 *)T, s, p.tune, ke, fl);
    }
    // rows of J (HOOI): every slot is written; only the long-slot list applies
    FibreList sl;
    sl.ls = fl.ls;
    sl.nls = fl.nls;
    sl.slot_maxlen = fl.slot_maxlen;
    if (out_prec == P64)
        return project<double, double, double>(ptr, lidx, p.lval64[m], F64, I, J, J, ld, ns, p.nnz, (double *)T, s,
                                               p.tune, ke, sl);
    if (out_prec == P32)
        return project<float, float, float>(ptr, lidx, p.lval32[m], p.F32[m], I, J, J, ld, ns, p.nnz, (float *)T, s,
                                            p.tune, ke, sl);
    return project<float, float, bf16>(ptr, lidx, p.lval32[m], p.F32[m], I, J, J, ld, ns, p.nnz, (bf16 *)T, s,
                                       p.tune, ke, sl);
}

static hipError_t refresh_copies(Plan &p, int n, const double *F, hipStream_t s) {
    const int64_t cnt = p.I[n] * p.J[n];
    if (p.F32[n]) TK_HIP(convert_f64<float>(F, p.F32[n], cnt, s));
    if (p.Fbf[n]) TK_HIP(convert_f64<bf16>(F, p.Fbf[n], cnt, s));
    if (p.Fc && n == 2) TK_HIP(pad_rows<float>(F, p.I[2], p.J[2], p.ldc, p.Fc, s));
    if (p.Fp[n]) {
        if (p.prec == P64)
            TK_HIP(pad_rows<double>(F, p.I[n], p.J[n], p.ldT[n], (double *)p.Fp[n], s));
        else if (p.prec == P32 || p.split)
            TK_HIP(pad_rows<float>(F, p.I[n], p.J[n], p.ldT[n], (float *)p.Fp[n], s));
        else
            TK_HIP(pad_rows<f16>(F, p.I[n], p.J[n], p.ldT[n], (f16 *)p.Fp[n], s));
    }
    return hipSuccess;
}

// MP core from T(2) = X x_3 C^T stored [i1][i0][r2] (FP64 or FP32):
// Z[i1][p][r] = sum_i0 A[i0][p] T[i1][i0][r]; G'[q][p][r] = sum_i1 B[i1][q] Z[i1][p][r];
// core[p][q][r] = G'[q][p][r].
static hipError_t core_from_T2(Plan &p, const void *T2, int ldt, bool t2_is_f64, const double *A, const double *B,
                               double *core, hipStream_t s) {
    const int J0 = p.J[0], J1 = p.J[1], J2 = p.J[2];
    GemmArgs g;
    g.M = J0;
    g.N = J2;
    g.K = (int)p.I[0];
    g.batch = (int)p.I[1];
    g.A = A;
    g.lda = J0;
    g.a_trans = true;
    g.B = T2;
    g.ldb = ldt;
    g.sB = p.I[0] * ldt;
    g.C = p.Z;
    g.ldc = J2;
    g.sC = (int64_t)J0 * J2;
    g.prec = t2_is_f64 ? P64 : 3;
    g.out_type = P64;
    TK_HIP(gemm(g, s));
    GemmArgs h;
    h.M = J1;
    h.N = J0 * J2;
    h.K = (int)p.I[1];
    h.batch = 1;
    h.A = B;
    h.lda = J1;
    h.a_trans = true;
    h.B = p.Z;
    h.ldb = (int64_t)J0 * J2;
    h.sB = 0;
    h.C = p.Gp;
    h.ldc = (int64_t)J0 * J2;
    h.sC = 0;
    h.prec = P64;
    h.out_type = P64;
    int tiles = (int)(ceil_div(J1, 64) * ceil_div((int64_t)J0 * J2, 64));
    h.splitk = std::max(1, std::min(8, 256 / std::max(1, tiles)));
    h.split_scratch = p.core_split;
    TK_HIP(gemm(h, s));
    // G' is [q][p][r]: core[p][q][r] = G'[q][p][r]
    k_permute3<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)J0 * J1 * J2, 256), 65536), 256, 0, s>>>(
        p.Gp, core, J0, J1, J2, J1, J0, J2, 1, 0, 2);
    TK_LAUNCHED();
    return hipSuccess;
}

// fit = 1 - sqrt(||X||^2 - ||G||^2) / ||X|| (the identity for orthonormal
// factors and G = X x_n A(n)^T); *g2 (optional) receives ||G||^2.
static int finish_fit(Plan &p, const double *core, hipStream_t s, double *fit, double *g2 = nullptr) {
    const int64_t nJ = (int64_t)p.J[0] * p.J[1] * p.J[2];
    ST(sumsq(core, nJ, p.partials, p.scal + 1, s));
    k_fit<<<1, 1, 0, s>>>(p.scal + 0, p.scal + 1, nullptr, nullptr, p.scal + 2, 0);
    ST(hipGetLastError());
    double gf[2];  // ||G||^2, fit
    ST(hipMemcpyAsync(gf, p.scal + 1, 16, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    *fit = gf[1];
    if (g2) *g2 = gf[0];
    return TK_OK;
}

static int run_eig(Plan &p, int n, double *M, double *F, bool warm, const tk_opts *o, tk_stats *st,
                   int *noconv_any, hipStream_t s, void *eigw = nullptr, double *theta = nullptr) {
    EigOpts eo;
    eo.max_iters = o->eig_max_iters;
    // 0 = by precision: FP64 follows the oracle's exact eigensolver closely;
    // FP32 projections limit the Gram to about 1e-7 relative, BF16 ones (8
    // significant bits) to about 1e-3, so the sum of the leading Ritz values
    // is resolved to a tenth of that: 1e-8 and 1e-4 of itself respectively
    eo.tol = o->eig_tol > 0 ? o->eig_tol : (p.eprec == P64 ? 1e-12 : (p.eprec == P32 ? 1e-8 : 1e-4));
    eo.warm = warm && p.blk_ok[n];
    // a block left by the previous sweep's solve of this mode is usually
    // converged or nearly so: its filter starts at a low degree. Blocks from
    // the start (HO-SVD of X_(n) X_(n)^T, or the learned start) belong to
    // another matrix and get the full degree at once.
    if (eo.warm && p.sweep_solves[n] == 0) eo.warm_degree = eo.degree;
    if (warm) p.sweep_solves[n] += 1;
    eo.seed = 0x5eed0000ull + (uint64_t)n;
    int it = 0, nc = 0;
    ST(lead_eig(M, (int)p.I[n], p.J[n], p.Xblk[n], F, theta ? theta : p.theta, eigw ? eigw : p.eigw, eo, &it, &nc,
                s));
    if (st) {
        st->eig_iters += it;
        st->eig_noconv += nc;
    }
    if (nc) *noconv_any = 1;
    p.blk_ok[n] = true;
    ST(refresh_copies(p, n, F, s));
    return TK_OK;
}

static int common_start(int algo, const tk_coo *X, const int32_t *J, const tk_opts *o, double *core,
                        double *const *factors, double *fit_history, int32_t *iters_done, void *ws, size_t wsb,
                        Plan &p) {
    int st = check_coo(X, J);
    if (st) return st;
    if ((st = check_opts(o, X, algo))) return st;
    if (!core || !factors || !factors[0] || !factors[1] || !factors[2] || !iters_done) return TK_ERR_ARG;
    if (o->max_iters > 0 && !fit_history) return TK_ERR_ARG;
    if (X->nnz == 0) return TK_ERR_EMPTY;
    plan_init(p, algo, o->precision, X, J, o->init, o->tune, o->hosvd_fit != 0);
    Arena ar;
    carve(p, ar);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    carve(p, ar);
    g_err[0] = 0;
    return TK_OK;
}

// Learned start of mode n into F (In x Jn): sketch, network, Rayleigh-Ritz of
// H_n on the span of the network's first K outputs. Returns 1 when the start
// is accepted, 0 when the mode must fall back to HO-SVD (H_n is left in p.Mg
// either way), or a negative status.
static int learned_mode(Plan &p, int n, const tk_opts *o, double *F, double nx2, hipStream_t s, LearnBufs &lb,
                        double *Mg) {
    const int64_t dims[3] = {p.I[0], p.I[1], p.I[2]};
    const int64_t In = p.I[n];
    const int J = p.J[n], K = learn_test_width(J);
    const int sl = (n + 1) % 3;  // ordering whose slots are the mode-n slices
    if (p.lval32[sl])
        ST(learn_sketch<float>(p.ptr[sl], p.lidx[sl], p.lval32[sl], In, p.I[lo_of(sl)], n, o->seed, lb.LF, lb.Lrho,
                               s));
    else
        ST(learn_sketch<double>(p.ptr[sl], p.lidx[sl], p.lval64[sl], In, p.I[lo_of(sl)], n, o->seed, lb.LF,
                                lb.Lrho, s));
    ST(learn_forward(lb.LF, lb.Lrho, In, o->model, lb.LR, nullptr, s));
    ST(hosvd_gram(n, dims, p.ptr[n], p.lidx[n], p.lval64[n], p.ptr[sl], p.lidx[sl], p.lval64[sl], Mg, s));
    if (K > In) return 0;  // no room for a test subspace: HO-SVD
    ST(learn_start(lb.LR, In, J, Mg, F, lb.Ltheta, lb.Lg, lb.LQ, lb.LHQ, lb.LC, lb.LV, lb.Leigw, lb.Lpart,
                   lb.Lpart_elems, s));
    std::vector<double> th(J), g(K);
    ST(hipMemcpyAsync(th.data(), lb.Ltheta, sizeof(double) * J, hipMemcpyDeviceToHost, s));
    ST(hipMemcpyAsync(g.data(), lb.Lg, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    // the start's captured energy tr(F^T H_n F) = sum of the Ritz values,
    // against Jn/In of ||X||^2 (a random Jn-dimensional subspace's mean)
    double e = 0.0;
    for (double v : th) e += v;
    // squared Cholesky pivots of Rk^T Rk: their spread measures the rank
    double gmax = 0.0, gmin = HUGE_VAL;
    bool finite = true;
    for (double v : g) {
        finite = finite && std::isfinite(v);
        gmax = std::max(gmax, v);
        gmin = std::min(gmin, v);
    }
    const bool full_rank = finite && gmax > 0.0 && gmin >= 1e-12 * gmax;
    const bool better = std::isfinite(e) && e > (double)J / (double)In * nx2;
    return full_rank && better ? 1 : 0;
}

// Start of mode n (1 or 2) from slot k's buffers (0: p.Mg, p.eigw, p.theta,
// p.L[0]; 1: the second set) on stream s: HO-SVD (the leading eigenvectors
// of X_(n) X_(n)^T), or the learned start with HO-SVD as its fallback.
static int start_mode(Plan &p, int n, int k, const tk_opts *o, double *const *factors, tk_stats *st, int *noconv,
                      double nx2, hipStream_t s) {
    double *Mg = k == 0 ? p.Mg : p.Mg2;
    void *eigw = k == 0 ? p.eigw : (void *)p.eigw2;
    double *theta = k == 0 ? p.theta : p.theta2;
    if (o->init == TK_INIT_LEARNED) {
        const int ok = learned_mode(p, n, o, factors[n], nx2, s, p.L[k], Mg);
        if (ok < 0) return ok;
        if (ok == 1) {
            // the eigensolves of the sweeps start from this factor
            ST(eig_seed_block(p.Xblk[n], (int)p.I[n], p.J[n], factors[n], eigw, 0x1ea7ull + n, s));
            p.blk_ok[n] = true;
            ST(refresh_copies(p, n, factors[n], s));
            return TK_OK;
        }
        if (st) st->init_fallbacks += 1;
        return run_eig(p, n, Mg, factors[n], false, o, st, noconv, s, eigw, theta);  // H_n is in Mg
    }
    const int64_t dims[3] = {p.I[0], p.I[1], p.I[2]};
    const int sl = (n + 1) % 3;  // ordering whose slots are the mode-n slices
    ST(hosvd_gram(n, dims, p.ptr[n], p.lidx[n], p.lval64[n], p.ptr[sl], p.lidx[sl], p.lval64[sl], Mg, s));
    return run_eig(p, n, Mg, factors[n], false, o, st, noconv, s, eigw, theta);
}

// Starts of modes 2 and 3. Each comes from its own unfolding (Figure 1) and
// does not depend on the other; an eigensolve is a chain of small launches
// with host decisions between them, so mode 3's start runs on a second stream
// driven by a second host thread, with its own buffers, beside mode 2's on s.
static int start_pair(Plan &p, const tk_opts *o, double *const *factors, tk_stats *st, int *noconv, double nx2,
                      hipStream_t s) {
    int dev = 0;
    ST(hipGetDevice(&dev));
    hipStream_t s2 = nullptr;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    int r = TK_OK;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
        hipStreamWaitEvent(s2, e1, 0) != hipSuccess)
        r = TK_ERR_DEVICE;
    tk_stats st2{};
    int nc2 = 0, r2 = TK_OK;
    if (r == TK_OK) {
        auto second = [&] {
            if (hipSetDevice(dev) != hipSuccess) {
                r2 = TK_ERR_DEVICE;
                return;
            }
            r2 = start_mode(p, 2, 1, o, factors, st ? &st2 : nullptr, &nc2, nx2, s2);
        };
        std::thread th;
        try {
            th = std::thread(second);
        } catch (...) {  // no thread to be had: mode 3 after mode 2, from this thread
        }
        // mode 2 here; no early return while the other thread runs
        r = start_mode(p, 1, 0, o, factors, st, noconv, nx2, s);
        if (th.joinable())
            th.join();
        else
            second();
        if (r == TK_OK) r = r2;
        // the sweeps on s follow mode 3's work
        if (hipEventRecord(e2, s2) != hipSuccess || hipStreamWaitEvent(s, e2, 0) != hipSuccess)
            r = r ? r : TK_ERR_DEVICE;
        if (hipStreamSynchronize(s2) != hipSuccess) r = r ? r : TK_ERR_DEVICE;
    }
    if (st) {
        st->eig_iters += st2.eig_iters;
        st->eig_noconv += st2.eig_noconv;
        st->init_fallbacks += st2.init_fallbacks;
    }
    if (nc2) *noconv = 1;
    if (e2) (void)hipEventDestroy(e2);
    if (e1) (void)hipEventDestroy(e1);
    if (s2) (void)hipStreamDestroy(s2);
    return r;
}

// ------------------------------------------------------------------ random start
// Output number k of SplitMix64 seeded with `seed` (the state advances by the
// golden gamma before each output, then the variant-13 finaliser).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One workgroup per column r of the I x J start of mode n: entries uniform
// on [0, 1) from SplitMix64 output n * 2^40 + i * J + r, then the column
// divided by its norm (sum of squares in a fixed order).
__global__ void __launch_bounds__(256) k_random_start(double *F, int64_t I, int J, int n, uint64_t seed) {
    const int r = blockIdx.x;
    const uint64_t base = ((uint64_t)n << 40) + (uint64_t)r;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) {
        const double u = (double)(splitmix64_at(seed, base + (uint64_t)i * J) >> 11) * 0x1.0p-53;
        F[i * J + r] = u;
        acc += u * u;
    }
    __shared__ double ws[4];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double nrm = sqrt(ws[0] + ws[1] + ws[2] + ws[3]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) F[i * J + r] *= inv;
}

// Columns of F (I x J) divided by their norms, in place (the given start of SP).
__global__ void __launch_bounds__(256) k_normalise_cols(double *F, int64_t I, int J) {
    const int r = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) {
        const double v = F[i * J + r];
        acc += v * v;
    }
    __shared__ double ws[4];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double nrm = sqrt(ws[0] + ws[1] + ws[2] + ws[3]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) F[i * J + r] *= inv;
}

hipError_t random_start_fill(double *F, int64_t I, int J, int n, uint64_t seed, hipStream_t s) {
    k_random_start<<<J, 256, 0, s>>>(F, I, J, n, seed);
    TK_LAUNCHED();
    return hipSuccess;
}

static int random_mode(Plan &p, int n, double *F, uint64_t seed, hipStream_t s) {
    ST(random_start_fill(F, p.I[n], p.J[n], n, seed, s));
    ST(refresh_copies(p, n, F, s));
    return TK_OK;
}

static int init_factors(Plan &p, const tk_opts *o, double *const *factors, tk_stats *st, int *noconv, double nx2,
                        hipStream_t s) {
    if (o->init == TK_INIT_GIVEN) {
        for (int n = 1; n < 3; ++n) ST(refresh_copies(p, n, factors[n], s));
        return TK_OK;
    }
    if (o->init == TK_INIT_RANDOM) {
        for (int n = 1; n < 3; ++n)
            if (int r = random_mode(p, n, factors[n], o->seed, s)) return r;
        return TK_OK;
    }
    if (o->init == TK_INIT_LEARNED) {
        // mode 1 has no start in HOOI and MP (Figures 3 and 7), but its first
        // eigensolve can start from a learned block instead of a random one
        // (factors[0] is only scratch here; the first sweep overwrites it)
        const int ok = learned_mode(p, 0, o, factors[0], nx2, s, p.L[0], p.Mg);
        if (ok < 0) return ok;
        if (ok == 1) {
            ST(eig_seed_block(p.Xblk[0], (int)p.I[0], p.J[0], factors[0], p.eigw, 0x1ea7ull, s));
            p.blk_ok[0] = true;
        }
    }
    if (p.Mg2) return start_pair(p, o, factors, st, noconv, nx2, s);
    for (int n = 1; n < 3; ++n) {
        const int r = start_mode(p, n, 0, o, factors, st, noconv, nx2, s);
        if (r) return r;
    }
    return TK_OK;
}


// ------------------------------------------------------------------ HO-SVD core and fit
// G = [[X; A^T, B^T, C^T]] from an FP64 projection T(2) = X x_3 C^T (rows
// of J3) and its fit; the core goes to `core`.
static int hosvd_core_fit(Plan &p, const double *A, const double *B, const double *C, double *core, hipStream_t s,
                          double *fit) {
    ST((project<double, double, double>(p.ptr[2], p.lidx[2], p.lval64[2], C, p.I[2], p.J[2], p.J[2], p.J[2],
                                        p.nslots[2], p.nnz, p.Th, s)));
    ST(core_from_T2(p, p.Th, p.J[2], true, A, B, core, s));
    return finish_fit(p, core, s, fit);
}

// The HO-SVD fit of Figure 1 reported beside a decomposition. The HO-SVD
// factors of the modes in `todo` (those the start has not computed already)
// go to the caller's factor buffers as scratch and the core to `core`; the
// start and the sweeps overwrite both afterwards. Called after an HO-SVD
// start (todo = the modes it lacks) or before a random start (all three).
// The eigensolver blocks these solves leave are discarded, so the
// decomposition runs exactly as it would without the report.
static int report_hosvd_fit(Plan &p, const tk_opts *o, const bool todo[3], double *core, double *const *factors,
                            tk_stats *st, int *noconv, hipStream_t s) {
    const int64_t dims[3] = {p.I[0], p.I[1], p.I[2]};
    for (int n = 0; n < 3; ++n) {
        if (!todo[n]) continue;
        const int sl = (n + 1) % 3;
        ST(hosvd_gram(n, dims, p.ptr[n], p.lidx[n], p.lval64[n], p.ptr[sl], p.lidx[sl], p.lval64[sl], p.Mg, s));
        const int r = run_eig(p, n, p.Mg, factors[n], false, o, nullptr, noconv, s);
        if (r) return r;
        p.blk_ok[n] = false;
    }
    double fit = 0.0;
    if (int r = hosvd_core_fit(p, factors[0], factors[1], factors[2], core, s, &fit)) return r;
    if (st) st->hosvd_fit = fit;
    return TK_OK;
}


// Start of B and C with the HO-SVD fit report around it when asked for:
// before a random start (it needs all three HO-SVD factors), after an
// HO-SVD start (it needs only A's).
static int hosvd_report_around_start(Plan &p, const tk_opts *o, double *core, double *const *factors,
                                     tk_stats *st, int *noconv, double nx2, hipStream_t s) {
    if (p.hfit && o->init == TK_INIT_RANDOM) {
        const bool all[3] = {true, true, true};
        if (int r = report_hosvd_fit(p, o, all, core, factors, st, noconv, s)) return r;
    }
    if (int r = init_factors(p, o, factors, st, noconv, nx2, s)) return r;
    if (p.hfit && o->init == TK_INIT_HOSVD) {
        const bool a_only[3] = {true, false, false};
        if (int r = report_hosvd_fit(p, o, a_only, core, factors, st, noconv, s)) return r;
    }
    return TK_OK;
}

// MP and SP core from T(2)(C): the projection itself when it is FP64 or
// FP32, else (BF16 Grams) an FP32 projection with rows of ldc for it.
// The last projection of an MP / SP sweep, T(2)(C), which both the core and
// the next sweep's first Gram read. Mixed precision without split parts: one
// pass writes the core's FP32 copy (from the FP32 factor rows) and the BF16
// Gram copy rounded from it; *core_done then says that slice_core need not
// project again.
static hipError_t project_last(Plan &p, const double *C, hipStream_t s, Timer &tm, bool *core_done) {
    *core_done = false;
    const FibreList fl = fibres_of(p, 2, true);
    if (p.prec == PBF16 && !p.split && p.Fc &&
        project_dual_ok(p.Fc, p.I[2], p.ldc, p.Tcore, (const bf16 *)p.T[2], p.ldT[2], p.nslots[2], p.nnz, p.tune,
                        fl)) {
        TK_HIP(project_dual(p.ptr[2], p.lidx[2], p.lval32[2], p.Fc, p.I[2], p.ldc, p.J[2], p.nslots[2], p.nnz,
                            p.Tcore, (bf16 *)p.T[2], p.ldT[2], s, p.tune, tm.kernel(kProj, 2, P32), fl));
        *core_done = true;
        return hipSuccess;
    }
    return project_m(p, 2, C, p.T[2], p.prec, s, 0, tm.kernel(kProj, 2, p.prec));
}

static hipError_t slice_core(Plan &p, const double *A, const double *B, double *core, hipStream_t s, Timer &tm,
                             bool projected = false) {
    const void *T2c = p.T[2];
    if (p.prec == PBF16 && projected) {
        T2c = p.Tcore;
    } else if (p.prec == PBF16) {
        TK_HIP((project<float, float, float>(p.ptr[2], p.lidx[2], p.lval32[2], p.Fc, p.I[2], p.ldc, p.J[2], p.ldc,
                                             p.nslots[2], p.nnz, p.Tcore, s, p.tune, tm.kernel(kProj, 2, P32),
                                             fibres_of(p, 2, true))));
        T2c = p.Tcore;
    }
    tm.begin(kCore, -1, p.prec == P64 ? P64 : P32);
    TK_HIP(core_from_T2(p, T2c, p.prec == PBF16 ? p.ldc : p.ldT[2], p.prec == P64, A, B, core, s));
    tm.end();
    return hipSuccess;
}

}  // namespace tk

extern "C" int tucker_mp(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *factors,
                         double *fit_history, int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb,
                         void *stream) {
    if (X && X->order == 4)
        return order_n_mp(X, J, o, core, factors, fit_history, iters_done, stats, ws, wsb, stream);
    Plan p;
    int st = common_start(TK_ALGO_MP, X, J, o, core, factors, fit_history, iters_done, ws, wsb, p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    Timer tm(o, s);
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    if ((st = hosvd_report_around_start(p, o, core, factors, stats, &noconv, nx2, s))) return st;
    ST(hipStreamSynchronize(s));
    double t2 = now_ms();
    const int prec = p.prec;
    double *A = factors[0], *B = factors[1], *C = factors[2];
    double g2 = 0.0;
    // projections of the start: T(1)(B), T(2)(C)
    // (part of the start, not of a sweep's TTMc phase: untimed)
    ST(project_m(p, 1, B, p.T[1], prec, s));
    ST(project_m(p, 2, C, p.T[2], prec, s));
    double prev = 0.0;
    int t = 0;
    *iters_done = 0;
    for (t = 1; t <= o->max_iters; ++t) {
        // M1 (mode 0) from T(1) and T(2)
        tm.begin(kGram, 0, p.prec);
        ST(mp_gram(p, 0, 1, 2, s));
        tm.end();
        tm.begin(kEig, 0, P64);
        if ((st = run_eig(p, 0, p.Mg, A, true, o, stats, &noconv, s))) return st;
        tm.end();
        ST(project_m(p, 0, A, p.T[0], prec, s, 0, tm.kernel(kProj, 0, prec)));
        // M2 (mode 1) from T(0) and T(2)
        tm.begin(kGram, 1, p.prec);
        ST(mp_gram(p, 1, 0, 2, s));
        tm.end();
        tm.begin(kEig, 1, P64);
        if ((st = run_eig(p, 1, p.Mg, B, true, o, stats, &noconv, s))) return st;
        tm.end();
        ST(project_m(p, 1, B, p.T[1], prec, s, 0, tm.kernel(kProj, 1, prec)));
        // M3 (mode 2) from T(0) and T(1)
        tm.begin(kGram, 2, p.prec);
        ST(mp_gram(p, 2, 0, 1, s));
        tm.end();
        tm.begin(kEig, 2, P64);
        if ((st = run_eig(p, 2, p.Mg, C, true, o, stats, &noconv, s))) return st;
        tm.end();
        bool core_done = false;
        ST(project_last(p, C, s, tm, &core_done));
        // core from T(2)(C) (FP64 or FP32, never BF16)
        ST(slice_core(p, A, B, core, s, tm, core_done));
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
        tm.collect();
        fit_history[t - 1] = fit;
        *iters_done = t;
        if (o->tol > 0 && fit - prev < o->tol) break;
        prev = fit;
    }
    if (o->max_iters == 0) {
        // no sweep: A from the start factors, then the core
        tm.begin(kGram, 0, p.prec);
        ST(mp_gram(p, 0, 1, 2, s));
        tm.end();
        tm.begin(kEig, 0, P64);
        if ((st = run_eig(p, 0, p.Mg, A, true, o, stats, &noconv, s))) return st;
        tm.end();
        ST(slice_core(p, A, B, core, s, tm));
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
    }
    double t3 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->sweeps_ms = t3 - t2;
        tm.report(stats);
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

namespace tk {
// HOOI second stage, see the driver below for the index bookkeeping.
static hipError_t ttm(int M, int N, int K, int batch, const void *A, int64_t lda, const void *B, int64_t ldb,
                      int64_t sB, void *C, int64_t ldc, int64_t sC, int prec, int out_type, hipStream_t s) {
    GemmArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.batch = batch;
    g.A = A;
    g.lda = lda;
    g.a_trans = true;
    g.B = B;
    g.ldb = ldb;
    g.sB = sB;
    g.C = C;
    g.ldc = ldc;
    g.sC = sC;
    g.prec = prec;
    g.out_type = out_type;
    return gemm(g, s);
}
}  // namespace tk

extern "C" int tucker_hooi(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *factors,
                           double *fit_history, int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb,
                           void *stream) {
    if (X && X->order == 4)
        return order_n_hooi(X, J, o, core, factors, fit_history, iters_done, stats, ws, wsb, stream);
    Plan p;
    int st = common_start(TK_ALGO_HOOI, X, J, o, core, factors, fit_history, iters_done, ws, wsb, p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    Timer tm(o, s);
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    if ((st = hosvd_report_around_start(p, o, core, factors, stats, &noconv, nx2, s))) return st;
    ST(hipStreamSynchronize(s));
    double t2 = now_ms();
    double g2 = 0.0;
    const int prec = p.prec;
    const int64_t I0 = p.I[0], I1 = p.I[1], I2 = p.I[2];
    const int J0 = p.J[0], J1 = p.J[1], J2 = p.J[2];
    double *A = factors[0], *B = factors[1], *C = factors[2];
    // element types: FP64 mode all double; FP32 mode float; mixed: T(2)
    // in BF16 with BF16 MFMA for modes 1 and 2, T(0) in FP32 for mode 3
    const int tprec = prec;                  // T(2) storage
    const int kprec01 = prec == P64 ? P64 : prec;  // MFMA kind, modes 0/1
    const int yprec = prec == P64 ? P64 : P32;      // Y storage / Gram precision
    double prev = 0.0;
    *iters_done = 0;
    int maxit = o->max_iters > 0 ? o->max_iters : 0;
    for (int t = 1; t <= std::max(maxit, 1); ++t) {
        const bool last_only = (maxit == 0);
        ST(project_m(p, 2, C, p.T[2], tprec, s, 0, tm.kernel(kProj, 2, tprec)));
        const void *Bop = prec == P64 ? (const void *)B : (prec == P32 ? (const void *)p.F32[1] : (const void *)p.Fbf[1]);
        // mode 0: Y0[q][i0][r2] = sum_i1 B[i1][q] T2[i1][i0][r2]
        tm.begin(kTtmc, 0, kprec01);
        ST(ttm(J1, (int)(I0 * J2), (int)I1, 1, Bop, J1, p.T[2], I0 * J2, 0, p.Y, I0 * J2, 0, kprec01,
               yprec == P64 ? P64 : P32, s));
        tm.end();
        {
            GramTerm g;
            g.base = p.Y;
            g.s_row = J2;
            g.chunk_len = J2;
            g.nchunks = J1;
            g.s_chunk = I0 * J2;
            tm.begin(kGram, 0, yprec);
            ST(gram((int)I0, yprec, 1, &g, p.Mg, p.gram_scratch, s, p.tune));
            tm.end();
        }
        tm.begin(kEig, 0, P64);
        if ((st = run_eig(p, 0, p.Mg, A, true, o, stats, &noconv, s))) return st;
        tm.end();
        if (last_only) {
            // max_iters == 0: A only, then the core below
        }
        const void *Aop = prec == P64 ? (const void *)A : (prec == P32 ? (const void *)p.F32[0] : (const void *)p.Fbf[0]);
        // mode 1: Y1[i1][p][r2] = sum_i0 A[i0][p] T2[i1][i0][r2]
        if (!last_only) {
            tm.begin(kTtmc, 1, kprec01);
            ST(ttm(J0, J2, (int)I0, (int)I1, Aop, J0, p.T[2], J2, I0 * J2, p.Y, J2, (int64_t)J0 * J2, kprec01,
                   yprec == P64 ? P64 : P32, s));
            tm.end();
            GramTerm g;
            g.base = p.Y;
            g.s_row = (int64_t)J0 * J2;
            g.chunk_len = (int64_t)J0 * J2;
            g.nchunks = 1;
            g.s_chunk = 0;
            tm.begin(kGram, 1, yprec);
            ST(gram((int)I1, yprec, 1, &g, p.Mg, p.gram_scratch, s, p.tune));
            tm.end();
            tm.begin(kEig, 1, P64);
            if ((st = run_eig(p, 1, p.Mg, B, true, o, stats, &noconv, s))) return st;
            tm.end();
        }
        // mode 2 (and the core): T(0)(A) = [i2][i1][r0] in FP64 / FP32
        void *T0 = prec == PBF16 ? (void *)p.T0f : p.T[0];
        const int t0prec = prec == P64 ? P64 : P32;
        ST(project_m(p, 0, A, T0, t0prec, s, 0, tm.kernel(kProj, 0, t0prec)));
        const void *Bop2 = prec == P64 ? (const void *)B : (const void *)p.F32[1];
        // Y2[i2][q][r0] = sum_i1 B[i1][q] T0[i2][i1][r0]
        tm.begin(kTtmc, 2, t0prec);
        ST(ttm(J1, J0, (int)I1, (int)I2, Bop2, J1, T0, J0, I1 * J0, p.Y, J0, (int64_t)J1 * J0, t0prec,
               yprec == P64 ? P64 : P32, s));
        tm.end();
        if (!last_only) {
            GramTerm g;
            g.base = p.Y;
            g.s_row = (int64_t)J1 * J0;
            g.chunk_len = (int64_t)J1 * J0;
            g.nchunks = 1;
            g.s_chunk = 0;
            tm.begin(kGram, 2, yprec);
            ST(gram((int)I2, yprec, 1, &g, p.Mg, p.gram_scratch, s, p.tune));
            tm.end();
            tm.begin(kEig, 2, P64);
            if ((st = run_eig(p, 2, p.Mg, C, true, o, stats, &noconv, s))) return st;
            tm.end();
        }
        // core: G'[r][q][p] = sum_i2 C[i2][r] Y2[i2][q][p]; core[p][q][r] = G'[r][q][p]
        {
            GemmArgs h;
            h.M = J2;
            h.N = J1 * J0;
            h.K = (int)I2;
            h.batch = 1;
            h.A = C;
            h.lda = J2;
            h.a_trans = true;
            h.B = p.Y;
            h.ldb = (int64_t)J1 * J0;
            h.sB = 0;
            h.C = p.Gp;
            h.ldc = (int64_t)J1 * J0;
            h.sC = 0;
            h.prec = yprec == P64 ? P64 : 3;
            h.out_type = P64;
            int tiles = (int)(ceil_div(J2, 64) * ceil_div((int64_t)J1 * J0, 64));
            h.splitk = std::max(1, std::min(8, 256 / std::max(1, tiles)));
            h.split_scratch = p.core_split;
            ST(gemm(h, s));
            k_permute3<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)J0 * J1 * J2, 256), 65536), 256, 0, s>>>(
                p.Gp, core, J0, J1, J2, J2, J1, J0, 2, 1, 0);
            ST(hipGetLastError());
        }
        if (last_only) {
            double fit = 0;
            if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
            break;
        }
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
        tm.collect();
        fit_history[t - 1] = fit;
        *iters_done = t;
        if (o->tol > 0 && fit - prev < o->tol) break;
        prev = fit;
    }
    double t3 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->sweeps_ms = t3 - t2;
        tm.report(stats);
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}


namespace tk {
// SP's Gram of mode n from the single projection T(m): one term, or three
// for split-BF16 (hi hi^T + hi lo^T + lo hi^T).
static hipError_t sp_gram(Plan &p, int n, int m, hipStream_t s) {
    GramTerm g[3];
    int nt = 0;
    g[nt++] = term_of(p, m, n, p.T[m]);
    if (p.split) {
        GramTerm hl = term_of(p, m, n, p.T[m]);
        hl.base_b = p.Tlo[m];
        GramTerm lh = term_of(p, m, n, p.Tlo[m]);
        lh.base_b = p.T[m];
        g[nt++] = hl;
        g[nt++] = lh;
    }
    return gram((int)p.I[n], p.prec, nt, g, p.Mg, p.gram_scratch, s, p.tune);
}
}  // namespace tk

extern "C" int tucker_sp(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *factors,
                         double *fit_history, int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb,
                         void *stream) {
    Plan p;
    int st = common_start(TK_ALGO_SP, X, J, o, core, factors, fit_history, iters_done, ws, wsb, p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    Timer tm(o, s);
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    double *A = factors[0], *B = factors[1], *C = factors[2];
    // the start of C (Figure 5): random (the paper's), given, or HO-SVD;
    // columns of unit length. The HO-SVD fit report, when asked for, comes
    // before a random start and after an HO-SVD one.
    if (p.hfit && o->init == TK_INIT_RANDOM) {
        const bool all[3] = {true, true, true};
        if ((st = report_hosvd_fit(p, o, all, core, factors, stats, &noconv, s))) return st;
    }
    if (o->init == TK_INIT_RANDOM) {
        if ((st = random_mode(p, 2, C, o->seed, s))) return st;
    } else if (o->init == TK_INIT_GIVEN) {
        k_normalise_cols<<<p.J[2], 256, 0, s>>>(C, p.I[2], p.J[2]);
        ST(hipGetLastError());
        ST(refresh_copies(p, 2, C, s));
    } else {
        if ((st = start_mode(p, 2, 0, o, factors, stats, &noconv, nx2, s))) return st;
        if (p.hfit) {
            const bool ab[3] = {true, true, false};
            if ((st = report_hosvd_fit(p, o, ab, core, factors, stats, &noconv, s))) return st;
        }
    }
    ST(hipStreamSynchronize(s));
    double t2 = now_ms();
    const int prec = p.prec;
    ST(project_m(p, 2, C, p.T[2], prec, s));  // part of the start: untimed
    double prev_norm = 0.0, g2 = 0.0;
    *iters_done = 0;
    const int maxit = std::max(o->max_iters, 1);
    for (int t = 1; t <= maxit; ++t) {
        // M13 = sum_j X_:j: C C^T X_:j:^T: Gram of T(2) = X x_3 C^T on mode 1
        tm.begin(kGram, 0, p.prec);
        ST(sp_gram(p, 0, 2, s));
        tm.end();
        tm.begin(kEig, 0, P64);
        if ((st = run_eig(p, 0, p.Mg, A, true, o, stats, &noconv, s))) return st;
        tm.end();
        // M21 = sum_k X_::k^T A A^T X_::k: Gram of T(0) = X x_1 A^T on mode 2
        ST(project_m(p, 0, A, p.T[0], prec, s, 0, tm.kernel(kProj, 0, prec)));
        tm.begin(kGram, 1, p.prec);
        ST(sp_gram(p, 1, 0, s));
        tm.end();
        tm.begin(kEig, 1, P64);
        if ((st = run_eig(p, 1, p.Mg, B, true, o, stats, &noconv, s))) return st;
        tm.end();
        // M32 = sum_i X_i::^T B B^T X_i::: Gram of T(1) = X x_2 B^T on mode 3
        ST(project_m(p, 1, B, p.T[1], prec, s, 0, tm.kernel(kProj, 1, prec)));
        tm.begin(kGram, 2, p.prec);
        ST(sp_gram(p, 2, 1, s));
        tm.end();
        tm.begin(kEig, 2, P64);
        if ((st = run_eig(p, 2, p.Mg, C, true, o, stats, &noconv, s))) return st;
        tm.end();
        // T(2)(C): the core now, mode 1's Gram in the next sweep
        bool core_done = false;
        ST(project_last(p, C, s, tm, &core_done));
        ST(slice_core(p, A, B, core, s, tm, core_done));
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
        tm.collect();
        const double gn = std::sqrt(g2);
        // Delta_G(t) = 1 - ||G(t-1)|| / ||G(t)||, ||G(0)|| = 0 (Section 4.3)
        const double dG = gn > 0.0 ? 1.0 - prev_norm / gn : 0.0;
        if (o->max_iters > 0) {
            fit_history[t - 1] = fit;
            *iters_done = t;
        }
        if (o->max_iters == 0 || (o->tol > 0 && dG < o->tol)) break;
        prev_norm = gn;
    }
    double t3 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->sweeps_ms = t3 - t2;
        tm.report(stats);
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

extern "C" int tucker_hosvd(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *factors,
                            double *fit, tk_stats *stats, void *ws, size_t wsb, void *stream) {
    if (X && X->order == 4) return order_n_hosvd(X, J, o, core, factors, fit, stats, ws, wsb, stream);
    int st = check_coo(X, J);
    if (st) return st;
    if ((st = check_opts(o, X, TK_ALGO_HOSVD))) return st;
    if (!core || !factors || !factors[0] || !factors[1] || !factors[2] || !fit) return TK_ERR_ARG;
    if (X->nnz == 0) return TK_ERR_EMPTY;
    Plan p;
    plan_init(p, TK_ALGO_HOSVD, P64, X, J);
    p.eprec = o->precision == TK_MIXED_BF16X3 ? P32 : o->precision;
    tk_opts oh = *o;  // the starts below are HO-SVD ones whatever opt->init says
    oh.init = TK_INIT_HOSVD;
    o = &oh;
    Arena ar;
    carve(p, ar);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    carve(p, ar);
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    // Figure 1: every factor from its own unfolding Gram; modes 2 and 3
    // side by side (as the starts of HOOI and MP), then mode 1
    if ((st = start_pair(p, o, factors, stats, &noconv, nx2, s))) return st;
    if ((st = start_mode(p, 0, 0, o, factors, stats, &noconv, nx2, s))) return st;
    if ((st = hosvd_core_fit(p, factors[0], factors[1], factors[2], core, s, fit))) return st;
    double t2 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->hosvd_fit = *fit;
        // ||G||^2 = ||X||^2 (1 - (1 - fit)^2) by the fit identity
        const double r = 1.0 - *fit;
        stats->core_norm = std::sqrt(std::max(0.0, nx2 * (1.0 - r * r)));
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

extern "C" int tucker_fit(const tk_coo *X, const int32_t *J, const double *core, const double *const *factors,
                          double *fit, void *ws, size_t wsb, void *stream) {
    int st = check_coo(X, J);
    if (st) return st;
    if (!core || !factors || !factors[0] || !factors[1] || !factors[2] || !fit) return TK_ERR_ARG;
    if (X->nnz == 0) return TK_ERR_EMPTY;
    Plan p;
    plan_init(p, TK_ALGO_FIT, P64, X, J);
    Arena ar;
    carve(p, ar);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    carve(p, ar);
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    const int J0 = J[0], J1 = J[1], J2 = J[2];
    const int64_t nJ = (int64_t)J0 * J1 * J2;
    // Gx = X x_n A(n)^T via T(2)(C) and the two contractions of the MP core
    ST((project<double, double, double>(p.ptr[2], p.lidx[2], p.lval64[2], factors[2], p.I[2], J2, J2, J2,
                                        p.nslots[2], p.nnz, (double *)p.T[2], s)));
    ST(core_from_T2(p, p.T[2], J2, true, factors[0], factors[1], p.Gx, s));
    ST(dot(p.Gx, core, nJ, p.partials, p.scal + 3, s));
    // P_n = A(n)^T A(n)
    for (int n = 0; n < 3; ++n) {
        GemmArgs g;
        g.M = J[n];
        g.N = J[n];
        g.K = (int)p.I[n];
        g.batch = 1;
        g.A = factors[n];
        g.lda = J[n];
        g.a_trans = true;
        g.B = factors[n];
        g.ldb = J[n];
        g.sB = 0;
        g.C = p.Pn[n];
        g.ldc = J[n];
        g.sC = 0;
        g.prec = P64;
        g.out_type = P64;
        ST(gemm(g, s));
    }
    // W = G x_1 P0 x_2 P1 x_3 P2 (each P symmetric)
    {
        GemmArgs g;  // W1[p'][(q,r)] = sum_p P0[p][p'] G[p][(q,r)]
        g.M = J0;
        g.N = J1 * J2;
        g.K = J0;
        g.batch = 1;
        g.A = p.Pn[0];
        g.lda = J0;
        g.a_trans = true;
        g.B = core;
        g.ldb = (int64_t)J1 * J2;
        g.sB = 0;
        g.C = p.W1;
        g.ldc = (int64_t)J1 * J2;
        g.sC = 0;
        g.prec = P64;
        g.out_type = P64;
        ST(gemm(g, s));
        GemmArgs h;  // W2[p][q'][r] = sum_q P1[q][q'] W1[p][q][r]
        h.M = J1;
        h.N = J2;
        h.K = J1;
        h.batch = J0;
        h.A = p.Pn[1];
        h.lda = J1;
        h.a_trans = true;
        h.B = p.W1;
        h.ldb = J2;
        h.sB = (int64_t)J1 * J2;
        h.C = p.W2;
        h.ldc = J2;
        h.sC = (int64_t)J1 * J2;
        h.prec = P64;
        h.out_type = P64;
        ST(gemm(h, s));
        GemmArgs k;  // W3[(p,q)][r'] = sum_r W2[(p,q)][r] P2[r][r']
        k.M = J0 * J1;
        k.N = J2;
        k.K = J2;
        k.batch = 1;
        k.A = p.W2;
        k.lda = J2;
        k.a_trans = false;
        k.B = p.Pn[2];
        k.ldb = J2;
        k.sB = 0;
        k.C = p.W1;
        k.ldc = J2;
        k.sC = 0;
        k.prec = P64;
        k.out_type = P64;
        ST(gemm(k, s));
    }
    ST(dot(core, p.W1, nJ, p.partials, p.scal + 4, s));
    k_fit<<<1, 1, 0, s>>>(p.scal + 0, nullptr, p.scal + 3, p.scal + 4, p.scal + 2, 1);
    ST(hipGetLastError());
    ST(hipMemcpyAsync(fit, p.scal + 2, 8, hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

// ------------------------------------------------------------------ step-level entry points
#include "../../include/tucker_steps.h"

namespace tk {
static void eig_step_layout(Arena &ar, int n, int J, double **Mc, double **Xb, void **w) {
    const int b = eig_block_width(n, J);
    *Mc = ar.take<double>((int64_t)n * n);
    *Xb = ar.take<double>((int64_t)n * b);
    *w = ar.take<char>((int64_t)eig_work_bytes(n, b));
}
}  // namespace tk

extern "C" int tucker_step_lead_eig_workspace(int32_t n, int32_t J, size_t *bytes) {
    if (!bytes || n < 1 || J < 1 || J > n || J > kMaxJ) return TK_ERR_ARG;
    Arena ar;
    double *a, *b;
    void *c;
    eig_step_layout(ar, n, J, &a, &b, &c);
    *bytes = ar.used + 256;
    return TK_OK;
}

extern "C" int tucker_step_lead_eig(const double *M, int32_t n, int32_t J, double *F, double *theta, int32_t *matvecs,
                                    double tol, int32_t warm, void *ws, size_t wsb, void *stream) {
    if (!M || !F || !theta || !matvecs || n < 1 || J < 1 || J > n || J > kMaxJ || !(tol >= 0.0)) return TK_ERR_ARG;
    Arena ar;
    double *Mc, *Xb;
    void *w;
    eig_step_layout(ar, n, J, &Mc, &Xb, &w);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    eig_step_layout(ar, n, J, &Mc, &Xb, &w);
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    ST(hipMemcpyAsync(Mc, M, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
    EigOpts eo;
    eo.tol = tol;
    eo.warm = warm != 0;
    int it = 0, nc = 0;
    ST(lead_eig(Mc, n, J, Xb, F, theta, w, eo, &it, &nc, s));
    ST(hipStreamSynchronize(s));
    *matvecs = it;
    return nc ? TK_WARN_NOCONV : TK_OK;
}

// ------------------------------------------------------------------ learned start
#include "../../include/tucker_learn.h"

extern "C" int tucker_learn_param_count(void) { return learn_param_count(); }

namespace tk {
static void sketch_plan(Plan &p, const tk_coo *X) {
    const int32_t ones[3] = {1, 1, 1};
    plan_init(p, TK_ALGO_FIT, P32, X, ones);
}
}  // namespace tk

extern "C" int tucker_learn_sketch_workspace(const tk_coo *X, size_t *bytes) {
    const int32_t ones[3] = {1, 1, 1};
    if (!bytes) return TK_ERR_ARG;
    int st = check_coo(X, ones);
    if (st) return st;
    Plan p;
    sketch_plan(p, X);
    Arena ar;
    carve(p, ar);
    *bytes = ar.used + 256;
    return TK_OK;
}

extern "C" int tucker_learn_sketch(const tk_coo *X, int32_t mode, uint64_t seed, float *F, float *rho, void *ws,
                                   size_t wsb, void *stream) {
    const int32_t ones[3] = {1, 1, 1};
    int st = check_coo(X, ones);
    if (st) return st;
    if (mode < 0 || mode > 2 || !F || !rho) return TK_ERR_ARG;
    if (X->nnz == 0) return TK_ERR_EMPTY;
    Plan p;
    sketch_plan(p, X);
    Arena ar;
    carve(p, ar);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    carve(p, ar);
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    const int sl = (mode + 1) % 3;
    ST(learn_sketch<float>(p.ptr[sl], p.lidx[sl], p.lval32[sl], p.I[mode], p.I[lo_of(sl)], mode, seed, F, rho, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

extern "C" int tucker_learn_forward(const float *F, const float *rho, int64_t rows, const float *params, float *R,
                                    float *Z1, void *stream) {
    if (rows < 0 || (rows > 0 && (!F || !rho || !params || !R))) return TK_ERR_ARG;
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    ST(learn_forward(F, rho, rows, params, R, Z1, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

extern "C" int tucker_learn_backward_workspace(int64_t rows, size_t *bytes) {
    if (!bytes || rows < 0) return TK_ERR_ARG;
    *bytes = learn_backward_scratch(rows) + 256;
    return TK_OK;
}

extern "C" int tucker_learn_backward(const float *F, const float *rho, int64_t rows, const float *params,
                                     const float *Z1, const float *dR, float *grad, void *ws, size_t wsb,
                                     void *stream) {
    if (rows < 0 || !grad || (rows > 0 && (!F || !rho || !params || !Z1 || !dR))) return TK_ERR_ARG;
    if (!ws || wsb < learn_backward_scratch(rows) + 256) return TK_ERR_WORKSPACE;
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    float *part = reinterpret_cast<float *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ST(learn_backward(F, rho, rows, params, Z1, dR, grad, part, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

extern "C" int tucker_learn_test_width(int32_t J) { return J >= 1 && J <= 128 ? learn_test_width(J) : TK_ERR_ARG; }

extern "C" int tucker_learn_align_workspace(int64_t rows, int32_t K, int32_t J, size_t *bytes) {
    if (!bytes || rows < 1 || K < 1 || K > 128 || J < 1 || J > 128 || J > rows) return TK_ERR_ARG;
    *bytes = sizeof(double) * (size_t)learn_align_scratch_doubles(rows, K, J) + 256;
    return TK_OK;
}

extern "C" int tucker_learn_align(const float *R, int64_t rows, int32_t K, const double *A, int32_t J, double shift,
                                  double *loss, float *dR, void *ws, size_t wsb, void *stream) {
    if (!R || !A || !loss || rows < 1 || K < 1 || K > 128 || J < 1 || J > 128 || J > rows || !(shift >= 0.0))
        return TK_ERR_ARG;
    if (rows >= (int64_t)INT32_MAX) return TK_ERR_ARG;
    if (!ws || wsb < sizeof(double) * (size_t)learn_align_scratch_doubles(rows, K, J) + 256)
        return TK_ERR_WORKSPACE;
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    double *scr = reinterpret_cast<double *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    double *loss_dev = scr;  // first 8 doubles, the rest for the computation
    ST(learn_align(R, rows, K, A, J, shift, loss_dev, dR, scr + 8, s));
    ST(hipMemcpyAsync(loss, loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

extern "C" int tucker_learn_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                                 float beta1, float beta2, float eps, int32_t step, void *stream) {
    if (!params || !grad || !m || !v || n < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return TK_ERR_ARG;
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    ST(learn_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step, s));
    ST(hipStreamSynchronize(s));
    return TK_OK;
}

// ------------------------------------------------------------------ many tensors
#include "../../include/tucker_batch.h"

#include <atomic>
#include <thread>

extern "C" int tucker_batched_workspace_bytes(int32_t algo, int32_t count, const tk_coo *X, const int32_t *core_dims,
                                              const tk_opts *opt, const tk_tune *tunes, size_t *bytes) {
    if (!bytes || !X || !core_dims || !opt || count < 1) return TK_ERR_ARG;
    if (algo != TK_ALGO_HOOI && algo != TK_ALGO_MP) return TK_ERR_ARG;
    if (opt->trace) return TK_ERR_ARG;  // one trace cannot serve concurrent decompositions
    size_t best = 0;
    for (int32_t t = 0; t < count; ++t) {
        size_t b = 0;
        tk_opts ot = *opt;
        if (tunes) ot.tune = tunes + t;
        int st = tucker_workspace_bytes(algo, X + t, core_dims + 3 * t, &ot, &b);
        if (st) return st;
        best = std::max(best, b);
    }
    *bytes = best;
    return TK_OK;
}

extern "C" int tucker_batched(int32_t algo, int32_t count, const tk_coo *X, const int32_t *core_dims,
                              const tk_opts *opt, double *const *cores, double *const *factors, double *fit_history,
                              int32_t *iters_done, int32_t *status, tk_stats *stats, const tk_tune *tunes,
                              int32_t nstreams, void *const *workspaces, size_t workspace_bytes,
                              void *const *streams) {
    if (!X || !core_dims || !opt || !cores || !factors || !iters_done || !status || !workspaces || !streams)
        return TK_ERR_ARG;
    if (count < 1 || nstreams < 1 || nstreams > 64) return TK_ERR_ARG;
    if (algo != TK_ALGO_HOOI && algo != TK_ALGO_MP) return TK_ERR_ARG;
    if (opt->max_iters > 0 && !fit_history) return TK_ERR_ARG;
    size_t need = 0;
    int st = tucker_batched_workspace_bytes(algo, count, X, core_dims, opt, tunes, &need);
    if (st) return st;
    for (int32_t s = 0; s < nstreams; ++s)
        if (!workspaces[s] || workspace_bytes < need) return TK_ERR_WORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TK_ERR_DEVICE;
    std::atomic<int32_t> next{0};
    const int64_t hist = opt->max_iters > 0 ? opt->max_iters : 0;
    auto worker = [&](int32_t s) {
        if (hipSetDevice(dev) != hipSuccess) {
            for (int32_t t; (t = next.fetch_add(1)) < count;) status[t] = TK_ERR_DEVICE;
            return;
        }
        for (int32_t t; (t = next.fetch_add(1)) < count;) {
            double *const *f = factors + 3 * (int64_t)t;
            double *h = hist ? fit_history + hist * t : nullptr;
            tk_stats *stt = stats ? stats + t : nullptr;
            tk_opts ot = *opt;
            if (tunes) ot.tune = tunes + t;
            status[t] = algo == TK_ALGO_MP
                            ? tucker_mp(X + t, core_dims + 3 * t, &ot, cores[t], f, h, iters_done + t, stt,
                                        workspaces[s], workspace_bytes, streams[s])
                            : tucker_hooi(X + t, core_dims + 3 * t, &ot, cores[t], f, h, iters_done + t, stt,
                                          workspaces[s], workspace_bytes, streams[s]);
        }
    };
    std::vector<std::thread> pool;
    for (int32_t s = 1; s < nstreams; ++s) pool.emplace_back(worker, s);
    worker(0);
    for (auto &th : pool) th.join();
    int worst = TK_OK;
    for (int32_t t = 0; t < count; ++t) {
        if (status[t] < 0) return status[t];
        if (status[t] > 0) worst = status[t];
    }
    return worst;
}

extern "C" int tucker_mp_streamed_workspace(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                                            size_t slab_bytes, size_t *bytes) {
    return tk::mp_streamed_workspace(X, core_dims, opt, slab_bytes, bytes);
}

extern "C" int tucker_mp_streamed(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt, size_t slab_bytes,
                                  double *core, double *const *factors, double *fit_history, int32_t *iters_done,
                                  tk_stats *stats, void *workspace, size_t workspace_bytes, void *stream) {
    tk::g_err_clear();
    return tk::mp_streamed(X, core_dims, opt, slab_bytes, core, factors, fit_history, iters_done, stats, workspace,
                           workspace_bytes, stream);
}

extern "C" int tucker_mp_implicit_workspace(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt,
                                            size_t *bytes) {
    return tk::mp_implicit_workspace(X, core_dims, opt, bytes);
}

extern "C" int tucker_mp_implicit(const tk_coo *X, const int32_t *core_dims, const tk_opts *opt, double *core,
                                  double *const *factors, double *fit_history, int32_t *iters_done, tk_stats *stats,
                                  void *workspace, size_t workspace_bytes, void *stream) {
    tk::g_err_clear();
    return tk::mp_implicit(X, core_dims, opt, core, factors, fit_history, iters_done, stats, workspace,
                           workspace_bytes, stream);
}
