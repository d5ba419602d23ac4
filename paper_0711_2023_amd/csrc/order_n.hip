// Tucker decompositions of sparse tensors of order four: HO-SVD (Section 4.1,
// Figure 2), HOOI (Section 4.2, Figure 4) and Multislice Projection
// (Section 4.4, Figure 8), reached through tucker_hosvd, tucker_hooi and
// tucker_mp when tk_coo.order is 4.
//
// The kernels are those of the third-order path (fibre orderings, fibre
// projection, Gram, MFMA products, eigensolver); what changes is the
// bookkeeping of a fourth index:
// * the ordering of leaf mode m has its slots keyed by the other modes in
//   the order (m-1, m-2, m-3) mod 4, most significant first; a projection
//   T(m) = X x_m A(m)^T is stored dense in that order with the J_m columns
//   (padded to whole 16-byte rows) fastest;
// * MP's matrix of mode n is the sum over the three other modes m of the
//   slice products X_s A(m) A(m)^T X_s^T (Figure 8), which regroup into the
//   Gram T(m)_(n) T(m)_(n)^T of the unfolding of T(m) along n: one Gram
//   kernel call with three terms whose strides follow n's position among
//   T(m)'s keys; each sweep projects every mode once (Gauss-Seidel order);
// * HOOI's Z = X projected on every factor but A(n) (Figure 4) is one fibre
//   projection followed by two dense contractions (batched MFMA products);
// * the core is T(4) contracted with A(1), A(2), A(3), innermost key first,
//   then permuted to row-major J1 x J2 x J3 x J4; the fit follows from
//   ||G||^2 (identity of Section 3).
// The start of HOOI and MP takes A(2..4) from X_(n) X_(n)^T (MP's pseudo
// HO-SVD matrices are three times these, with the same eigenvectors).
#include "../../include/tucker.h"
#include "common.h"
#include "guards.h"
#include "timer.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace tk {

namespace {

constexpr int kMaxJn = 128;
constexpr int64_t kMaxStartDim = 8192;
// Start Grams from the dense unfolding: X_(n) X_(n)^T costs about
// nnz * (nnz / cells) * I_n products when walked sparsely, and 2 I_n cells
// flops on FP64 MFMA when X_(n) is held dense; the dense form wins from a
// density of about one cell in sixteen (measured at 100^4 with 10 % of the
// cells: 4.2 ms per sparse Gram), and is taken there if the tensor has at
// most kDenseStartCells cells (2 GiB of doubles).
constexpr int64_t kDenseStartCells = int64_t(1) << 28;
constexpr int64_t kDenseStartInv = 16;

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int elem_of(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// A dense tensor in a contraction chain: sizes of its axes (the last one is
// the column axis, stored with row stride ld) and the mode of each axis.
struct Shape {
    int r = 0;  // axes
    int64_t size[kMaxOrder] = {};
    int mode[kMaxOrder] = {};
    int ld = 0;
    int64_t rows_between(int a, int b) const {  // product of sizes of axes a..b-1
        int64_t p = 1;
        for (int k = a; k < b; ++k) p *= size[k];
        return p;
    }
    int64_t elems() const { return rows_between(0, r - 1) * ld; }
};

struct PlanN {
    int N = 4, algo = 0, prec = P64, eprec = P64, init = TK_INIT_HOSVD;
    Tune tune;
    int64_t I[kMaxOrder] = {}, nnz = 0;
    int J[kMaxOrder] = {};
    int key[kMaxOrder][kMaxOrder - 1] = {};
    int64_t nslots[kMaxOrder] = {};
    int ld[kMaxOrder] = {};
    int b[kMaxOrder] = {};
    int32_t *flags = nullptr, *nu = nullptr;
    double *scal = nullptr, *partials = nullptr;
    int32_t *perm = nullptr, *tmp = nullptr, *heads = nullptr, *pos = nullptr, *counts = nullptr, *cursor = nullptr,
            *scan = nullptr, *merged = nullptr;
    int32_t *cidx[kMaxOrder] = {};
    double *cval = nullptr;
    int32_t *ptr[kMaxOrder] = {}, *lidx[kMaxOrder] = {}, *fib[kMaxOrder] = {}, *fptr[kMaxOrder] = {};
    double *lval64[kMaxOrder] = {};
    float *lval32[kMaxOrder] = {};
    int64_t nfib[kMaxOrder] = {};
    void *T[kMaxOrder] = {};
    float *Tcore = nullptr, *Fc = nullptr;
    int ldc = 0;
    void *Fp[kMaxOrder] = {};
    float *F32[kMaxOrder] = {};
    bf16 *Fbf[kMaxOrder] = {};  // BF16 factor copies (rows of J), MFMA operands
    void *Y[2] = {nullptr, nullptr};
    int64_t ybytes = 0;
    double *Mg = nullptr, *theta = nullptr, *Xblk[kMaxOrder] = {}, *core_split = nullptr;
    void *gram_scratch = nullptr, *eigw = nullptr;
    double *dense = nullptr;  // dense unfolding for the start Grams (null: sparse form)
    int64_t core_split_elems = 0;
    bool blk_ok[kMaxOrder] = {};
    int sweep_solves[kMaxOrder] = {};
};

// The shape of the projection T(m): its key axes, then J_m columns of stride ld.
Shape proj_shape_of(const PlanN &p, int m, int ld) {
    Shape sh;
    sh.r = p.N;
    for (int k = 0; k < p.N - 1; ++k) {
        sh.mode[k] = p.key[m][k];
        sh.size[k] = p.I[p.key[m][k]];
    }
    sh.mode[p.N - 1] = m;
    sh.size[p.N - 1] = p.J[m];
    sh.ld = ld;
    return sh;
}

// The largest tensor a contraction chain from T(m) produces (elements), for
// the chain that contracts every key except `keep` (-1: all).
int64_t chain_max(const PlanN &p, int m, int ld, int keep) {
    Shape sh = proj_shape_of(p, m, ld);
    int64_t best = 0;
    for (int a = p.N - 2; a >= 0; --a) {
        if (sh.mode[a] == keep) continue;
        sh.size[a] = p.J[sh.mode[a]];
        best = std::max(best, sh.elems());
    }
    return best;
}

void plan_init(PlanN &p, int algo, int prec, const tk_coo *X, const int32_t *J, int init, const tk_tune *tune) {
    p.N = X->order;
    p.algo = algo;
    p.prec = prec;
    p.eprec = prec;
    p.init = init;
    if (tune) {
        if (tune->proj_elems) p.tune.proj_elems = tune->proj_elems;
        if (tune->proj_min_blocks) p.tune.proj_min_blocks = tune->proj_min_blocks;
        if (tune->gram_items) p.tune.gram_items = tune->gram_items;
        if (tune->gram_min_stages) p.tune.gram_min_stages = tune->gram_min_stages;
    }
    p.nnz = X->nnz;
    for (int n = 0; n < p.N; ++n) {
        p.I[n] = X->dims[n];
        p.J[n] = J[n];
    }
    for (int m = 0; m < p.N; ++m) {
        p.nslots[m] = 1;
        for (int k = 0; k < p.N - 1; ++k) {
            p.key[m][k] = ((m - 1 - k) % p.N + p.N) % p.N;
            p.nslots[m] *= p.I[p.key[m][k]];
        }
        // 16-byte rows of the projection's element type
        const int v = 16 / elem_of(prec);
        p.ld[m] = (int)ceil_div(p.J[m], v) * v;
    }
}

// Whether the HO-SVD start Grams take the dense form (see kDenseStartCells).
bool dense_start(const PlanN &p) {
    if (p.init != TK_INIT_HOSVD) return false;
    int64_t cells = 1;
    for (int k = 0; k < p.N; ++k) {
        cells *= p.I[k];
        if (cells > kDenseStartCells) return false;
    }
    return p.nnz * kDenseStartInv >= cells;
}

void carve(PlanN &p, Arena &ar) {
    const int N = p.N;
    const int64_t nnz = p.nnz > 0 ? p.nnz : 1;
    int64_t maxslots = 1, maxI = 1;
    for (int m = 0; m < N; ++m) {
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
    p.merged = ar.take<int32_t>(nnz);
    p.counts = ar.take<int32_t>(maxslots);
    p.cursor = ar.take<int32_t>(maxslots + 1);
    p.scan = ar.take<int32_t>(std::max(scan_scratch_ints(maxslots), scan_scratch_ints(nnz + 1)));
    for (int n = 0; n < N; ++n) p.cidx[n] = ar.take<int32_t>(nnz);
    p.cval = ar.take<double>(nnz);
    for (int m = 0; m < N; ++m) {
        p.ptr[m] = ar.take<int32_t>(p.nslots[m] + 1);
        p.lidx[m] = ar.take<int32_t>(nnz);
        p.lval64[m] = ar.take<double>(nnz);
        p.lval32[m] = p.prec != P64 ? ar.take<float>(nnz) : nullptr;
    }
    const int es = elem_of(p.prec);
    if (p.algo == TK_ALGO_MP) {
        for (int m = 0; m < N; ++m) {
            const int64_t cap = std::min(p.nslots[m], nnz);
            p.fib[m] = ar.take<int32_t>(cap);
            p.fptr[m] = ar.take<int32_t>(cap + 1);
            p.T[m] = ar.take<char>(p.nslots[m] * p.ld[m] * (int64_t)es);
        }
    } else if (p.algo == TK_ALGO_HOOI) {
        int64_t tmax = 0;
        for (int m = 0; m < N; ++m) tmax = std::max(tmax, p.nslots[m] * p.ld[m]);
        p.T[0] = ar.take<char>(tmax * (int64_t)es);
    } else {  // HO-SVD: FP64 projection of the last mode for the core
        p.T[0] = ar.take<char>(p.nslots[N - 1] * p.ld[N - 1] * (int64_t)es);
    }
    // core projection (FP32 rows of ldc) for mixed MP
    if (p.algo == TK_ALGO_MP && p.prec == PBF16) {
        p.ldc = (int)ceil_div(p.J[N - 1], 4) * 4;
        p.Tcore = ar.take<float>(p.nslots[N - 1] * p.ldc);
        p.Fc = ar.take<float>(p.I[N - 1] * p.ldc);
    }
    // contraction chains: the core's (from T(N-1)) and HOOI's (from T(m) keeping n)
    const int ldcore = p.algo == TK_ALGO_MP && p.prec == PBF16 ? p.ldc : p.ld[N - 1];
    int64_t ymax = chain_max(p, N - 1, ldcore, -1);
    if (p.algo == TK_ALGO_HOOI)
        for (int n = 0; n < N; ++n) {
            const int m = n == N - 1 ? N - 2 : N - 1;
            ymax = std::max(ymax, chain_max(p, m, p.ld[m], n));
        }
    p.ybytes = ymax * 8;
    p.Y[0] = ar.take<char>(p.ybytes);
    p.Y[1] = ar.take<char>(p.ybytes);
    p.Mg = ar.take<double>(maxI * maxI);
    size_t gs = 0;
    for (int n = 0; n < N && p.algo != TK_ALGO_HOSVD; ++n) {
        int64_t K[kGramMaxTerms];
        if (p.algo == TK_ALGO_MP) {
            int t = 0;
            for (int m = 0; m < N; ++m)
                if (m != n) K[t++] = p.nslots[m] / p.I[n] * p.ld[m];
            gs = std::max(gs, gram_scratch_bytes((int)p.I[n], p.prec, t, K, p.tune));
        } else {
            const int m = n == N - 1 ? N - 2 : N - 1;
            int64_t k = p.ld[m];
            for (int j = 0; j < N; ++j)
                if (j != n && j != m) k *= p.J[j];
            K[0] = k;
            gs = std::max(gs, gram_scratch_bytes((int)p.I[n], p.prec == P64 ? P64 : P32, 1, K, p.tune));
        }
    }
    p.dense = nullptr;
    if (dense_start(p)) {
        int64_t cells = 1;
        for (int k = 0; k < N; ++k) cells *= p.I[k];
        p.dense = ar.take<double>(cells);
        for (int n = 0; n < N; ++n) {
            const int64_t K = cells / p.I[n];
            gs = std::max(gs, gram_scratch_bytes((int)p.I[n], P64, 1, &K, p.tune));
        }
    }
    p.gram_scratch = ar.take<char>((int64_t)gs);
    size_t ew = 0;
    int bmax = 1;
    for (int n = 0; n < N; ++n) {
        p.b[n] = eig_block_width((int)p.I[n], p.J[n]);
        bmax = std::max(bmax, p.b[n]);
        p.Xblk[n] = ar.take<double>(p.I[n] * p.b[n]);
        ew = std::max(ew, eig_work_bytes((int)p.I[n], p.b[n]));
    }
    p.eigw = ar.take<char>((int64_t)ew);
    p.theta = ar.take<double>(std::max<int64_t>(bmax, maxI));
    for (int n = 0; n < N; ++n) {
        p.Fp[n] = ar.take<char>(p.I[n] * p.ld[n] * (int64_t)(p.prec == P64 ? 8 : (p.prec == P32 ? 4 : 2)));
        p.F32[n] = p.prec != P64 ? ar.take<float>(p.I[n] * p.J[n]) : nullptr;
        p.Fbf[n] = p.prec == PBF16 ? ar.take<bf16>(p.I[n] * p.J[n]) : nullptr;
    }
    int64_t nJ = 1;
    for (int n = 0; n < N; ++n) nJ *= p.J[n];
    p.core_split_elems = 8 * nJ;
    p.core_split = ar.take<double>(p.core_split_elems);
}

int check(int algo, const tk_coo *X, const int32_t *J, const tk_opts *o) {
    if (!X || !J || !X->dims || X->order != 4) return TK_ERR_ARG;
    if (X->nnz < 0 || X->nnz >= (int64_t)INT32_MAX - 1) return TK_ERR_ARG;
    if (X->nnz > 0) {
        for (int n = 0; n < 4; ++n)
            if (!X->idx[n]) return TK_ERR_ARG;
        if (!X->vals) return TK_ERR_ARG;
    }
    for (int n = 0; n < 4; ++n) {
        if (X->dims[n] < 1 || X->dims[n] >= INT32_MAX) return TK_ERR_ARG;
        if (J[n] < 1 || J[n] > X->dims[n] || J[n] > kMaxJn) return TK_ERR_ARG;
    }
    for (int m = 0; m < 4; ++m) {  // slots of each ordering: 32-bit
        int64_t s = 1;
        for (int n = 0; n < 4; ++n)
            if (n != m) s *= X->dims[n];
        if (s >= (int64_t)INT32_MAX) return TK_ERR_ARG;
    }
    if (!o) return TK_ERR_ARG;
    if (o->precision != TK_FP64 && o->precision != TK_FP32 && o->precision != TK_MIXED_BF16) return TK_ERR_ARG;
    if (o->eig_max_iters < 1 || !(o->eig_tol >= 0.0)) return TK_ERR_ARG;
    if (o->tune) {
        const tk_tune *t = o->tune;
        auto in = [](int32_t v, int32_t lo, int32_t hi) { return v == 0 || (v >= lo && v <= hi); };
        if (!in(t->proj_elems, 1024, 65536) || !in(t->proj_min_blocks, 64, 16384) ||
            !in(t->gram_items, 64, 16384) || !in(t->gram_min_stages, 1, 64))
            return TK_ERR_ARG;
    }
    if (algo == TK_ALGO_HOSVD) {
        for (int n = 0; n < 4; ++n)
            if (X->dims[n] > kMaxStartDim) return TK_ERR_ARG;
        return TK_OK;
    }
    if (o->init != TK_INIT_HOSVD && o->init != TK_INIT_GIVEN) return TK_ERR_ARG;
    if (o->hosvd_fit) return TK_ERR_ARG;
    if (o->max_iters < 1 || std::isnan(o->tol)) return TK_ERR_ARG;
    if (o->init == TK_INIT_HOSVD)
        for (int n = 1; n < 4; ++n)
            if (X->dims[n] > kMaxStartDim) return TK_ERR_ARG;
    return TK_OK;
}

#define STN(call)                         \
    do {                                  \
        hipError_t e_ = (call);           \
        if (e_ != hipSuccess) {           \
            set_hip_error(e_, #call);     \
            return TK_ERR_DEVICE;         \
        }                                 \
    } while (0)

// Validation, duplicate summing, the four orderings, ||X||^2, fibre lists.
int prep(PlanN &p, const tk_coo *X, hipStream_t s, int64_t *nu_out, double *nx2_out) {
    const int N = p.N;
    CoordsN c;
    c.n = N;
    for (int k = 0; k < N; ++k) {
        c.i[k] = X->idx[k];
        c.dim[k] = (int32_t)p.I[k];
    }
    STN(validate_n(c, X->vals, p.nnz, p.flags, s));
    int32_t flags = 0;
    STN(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    STN(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    OrderScratch sc{p.counts, p.cursor, p.tmp, p.scan};
    // full-coordinate order for the duplicates: the ordering of the last leaf
    {
        const int m = N - 1;
        const int *k = p.key[m];
        STN(merge_keys(X->idx[k[0]], X->idx[k[1]], p.nnz, (int32_t)p.I[k[1]], p.merged, s));
        STN(build_order_keys(p.merged, X->idx[k[2]], X->idx[m], p.nnz, (int32_t)p.I[k[2]], p.nslots[m], p.ptr[m],
                             p.perm, sc, p.flags, s));
    }
    STN(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    STN(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    CoordsOut out;
    for (int k = 0; k < N; ++k) out.i[k] = p.cidx[k];
    STN(dedup_n(c, X->vals, p.nnz, p.perm, p.heads, p.pos, p.scan, out, p.cval, p.nu, s));
    int32_t nu = 0;
    STN(hipMemcpyAsync(&nu, p.nu, 4, hipMemcpyDeviceToHost, s));
    STN(hipStreamSynchronize(s));
    STN(sumsq(p.cval, nu, p.partials, p.scal + 0, s));
    for (int m = 0; m < N; ++m) {
        const int *k = p.key[m];
        STN(merge_keys(p.cidx[k[0]], p.cidx[k[1]], nu, (int32_t)p.I[k[1]], p.merged, s));
        STN(build_order_keys(p.merged, p.cidx[k[2]], p.cidx[m], nu, (int32_t)p.I[k[2]], p.nslots[m], p.ptr[m],
                             p.perm, sc, p.flags, s));
        STN(gather_leaf<double>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval64[m], p.flags, s));
        if (p.lval32[m]) STN(gather_leaf<float>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval32[m], p.flags, s));
    }
    int32_t nfib[kMaxOrder] = {0, 0, 0, 0};
    if (p.fib[0])
        for (int m = 0; m < N; ++m) {
            STN(fibre_list(p.ptr[m], p.nslots[m], std::min<int64_t>(p.nslots[m], std::max<int64_t>(p.nnz, 1)),
                           p.fib[m], p.fptr[m], p.counts, p.cursor, p.scan, p.flags, s));
            STN(hipMemcpyAsync(&nfib[m], p.cursor + p.nslots[m], 4, hipMemcpyDeviceToHost, s));
        }
    double nx2 = 0;
    STN(hipMemcpyAsync(&nx2, p.scal + 0, 8, hipMemcpyDeviceToHost, s));
    STN(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    STN(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) {
        if (r == TK_ERR_DEVICE) set_hip_error(hipErrorUnknown, "fibre ordering failed its range checks");
        return r;
    }
    for (int m = 0; m < N; ++m) p.nfib[m] = nfib[m];
    *nu_out = nu;
    *nx2_out = nx2;
    if (!(nx2 > 0.0)) return TK_ERR_EMPTY;
    // MP: the projections write the rows of non-empty fibres only
    if (p.fib[0]) {
        const int es = elem_of(p.prec);
        for (int m = 0; m < N; ++m) STN(fill_i32((int32_t *)p.T[m], p.nslots[m] * p.ld[m] * es / 4, 0, s));
        if (p.Tcore) STN(fill_i32((int32_t *)p.Tcore, p.nslots[N - 1] * p.ldc, 0, s));
    }
    return TK_OK;
}

// FP32 / BF16 copies of factor n and its padded rows for the projections.
hipError_t refresh(PlanN &p, int n, const double *F, hipStream_t s) {
    const int64_t cnt = p.I[n] * p.J[n];
    if (p.F32[n]) TK_HIP(convert_f64<float>(F, p.F32[n], cnt, s));
    if (p.Fbf[n]) TK_HIP(convert_f64<bf16>(F, p.Fbf[n], cnt, s));
    if (p.prec == P64)
        TK_HIP(pad_rows<double>(F, p.I[n], p.J[n], p.ld[n], (double *)p.Fp[n], s));
    else if (p.prec == P32)
        TK_HIP(pad_rows<float>(F, p.I[n], p.J[n], p.ld[n], (float *)p.Fp[n], s));
    else
        TK_HIP(pad_rows<f16>(F, p.I[n], p.J[n], p.ld[n], (f16 *)p.Fp[n], s));
    if (p.Fc && n == p.N - 1) TK_HIP(pad_rows<float>(F, p.I[n], p.J[n], p.ldc, p.Fc, s));
    return hipSuccess;
}

// T(m) = X x_m A(m)^T into T (rows of ld[m], the precision's type). With the
// fibre lists (MP) only the rows of non-empty fibres are written.
hipError_t project_m(PlanN &p, int m, void *T, bool fibres, hipStream_t s, KernelEvents ke = KernelEvents()) {
    FibreList fl;
    if (fibres && p.fib[m]) {
        fl.fib = p.fib[m];
        fl.fptr = p.fptr[m];
        fl.n = p.nfib[m];
    }
    const int ld = p.ld[m];
    if (p.prec == P64)
        return project<double, double, double>(p.ptr[m], p.lidx[m], p.lval64[m], (const double *)p.Fp[m], p.I[m], ld,
                                               p.J[m], ld, p.nslots[m], p.nnz, (double *)T, s, p.tune, ke, fl);
    if (p.prec == P32)
        return project<float, float, float>(p.ptr[m], p.lidx[m], p.lval32[m], (const float *)p.Fp[m], p.I[m], ld,
                                            p.J[m], ld, p.nslots[m], p.nnz, (float *)T, s, p.tune, ke, fl);
    return project<float, f16, bf16>(p.ptr[m], p.lidx[m], p.lval32[m], (const f16 *)p.Fp[m], p.I[m], ld, p.J[m], ld,
                                     p.nslots[m], p.nnz, (bf16 *)T, s, p.tune, ke, fl);
}

// Contract axis a of `sh` (a key axis, mode n = sh.mode[a]) with A(n):
// out[o][q][rest] = sum_i A(n)[i][q] in[o][i][rest], one batched MFMA
// product; sh is updated to the result's shape. `kind` is the gemm element
// kind of the operands, `out_type` the result's type.
hipError_t contract(const PlanN &p, const void *in, Shape &sh, int a, const void *A, int kind, int out_type,
                    void *out, hipStream_t s) {
    const int n = sh.mode[a];
    const int64_t outer = sh.rows_between(0, a);
    const int64_t inner = sh.rows_between(a + 1, sh.r - 1) * sh.ld;
    GemmArgs g;
    g.M = p.J[n];
    g.N = (int)inner;
    g.K = (int)sh.size[a];
    g.batch = (int)outer;
    g.A = A;
    g.lda = p.J[n];
    g.a_trans = true;
    g.B = in;
    g.ldb = inner;
    g.sB = sh.size[a] * inner;
    g.C = out;
    g.ldc = inner;
    g.sC = (int64_t)p.J[n] * inner;
    g.prec = kind;
    g.out_type = out_type;
    if (outer == 1) {  // one product: split its summed dimension for parallelism
        const int tiles = (int)(ceil_div(g.M, 64) * ceil_div(g.N, 64));
        const int64_t per = (int64_t)g.M * g.N;
        int sk = std::max(1, std::min(8, 256 / std::max(1, tiles)));
        while (sk > 1 && sk * per > p.core_split_elems) --sk;
        g.splitk = sk;
        g.split_scratch = p.core_split;
    }
    sh.size[a] = p.J[n];
    return gemm(g, s);
}

// out[p_0]...[p_{N-1}] (row-major core) = in at the axis order of `sh` (all
// axes contracted; the last has row stride sh.ld).
struct PermArgs {
    int N;
    int64_t J[kMaxOrder];      // core sizes by mode
    int64_t stride[kMaxOrder]; // input stride of each mode
};
__global__ void k_permute_core(const double *in, double *out, PermArgs a) {
    int64_t tot = 1;
    for (int k = 0; k < a.N; ++k) tot *= a.J[k];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = t, off = 0;
        for (int k = a.N - 1; k >= 0; --k) {
            const int64_t q = rem % a.J[k];
            rem /= a.J[k];
            off += q * a.stride[k];
        }
        out[t] = in[off];
    }
}

hipError_t permute_core(const PlanN &p, const double *in, const Shape &sh, double *core, hipStream_t s) {
    PermArgs a;
    a.N = p.N;
    int64_t st = 1;
    for (int k = sh.r - 1; k >= 0; --k) {
        a.stride[sh.mode[k]] = st;
        st *= k == sh.r - 1 ? sh.ld : sh.size[k];
    }
    int64_t tot = 1;
    for (int n = 0; n < p.N; ++n) {
        a.J[n] = p.J[n];
        tot *= p.J[n];
    }
    k_permute_core<<<(unsigned)std::min<int64_t>(ceil_div(tot, 256), 65536), 256, 0, s>>>(in, core, a);
    TK_LAUNCHED();
    return hipSuccess;
}

// G = [[X; A(1)^T, ..., A(N)^T]] from the projection T(N-1) (FP64 or FP32
// rows of ld): its key axes are contracted innermost first with the FP64
// factors (FP64 accumulation), then permuted to row-major order.
hipError_t core_from_last(PlanN &p, const void *T, bool t_f64, int ld, double *const *F, double *core,
                          hipStream_t s) {
    Shape sh = proj_shape_of(p, p.N - 1, ld);
    const void *src = T;
    int kind = t_f64 ? P64 : 3;  // FP64 factor with FP64 or FP32 projection, FP64 MFMA
    int buf = 0;
    for (int a = p.N - 2; a >= 0; --a) {
        void *dst = p.Y[buf];
        TK_HIP(contract(p, src, sh, a, F[sh.mode[a]], kind, P64, dst, s));
        src = dst;
        buf ^= 1;
        kind = P64;
    }
    return permute_core(p, (const double *)src, sh, core, s);
}

int finish_fit(PlanN &p, const double *core, hipStream_t s, double *fit, double *g2) {
    int64_t nJ = 1;
    for (int n = 0; n < p.N; ++n) nJ *= p.J[n];
    STN(sumsq(core, nJ, p.partials, p.scal + 1, s));
    double v[2];
    STN(hipMemcpyAsync(v, p.scal, 16, hipMemcpyDeviceToHost, s));
    STN(hipStreamSynchronize(s));
    *g2 = v[1];
    *fit = 1.0 - std::sqrt(std::max(0.0, v[0] - v[1])) / std::sqrt(v[0]);
    return TK_OK;
}

int run_eig(PlanN &p, int n, double *M, double *F, bool warm, const tk_opts *o, tk_stats *st, int *noconv,
            hipStream_t s) {
    EigOpts eo;
    eo.max_iters = o->eig_max_iters;
    eo.tol = o->eig_tol > 0 ? o->eig_tol : (p.eprec == P64 ? 1e-12 : (p.eprec == P32 ? 1e-8 : 1e-4));
    eo.warm = warm && p.blk_ok[n];
    if (eo.warm && p.sweep_solves[n] == 0) eo.warm_degree = eo.degree;
    if (warm) p.sweep_solves[n] += 1;
    eo.seed = 0x5eed0000ull + (uint64_t)n;
    int it = 0, nc = 0;
    STN(lead_eig(M, (int)p.I[n], p.J[n], p.Xblk[n], F, p.theta, p.eigw, eo, &it, &nc, s));
    if (st) {
        st->eig_iters += it;
        st->eig_noconv += nc;
    }
    if (nc) *noconv = 1;
    p.blk_ok[n] = true;
    STN(refresh(p, n, F, s));
    return TK_OK;
}

// The leaf-n ordering's nonzeros written into the dense unfolding D
// (I_n rows of S, zeroed beforehand): D[i_n][slot] = x; every cell holds at
// most one nonzero once duplicates are summed.
__global__ void k_dense_unfold(const int32_t *ptr, const int32_t *lidx, const double *lval, int64_t S, double *D) {
    for (int64_t sl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sl < S; sl += (int64_t)gridDim.x * blockDim.x)
        for (int32_t e = ptr[sl]; e < ptr[sl + 1]; ++e) D[(int64_t)lidx[e] * S + sl] = lval[e];
}

// A(n) from X_(n) X_(n)^T (Figure 2; the start of Figures 4 and 8).
int hosvd_mode(PlanN &p, int n, double *F, const tk_opts *o, tk_stats *st, int *noconv, hipStream_t s) {
    if (p.dense) {
        // X_(n) dense: row i_n, column = slot of the leaf-n ordering (any
        // fixed numbering of the other modes' cells gives the same Gram)
        const int64_t S = p.nslots[n];
        STN(fill_f64(p.dense, p.I[n] * S, 0.0, s));
        k_dense_unfold<<<(unsigned)std::min<int64_t>(ceil_div(S, 256), 65536), 256, 0, s>>>(
            p.ptr[n], p.lidx[n], p.lval64[n], S, p.dense);
        STN(hipGetLastError());
        const GramTerm t{p.dense, S, 0, S, 1};
        STN(gram((int)p.I[n], P64, 1, &t, p.Mg, p.gram_scratch, s, p.tune));
        return run_eig(p, n, p.Mg, F, false, o, st, noconv, s);
    }
    const int n1 = (n + 1) % p.N;
    int64_t S = 1;
    for (int k = 0; k < p.N; ++k)
        if (k != n && k != n1) S *= p.I[k];
    STN(hosvd_gram_sized((int32_t)p.I[n], (int32_t)p.I[n1], (int32_t)S, p.ptr[n], p.lidx[n], p.lval64[n], p.ptr[n1],
                         p.lidx[n1], p.lval64[n1], p.Mg, s));
    return run_eig(p, n, p.Mg, F, false, o, st, noconv, s);
}

int common(int algo, const tk_coo *X, const int32_t *J, const tk_opts *o, void *ws, size_t wsb, PlanN &p) {
    int st = check(algo, X, J, o);
    if (st) return st;
    plan_init(p, algo, o->precision, X, J, algo == TK_ALGO_HOSVD ? TK_INIT_HOSVD : o->init, o->tune);
    Arena ar;
    carve(p, ar);
    if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
    ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    ar.used = 0;
    carve(p, ar);
    if (X->nnz == 0) return TK_ERR_EMPTY;
    return TK_OK;
}

// The starting factors A(2..N): HO-SVD or the caller's.
int start(PlanN &p, const tk_opts *o, double *const *F, tk_stats *st, int *noconv, hipStream_t s) {
    for (int n = 1; n < p.N; ++n) {
        if (o->init == TK_INIT_GIVEN) {
            STN(refresh(p, n, F[n], s));
        } else {
            int r = hosvd_mode(p, n, F[n], o, st, noconv, s);
            if (r) return r;
        }
    }
    return TK_OK;
}

}  // namespace

size_t order_n_workspace(int algo, const tk_coo *X, const int32_t *J, const tk_opts *o, int *status) {
    *status = check(algo, X, J, o);
    if (*status) return 0;
    PlanN p;
    plan_init(p, algo, algo == TK_ALGO_HOSVD ? TK_FP64 : o->precision, X, J, TK_INIT_HOSVD, o->tune);
    Arena ar;
    carve(p, ar);
    return ar.used + 256;
}

int order_n_mp(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
               int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream) {
    if (!core || !F || !iters_done || (o && o->max_iters > 0 && !hist)) return TK_ERR_ARG;
    for (int n = 0; n < 4; ++n)
        if (!F[n]) return TK_ERR_ARG;
    PlanN p;
    int st = common(TK_ALGO_MP, X, J, o, ws, wsb, p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    Timer tm(o, s);
    const int N = p.N;
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    if ((st = start(p, o, F, stats, &noconv, s))) return st;
    // projections of the start: T(m) for m = 2..N (the Grams of A(1) use them)
    for (int m = 1; m < N; ++m) STN(project_m(p, m, p.T[m], true, s));
    STN(hipStreamSynchronize(s));
    double t2 = now_ms();
    double prev = 0.0, g2 = 0.0;
    *iters_done = 0;
    const int maxit = std::max(o->max_iters, 1);
    for (int t = 1; t <= maxit; ++t) {
        for (int n = 0; n < N; ++n) {
            // M_n = sum over the other modes m of T(m)_(n) T(m)_(n)^T (Figure 8)
            GramTerm g[kGramMaxTerms];
            int nt = 0;
            for (int m = 0; m < N; ++m) {
                if (m == n) continue;
                const Shape sh = proj_shape_of(p, m, p.ld[m]);
                int a = 0;
                while (sh.mode[a] != n) ++a;
                GramTerm q;
                q.base = p.T[m];
                const int64_t inner = sh.rows_between(a + 1, sh.r - 1) * sh.ld;
                q.s_row = inner;
                q.chunk_len = inner;
                q.nchunks = sh.rows_between(0, a);
                q.s_chunk = q.nchunks > 1 ? p.I[n] * inner : 0;
                g[nt++] = q;
            }
            tm.begin(kGram, n, p.prec);
            STN(gram((int)p.I[n], p.prec, nt, g, p.Mg, p.gram_scratch, s, p.tune));
            tm.end();
            tm.begin(kEig, n, P64);
            if ((st = run_eig(p, n, p.Mg, F[n], true, o, stats, &noconv, s))) return st;
            tm.end();
            STN(project_m(p, n, p.T[n], true, s, tm.kernel(kProj, n, p.prec)));
        }
        // core from the last mode's projection (FP64 / FP32; an FP32 one for BF16)
        const void *Tc = p.T[N - 1];
        int ldc = p.ld[N - 1];
        if (p.prec == PBF16) {
            FibreList fl;
            fl.fib = p.fib[N - 1];
            fl.fptr = p.fptr[N - 1];
            fl.n = p.nfib[N - 1];
            STN((project<float, float, float>(p.ptr[N - 1], p.lidx[N - 1], p.lval32[N - 1], p.Fc, p.I[N - 1], p.ldc,
                                              p.J[N - 1], p.ldc, p.nslots[N - 1], p.nnz, p.Tcore, s, p.tune,
                                              tm.kernel(kProj, N - 1, P32), fl)));
            Tc = p.Tcore;
            ldc = p.ldc;
        }
        tm.begin(kCore, -1, p.prec == P64 ? P64 : P32);
        STN(core_from_last(p, Tc, p.prec == P64, ldc, F, core, s));
        tm.end();
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
        tm.collect();
        hist[t - 1] = fit;
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

int order_n_hooi(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
                 int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream) {
    if (!core || !F || !iters_done || (o && o->max_iters > 0 && !hist)) return TK_ERR_ARG;
    for (int n = 0; n < 4; ++n)
        if (!F[n]) return TK_ERR_ARG;
    PlanN p;
    int st = common(TK_ALGO_HOOI, X, J, o, ws, wsb, p);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    Timer tm(o, s);
    const int N = p.N;
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    if ((st = start(p, o, F, stats, &noconv, s))) return st;
    STN(hipStreamSynchronize(s));
    double t2 = now_ms();
    // element kinds: the projection in the precision's type; FP64 runs FP64
    // products and Grams; FP32 and mixed produce FP32 (mixed: its first
    // product takes BF16 operands)
    const int yt = p.prec == P64 ? P64 : P32;
    double prev = 0.0, g2 = 0.0;
    *iters_done = 0;
    const int maxit = std::max(o->max_iters, 1);
    for (int t = 1; t <= maxit; ++t) {
        Shape last;
        const void *ylast = nullptr;
        for (int n = 0; n < N; ++n) {
            // Z = X x_m A(m)^T, then every other key but n contracted (Figure 4)
            const int m = n == N - 1 ? N - 2 : N - 1;
            STN(project_m(p, m, p.T[0], false, s, tm.kernel(kProj, m, p.prec)));
            Shape sh = proj_shape_of(p, m, p.ld[m]);
            const void *src = p.T[0];
            int buf = 0;
            int kind = p.prec;
            tm.begin(kTtmc, n, p.prec);
            for (int a = N - 2; a >= 0; --a) {
                if (sh.mode[a] == n) continue;
                const int k = sh.mode[a];
                const void *A = kind == P64 ? (const void *)F[k]
                                : (kind == P32 ? (const void *)p.F32[k] : (const void *)p.Fbf[k]);
                STN(contract(p, src, sh, a, A, kind, yt, p.Y[buf], s));
                src = p.Y[buf];
                buf ^= 1;
                kind = yt;
            }
            tm.end();
            // M_n = Z_(n) Z_(n)^T
            int a = 0;
            while (sh.mode[a] != n) ++a;
            GramTerm q;
            q.base = src;
            const int64_t inner = sh.rows_between(a + 1, sh.r - 1) * sh.ld;
            q.s_row = inner;
            q.chunk_len = inner;
            q.nchunks = sh.rows_between(0, a);
            q.s_chunk = q.nchunks > 1 ? p.I[n] * inner : 0;
            tm.begin(kGram, n, yt);
            STN(gram((int)p.I[n], yt, 1, &q, p.Mg, p.gram_scratch, s, p.tune));
            tm.end();
            tm.begin(kEig, n, P64);
            if ((st = run_eig(p, n, p.Mg, F[n], true, o, stats, &noconv, s))) return st;
            tm.end();
            last = sh;
            ylast = src;
        }
        // core: the last Z (all keys but the last mode's contracted)
        // contracted with A(N) (FP64 factor, FP64 accumulation), then permuted
        tm.begin(kCore, -1, yt);
        {
            int a = 0;
            while (last.mode[a] != N - 1) ++a;
            void *dst = ylast == p.Y[0] ? p.Y[1] : p.Y[0];
            STN(contract(p, ylast, last, a, F[N - 1], yt == P64 ? P64 : 3, P64, dst, s));
            STN(permute_core(p, (const double *)dst, last, core, s));
        }
        tm.end();
        double fit = 0;
        if ((st = finish_fit(p, core, s, &fit, &g2))) return st;
        tm.collect();
        hist[t - 1] = fit;
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

int order_n_hosvd(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *fit,
                  tk_stats *stats, void *ws, size_t wsb, void *stream) {
    if (!core || !F || !fit) return TK_ERR_ARG;
    for (int n = 0; n < 4; ++n)
        if (!F[n]) return TK_ERR_ARG;
    tk_opts oh = *o;
    oh.precision = TK_FP64;  // FP64 projection for the core
    PlanN p;
    int st = common(TK_ALGO_HOSVD, X, J, &oh, ws, wsb, p);
    if (st) return st;
    p.eprec = o->precision == TK_FP32 ? P32 : (o->precision == TK_MIXED_BF16 ? PBF16 : P64);
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    double t1 = now_ms();
    int noconv = 0;
    for (int n = 0; n < p.N; ++n)
        if ((st = hosvd_mode(p, n, F[n], &oh, stats, &noconv, s))) return st;
    STN(project_m(p, p.N - 1, p.T[0], false, s));
    STN(core_from_last(p, p.T[0], true, p.ld[p.N - 1], F, core, s));
    double g2 = 0;
    if ((st = finish_fit(p, core, s, fit, &g2))) return st;
    double t2 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
        stats->hosvd_fit = *fit;
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

}  // namespace tk
