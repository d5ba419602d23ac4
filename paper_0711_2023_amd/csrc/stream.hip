// Multislice Projection of a third-order tensor held in host memory, streamed
// through bounded device memory (tucker_mp_streamed).
//
// The paper scales MP past RAM by sorting the nonzeros once and reading one
// slice file at a time in every sweep (Section 4.3, slice construction;
// Section 5.1). Here the host sorts the nonzeros once into six orderings and
// every sweep streams slabs of them to the device:
// * M_n = sum over the two other modes m of T(m)_(n) T(m)_(n)^T with
//   T(m) = X x_m A(m)^T (Figure 7, slice products regrouped). For the term
//   (n, m) the third mode k slices T(m) into slabs of consecutive i_k: within
//   a slab T is dense [i_k][i_n][r], and the slab's share of the Gram,
//   sum over its i_k of T[i_k] T[i_k]^T, is a Gram kernel call with i_k as
//   the batch. So the term streams the ordering of leaf m keyed by (i_k,
//   i_n); the six (leaf, major key) pairs are the six orderings.
// * Each slab is projected into a dense buffer, its Gram share accumulated in
//   FP64 in slab order (deterministic), and the buffers are reused.
// * The core comes from T(3) streamed in slabs of i_2 (the ordering of leaf
//   3 keyed by (i_2, i_1)): Z[i_2][p][r] = sum_i1 A[i_1][p] T[i_2][i_1][r] per
//   slab, then G from B^T Z and a permutation; the fit from ||G||^2.
// Slabs alternate between two pinned host staging buffers and two device
// buffers: the host copies slab s+1 into its staging buffer and a second
// stream uploads it while the caller's stream projects slab s.
#include "../../include/tucker.h"
#include "common.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace tk {
namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxJs = 128;

// One ordering on the host: entries sorted by (i_k, i_j, i_m) (major k,
// minor j, leaf m), slot pointers over (i_k, i_j).
struct HostOrder {
    int m = 0, k = 0, j = 0;
    std::vector<int32_t> lidx;
    std::vector<double> lval;
    std::vector<int64_t> ptr;  // I_k * I_j + 1
};

// A slab: consecutive i_k in [k0, k1), entries [e0, e1) of the ordering.
struct Slab {
    int64_t k0, k1, e0, e1;
};

// Stable counting sort of the positions `in` by key[pos] (0 <= key < nkeys).
void counting_sort(const std::vector<int64_t> &in, const int32_t *key, int64_t nkeys, std::vector<int64_t> &out) {
    std::vector<int64_t> cnt(nkeys + 1, 0);
    for (int64_t p : in) cnt[key[p] + 1]++;
    for (int64_t i = 0; i < nkeys; ++i) cnt[i + 1] += cnt[i];
    out.resize(in.size());
    for (int64_t p : in) out[cnt[key[p]]++] = p;
}

// Positions 0..n-1 sorted by (c0, c1, c2) lexicographically (LSD counting sorts).
std::vector<int64_t> lex_order(int64_t n, const int32_t *c0, int64_t n0, const int32_t *c1, int64_t n1,
                               const int32_t *c2, int64_t n2) {
    std::vector<int64_t> a(n), b;
    for (int64_t i = 0; i < n; ++i) a[i] = i;
    counting_sort(a, c2, n2, b);
    counting_sort(b, c1, n1, a);
    counting_sort(a, c0, n0, b);
    return b;
}

struct StreamPlan {
    int prec = P64;
    int64_t I[3] = {}, nnz = 0;  // nnz after duplicate summing
    int J[3] = {};
    int ld[3] = {};   // row stride of the Gram projections (16-byte rows)
    int ldc = 0;      // row stride of the core's projection (FP32 / FP64)
    // device layout
    size_t slab_T_bytes = 0;     // one dense slab buffer
    int64_t slab_nnz = 0;        // entries per slab buffer
    int64_t slab_slots = 0;      // slot pointers per slab buffer
    // the six orderings: index o = 2 * m + (k == (m + 1) % 3 ? 0 : 1)
    HostOrder ord[6];
    std::vector<Slab> slabs[6];
    // device buffers
    double *M = nullptr, *Mt = nullptr, *theta = nullptr, *Xblk[3] = {}, *Z = nullptr, *Gp = nullptr,
           *core_split = nullptr, *scal = nullptr, *partials = nullptr;
    int64_t core_split_elems = 0;
    void *eigw = nullptr, *gram_scratch = nullptr, *Fp[3] = {}, *Fc = nullptr;
    void *T[2] = {};
    int32_t *dptr[2] = {}, *didx[2] = {};
    void *dval[2] = {};
    int b[3] = {};
    bool blk_ok[3] = {};
    int sweep_solves[3] = {};
};

int ord_index(int m, int k) { return 2 * m + (k == (m + 1) % 3 ? 0 : 1); }

int elem_of(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// Device slab buffers and the fixed part of the workspace.
void carve(StreamPlan &p, Arena &ar) {
    int64_t maxI = std::max({p.I[0], p.I[1], p.I[2]});
    p.M = ar.take<double>(maxI * maxI);
    p.Mt = ar.take<double>(maxI * maxI);
    p.scal = ar.take<double>(8);
    p.partials = ar.take<double>(kReduceBlocks);
    size_t gs = 0;
    for (int n = 0; n < 3; ++n)
        for (int m = 0; m < 3; ++m) {
            if (m == n) continue;
            int64_t K = p.slab_T_bytes / std::max<int64_t>(1, (int64_t)elem_of(p.prec) * p.I[n]);
            gs = std::max(gs, gram_scratch_bytes((int)p.I[n], p.prec, 1, &K));
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
    for (int n = 0; n < 3; ++n) p.Fp[n] = ar.take<char>(p.I[n] * p.ld[n] * (int64_t)elem_of(p.prec == P64 ? P64 : (p.prec == P32 ? P32 : PBF16)));
    p.Fc = p.prec == PBF16 ? ar.take<float>(p.I[2] * p.ldc) : nullptr;
    p.Z = ar.take<double>(std::max<int64_t>(1, p.I[1] * p.J[0] * p.ldc));
    p.Gp = ar.take<double>((int64_t)p.J[0] * p.J[1] * p.ldc);
    p.core_split_elems = 8 * (int64_t)p.J[0] * p.J[1] * p.ldc;
    p.core_split = ar.take<double>(p.core_split_elems);
    for (int q = 0; q < 2; ++q) {
        p.T[q] = ar.take<char>((int64_t)p.slab_T_bytes);
        p.dptr[q] = ar.take<int32_t>(p.slab_slots + 1);
        p.didx[q] = ar.take<int32_t>(p.slab_nnz);
        p.dval[q] = ar.take<char>(p.slab_nnz * (p.prec == P64 ? 8 : 4));
    }
}

// Slabs of ordering o: consecutive major indices while the dense slab (rows
// of the widest projection this ordering feeds) and its entries fit.
void plan_slabs(StreamPlan &p, int o, int64_t rows_per_k, int64_t row_bytes) {
    const HostOrder &h = p.ord[o];
    const int64_t Ik = p.I[h.k], Ij = p.I[h.j];
    std::vector<Slab> &sl = p.slabs[o];
    sl.clear();
    const int64_t kmax_T = std::max<int64_t>(1, (int64_t)p.slab_T_bytes / std::max<int64_t>(1, rows_per_k * row_bytes));
    int64_t k0 = 0;
    while (k0 < Ik) {
        int64_t k1 = k0;
        while (k1 < Ik && k1 - k0 < kmax_T && h.ptr[(k1 + 1) * Ij] - h.ptr[k0 * Ij] <= p.slab_nnz) ++k1;
        if (k1 == k0) k1 = k0 + 1;  // a single slice beyond the entry budget: planned larger (checked)
        sl.push_back(Slab{k0, k1, h.ptr[k0 * Ij], h.ptr[k1 * Ij]});
        k0 = k1;
    }
}

// Duplicate summing and the six orderings, on the host.
int host_orders(StreamPlan &p, const tk_coo *X, double *nx2) {
    const int64_t n = X->nnz;
    for (int64_t q = 0; q < n; ++q) {
        for (int d = 0; d < 3; ++d)
            if (X->idx[d][q] < 0 || X->idx[d][q] >= p.I[d]) return TK_ERR_INDEX;
        if (!std::isfinite(X->vals[q])) return TK_ERR_VALUE;
    }
    std::vector<int64_t> o = lex_order(n, X->idx[0], p.I[0], X->idx[1], p.I[1], X->idx[2], p.I[2]);
    std::vector<int32_t> c[3];
    std::vector<double> v;
    for (int d = 0; d < 3; ++d) c[d].reserve(n);
    v.reserve(n);
    for (int64_t t = 0; t < n; ++t) {
        const int64_t q = o[t];
        if (!v.empty() && c[0].back() == X->idx[0][q] && c[1].back() == X->idx[1][q] && c[2].back() == X->idx[2][q]) {
            v.back() += X->vals[q];  // duplicates in input order
            continue;
        }
        for (int d = 0; d < 3; ++d) c[d].push_back(X->idx[d][q]);
        v.push_back(X->vals[q]);
    }
    p.nnz = (int64_t)v.size();
    // ||X||^2, compensated (Neumaier)
    double sum = 0.0, comp = 0.0;
    for (double x : v) {
        const double y = x * x, t = sum + y;
        comp += std::fabs(sum) >= std::fabs(y) ? (sum - t) + y : (y - t) + sum;
        sum = t;
    }
    *nx2 = sum + comp;
    for (int m = 0; m < 3; ++m)
        for (int kk = 0; kk < 2; ++kk) {
            const int k = (m + 1 + kk) % 3, j = 3 - m - k;
            HostOrder &h = p.ord[ord_index(m, k)];
            h.m = m;
            h.k = k;
            h.j = j;
            std::vector<int64_t> oo = lex_order(p.nnz, c[k].data(), p.I[k], c[j].data(), p.I[j], c[m].data(), p.I[m]);
            h.lidx.resize(p.nnz);
            h.lval.resize(p.nnz);
            h.ptr.assign(p.I[k] * p.I[j] + 1, 0);
            for (int64_t t = 0; t < p.nnz; ++t) {
                const int64_t q = oo[t];
                h.lidx[t] = c[m][q];
                h.lval[t] = v[q];
                h.ptr[(int64_t)c[k][q] * p.I[j] + c[j][q] + 1]++;
            }
            for (int64_t t = 0; t + 1 < (int64_t)h.ptr.size(); ++t) h.ptr[t + 1] += h.ptr[t];
        }
    return TK_OK;
}

#define STS(call)                         \
    do {                                  \
        hipError_t e_ = (call);           \
        if (e_ != hipSuccess) {           \
            set_hip_error(e_, #call);     \
            return TK_ERR_DEVICE;         \
        }                                 \
    } while (0)

void plan_init(StreamPlan &p, const tk_coo *X, const int32_t *J, int prec, size_t slab_bytes) {
    p.prec = prec;
    for (int n = 0; n < 3; ++n) {
        p.I[n] = X->dims[n];
        p.J[n] = J[n];
        const int v = 16 / elem_of(prec);
        p.ld[n] = (int)ceil_div(J[n], v) * v;
    }
    p.ldc = (int)ceil_div(J[2], prec == P64 ? 2 : 4) * (prec == P64 ? 2 : 4);
    p.slab_T_bytes = std::max<size_t>(slab_bytes, 256) / 256 * 256;
    p.slab_nnz = std::max<int64_t>(1, (int64_t)(slab_bytes / 8));
    int min_row = p.ldc * (prec == P64 ? 8 : 4);
    for (int n = 0; n < 3; ++n) min_row = std::min(min_row, p.ld[n] * elem_of(prec));
    p.slab_slots = (int64_t)(p.slab_T_bytes / (size_t)min_row) + 1;
}

// The caller's problem, its options and the slab size: TK_OK or TK_ERR_ARG.
int check(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t slab_bytes) {
    if (!X || !J || !o || !X->dims || X->order != 3) return TK_ERR_ARG;
    if (X->nnz < 0 || X->nnz >= (int64_t)INT32_MAX - 1) return TK_ERR_ARG;
    if (X->nnz > 0 && (!X->idx[0] || !X->idx[1] || !X->idx[2] || !X->vals)) return TK_ERR_ARG;
    for (int n = 0; n < 3; ++n) {
        if (X->dims[n] < 1 || X->dims[n] >= INT32_MAX) return TK_ERR_ARG;
        if (J[n] < 1 || J[n] > X->dims[n] || J[n] > kMaxJs) return TK_ERR_ARG;
    }
    if (o->precision != TK_FP64 && o->precision != TK_FP32 && o->precision != TK_MIXED_BF16) return TK_ERR_ARG;
    if (o->init != TK_INIT_RANDOM && o->init != TK_INIT_GIVEN) return TK_ERR_ARG;
    if (o->max_iters < 1 || o->eig_max_iters < 1 || !(o->eig_tol >= 0.0) || std::isnan(o->tol)) return TK_ERR_ARG;
    if (o->hosvd_fit || o->trace) return TK_ERR_ARG;
    // one slice of every ordering's dense slab must fit the slab buffer
    StreamPlan p;
    plan_init(p, X, J, o->precision, slab_bytes);
    for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
            if (n == m) continue;
            if ((size_t)(p.I[n] * p.ld[m] * elem_of(p.prec)) > p.slab_T_bytes) return TK_ERR_ARG;
        }
    if ((size_t)(p.I[0] * p.ldc * (p.prec == P64 ? 8 : 4)) > p.slab_T_bytes) return TK_ERR_ARG;
    return TK_OK;
}

// Projection of one slab (entries e0..e1 of the ordering, dense rows of
// `ld`), from the padded factor copy.
hipError_t project_slab(StreamPlan &p, int q, int m, int64_t nslots, int64_t nnz, bool core, hipStream_t s) {
    if (core && p.prec == PBF16)
        return project<float, float, float>(p.dptr[q], p.didx[q], (const float *)p.dval[q], (const float *)p.Fc,
                                            p.I[m], p.ldc, p.J[m], p.ldc, nslots, nnz, (float *)p.T[q], s);
    const int ld = core ? p.ldc : p.ld[m];
    if (p.prec == P64)
        return project<double, double, double>(p.dptr[q], p.didx[q], (const double *)p.dval[q],
                                               (const double *)p.Fp[m], p.I[m], ld, p.J[m], ld, nslots, nnz,
                                               (double *)p.T[q], s);
    if (p.prec == P32)
        return project<float, float, float>(p.dptr[q], p.didx[q], (const float *)p.dval[q], (const float *)p.Fp[m],
                                            p.I[m], ld, p.J[m], ld, nslots, nnz, (float *)p.T[q], s);
    return project<float, f16, bf16>(p.dptr[q], p.didx[q], (const float *)p.dval[q], (const f16 *)p.Fp[m], p.I[m],
                                     ld, p.J[m], ld, nslots, nnz, (bf16 *)p.T[q], s);
}

__global__ void k_add_f64(double *y, const double *x, int64_t n, int first) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        y[t] = first ? x[t] : y[t] + x[t];
}

// core[p][q][r] = G'[q][p][r] (r < J2; G' rows of ldc)
__global__ void k_core_out(const double *Gp, double *core, int J0, int J1, int J2, int ldc) {
    const int64_t tot = (int64_t)J0 * J1 * J2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / ((int64_t)J1 * J2));
        const int rem = (int)(t - (int64_t)p * J1 * J2);
        const int qq = rem / J2, r = rem - qq * J2;
        core[t] = Gp[((int64_t)qq * J0 + p) * ldc + r];
    }
}

// Slab streaming: two pinned staging buffers, a copy stream and events.
struct Streamer {
    StreamPlan &p;
    hipStream_t s, cs = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    char *stage[2] = {nullptr, nullptr};
    size_t stage_bytes = 0;
    int64_t bytes = 0, slabs = 0;
    explicit Streamer(StreamPlan &p_, hipStream_t s_) : p(p_), s(s_) {}
    ~Streamer() {
        if (cs) (void)hipStreamSynchronize(cs);
        if (s) (void)hipStreamSynchronize(s);
        for (int q = 0; q < 2; ++q) {
            if (copied[q]) (void)hipEventDestroy(copied[q]);
            if (used[q]) (void)hipEventDestroy(used[q]);
            if (stage[q]) (void)hipHostFree(stage[q]);
        }
        if (cs) (void)hipStreamDestroy(cs);
    }
    hipError_t init() {
        const size_t vb = p.prec == P64 ? 8 : 4;
        stage_bytes = align_up((size_t)(p.slab_slots + 1) * 4, 256) + align_up((size_t)p.slab_nnz * 4, 256) +
                      (size_t)p.slab_nnz * vb;
        TK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        for (int q = 0; q < 2; ++q) {
            TK_HIP(hipEventCreateWithFlags(&copied[q], hipEventDisableTiming));
            TK_HIP(hipEventCreateWithFlags(&used[q], hipEventDisableTiming));
            TK_HIP(hipHostMalloc((void **)&stage[q], stage_bytes, hipHostMallocDefault));
        }
        return hipSuccess;
    }
    // Upload slab `sl` of ordering o into device buffer set q (on the copy
    // stream, after the set's previous use on s), make s wait for it.
    hipError_t upload(int q, int o, const Slab &sl) {
        const HostOrder &h = p.ord[o];
        if (pending[q]) TK_HIP(hipEventSynchronize(used[q]));
        const int64_t Ij = p.I[h.j];
        const int64_t ns = (sl.k1 - sl.k0) * Ij, ne = sl.e1 - sl.e0;
        int32_t *hp = reinterpret_cast<int32_t *>(stage[q]);
        int32_t *hi = reinterpret_cast<int32_t *>(stage[q] + align_up((size_t)(p.slab_slots + 1) * 4, 256));
        char *hv = stage[q] + align_up((size_t)(p.slab_slots + 1) * 4, 256) + align_up((size_t)p.slab_nnz * 4, 256);
        for (int64_t t = 0; t <= ns; ++t) hp[t] = (int32_t)(h.ptr[sl.k0 * Ij + t] - sl.e0);
        std::memcpy(hi, h.lidx.data() + sl.e0, (size_t)ne * 4);
        if (p.prec == P64) {
            std::memcpy(hv, h.lval.data() + sl.e0, (size_t)ne * 8);
        } else {
            float *f = reinterpret_cast<float *>(hv);
            for (int64_t t = 0; t < ne; ++t) f[t] = (float)h.lval[sl.e0 + t];
        }
        const size_t vb = p.prec == P64 ? 8 : 4;
        TK_HIP(hipMemcpyAsync(p.dptr[q], hp, (size_t)(ns + 1) * 4, hipMemcpyHostToDevice, cs));
        TK_HIP(hipMemcpyAsync(p.didx[q], hi, (size_t)ne * 4, hipMemcpyHostToDevice, cs));
        TK_HIP(hipMemcpyAsync(p.dval[q], hv, (size_t)ne * vb, hipMemcpyHostToDevice, cs));
        TK_HIP(hipEventRecord(copied[q], cs));
        TK_HIP(hipStreamWaitEvent(s, copied[q], 0));
        bytes += (ns + 1) * 4 + ne * (4 + (int64_t)vb);
        slabs += 1;
        return hipSuccess;
    }
    hipError_t release(int q) {
        TK_HIP(hipEventRecord(used[q], s));
        pending[q] = true;
        return hipSuccess;
    }
};

int run_eig_s(StreamPlan &p, int n, double *F, bool warm, const tk_opts *o, tk_stats *st, int *noconv,
              hipStream_t s) {
    EigOpts eo;
    eo.max_iters = o->eig_max_iters;
    eo.tol = o->eig_tol > 0 ? o->eig_tol : (p.prec == P64 ? 1e-12 : (p.prec == P32 ? 1e-8 : 1e-4));
    eo.warm = warm && p.blk_ok[n];
    if (eo.warm && p.sweep_solves[n] == 0) eo.warm_degree = eo.degree;
    if (warm) p.sweep_solves[n] += 1;
    eo.seed = 0x5eed0000ull + (uint64_t)n;
    int it = 0, nc = 0;
    STS(lead_eig(p.M, (int)p.I[n], p.J[n], p.Xblk[n], F, p.theta, p.eigw, eo, &it, &nc, s));
    if (st) {
        st->eig_iters += it;
        st->eig_noconv += nc;
    }
    if (nc) *noconv = 1;
    p.blk_ok[n] = true;
    return TK_OK;
}

hipError_t refresh_s(StreamPlan &p, int n, const double *F, hipStream_t s) {
    if (p.prec == P64)
        TK_HIP(pad_rows<double>(F, p.I[n], p.J[n], p.ld[n], (double *)p.Fp[n], s));
    else if (p.prec == P32)
        TK_HIP(pad_rows<float>(F, p.I[n], p.J[n], p.ld[n], (float *)p.Fp[n], s));
    else
        TK_HIP(pad_rows<f16>(F, p.I[n], p.J[n], p.ld[n], (f16 *)p.Fp[n], s));
    if (p.Fc && n == 2) TK_HIP(pad_rows<float>(F, p.I[2], p.J[2], p.ldc, (float *)p.Fc, s));
    return hipSuccess;
}

}  // namespace

int mp_streamed_workspace(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t slab_bytes, size_t *bytes) {
    if (!bytes) return TK_ERR_ARG;
    int st = check(X, J, o, slab_bytes);
    if (st) return st;
    StreamPlan p;
    plan_init(p, X, J, o->precision, slab_bytes);
    Arena ar;
    carve(p, ar);
    *bytes = ar.used + 256;
    return TK_OK;
}

int mp_streamed(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t slab_bytes, double *core,
                double *const *F, double *hist, int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb,
                void *stream) {
    int st = check(X, J, o, slab_bytes);
    if (st) return st;
    if (!core || !F || !F[0] || !F[1] || !F[2] || !hist || !iters_done) return TK_ERR_ARG;
    StreamPlan p;
    plan_init(p, X, J, o->precision, slab_bytes);
    {
        Arena ar;
        carve(p, ar);
        if (!ws || wsb < ar.used + 256) return TK_ERR_WORKSPACE;
        ar.base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
        ar.used = 0;
        carve(p, ar);
    }
    if (X->nnz == 0) return TK_ERR_EMPTY;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    const double t0 = now_ms();
    double nx2 = 0.0;
    if ((st = host_orders(p, X, &nx2))) return st;
    if (!(nx2 > 0.0)) return TK_ERR_EMPTY;
    // slab plans: the Gram terms' orderings with their projection's rows,
    // the core's ordering (leaf 3, major 2) with FP32 / FP64 rows of ldc
    const int es = elem_of(p.prec);
    for (int m = 0; m < 3; ++m)
        for (int kk = 0; kk < 2; ++kk) {
            const int k = (m + 1 + kk) % 3, o_ = ord_index(m, k);
            const int j = 3 - m - k;
            plan_slabs(p, o_, p.I[j], (int64_t)p.ld[m] * es);
            for (const Slab &sl : p.slabs[o_])
                if (sl.e1 - sl.e0 > p.slab_nnz) return TK_ERR_ARG;  // one slice beyond the entry budget
        }
    std::vector<Slab> core_slabs;
    {
        const int o_ = ord_index(2, 1);
        std::vector<Slab> keep = p.slabs[o_];
        plan_slabs(p, o_, p.I[0], (int64_t)p.ldc * (p.prec == P64 ? 8 : 4));
        core_slabs = p.slabs[o_];
        p.slabs[o_] = keep;
        for (const Slab &sl : core_slabs)
            if (sl.e1 - sl.e0 > p.slab_nnz) return TK_ERR_ARG;
    }
    Streamer sm(p, s);
    STS(sm.init());
    const double t1 = now_ms();
    int noconv = 0;
    for (int n = 1; n < 3; ++n) {
        if (o->init == TK_INIT_RANDOM) STS(random_start_fill(F[n], p.I[n], p.J[n], n, o->seed, s));
        STS(refresh_s(p, n, F[n], s));
    }
    STS(hipStreamSynchronize(s));
    const double t2 = now_ms();
    double prev = 0.0, g2 = 0.0;
    *iters_done = 0;
    int slab_no = 0;
    for (int t = 1; t <= o->max_iters; ++t) {
        for (int n = 0; n < 3; ++n) {
            // M_n = sum over m != n of the slabs' Gram shares (Figure 7)
            bool first = true;
            for (int m = 0; m < 3; ++m) {
                if (m == n) continue;
                const int k = 3 - n - m, o_ = ord_index(m, k);
                for (const Slab &sl : p.slabs[o_]) {
                    const int q = slab_no++ & 1;
                    const int64_t nsl = (sl.k1 - sl.k0) * p.I[n];
                    STS(sm.upload(q, o_, sl));
                    STS(project_slab(p, q, m, nsl, sl.e1 - sl.e0, false, s));
                    GramTerm g;
                    g.base = p.T[q];
                    g.s_row = p.ld[m];
                    g.chunk_len = p.ld[m];
                    g.nchunks = sl.k1 - sl.k0;
                    g.s_chunk = g.nchunks > 1 ? p.I[n] * p.ld[m] : 0;
                    STS(gram((int)p.I[n], p.prec, 1, &g, p.Mt, p.gram_scratch, s));
                    const int64_t nn = p.I[n] * p.I[n];
                    k_add_f64<<<(unsigned)std::min<int64_t>(ceil_div(nn, 256), 4096), 256, 0, s>>>(p.M, p.Mt, nn,
                                                                                                 first ? 1 : 0);
                    STS(hipGetLastError());
                    STS(sm.release(q));
                    first = false;
                }
            }
            if ((st = run_eig_s(p, n, F[n], true, o, stats, &noconv, s))) return st;
            STS(refresh_s(p, n, F[n], s));
        }
        // core: Z rows from the slabs of T(3) (leaf 3, major 2), then B^T Z
        const int o_ = ord_index(2, 1);
        for (const Slab &sl : core_slabs) {
            const int q = slab_no++ & 1;
            STS(sm.upload(q, o_, sl));
            STS(project_slab(p, q, 2, (sl.k1 - sl.k0) * p.I[0], sl.e1 - sl.e0, true, s));
            GemmArgs g;
            g.M = p.J[0];
            g.N = p.ldc;
            g.K = (int)p.I[0];
            g.batch = (int)(sl.k1 - sl.k0);
            g.A = F[0];
            g.lda = p.J[0];
            g.a_trans = true;
            g.B = p.T[q];
            g.ldb = p.ldc;
            g.sB = p.I[0] * p.ldc;
            g.C = p.Z + sl.k0 * p.J[0] * p.ldc;
            g.ldc = p.ldc;
            g.sC = (int64_t)p.J[0] * p.ldc;
            g.prec = p.prec == P64 ? P64 : 3;
            g.out_type = P64;
            STS(gemm(g, s));
            STS(sm.release(q));
        }
        {
            GemmArgs h;
            h.M = p.J[1];
            h.N = p.J[0] * p.ldc;
            h.K = (int)p.I[1];
            h.batch = 1;
            h.A = F[1];
            h.lda = p.J[1];
            h.a_trans = true;
            h.B = p.Z;
            h.ldb = (int64_t)p.J[0] * p.ldc;
            h.sB = 0;
            h.C = p.Gp;
            h.ldc = (int64_t)p.J[0] * p.ldc;
            h.sC = 0;
            h.prec = P64;
            h.out_type = P64;
            const int tiles = (int)(ceil_div(p.J[1], 64) * ceil_div((int64_t)p.J[0] * p.ldc, 64));
            h.splitk = std::max(1, std::min(8, 256 / std::max(1, tiles)));
            h.split_scratch = p.core_split;
            STS(gemm(h, s));
            const int64_t nJ = (int64_t)p.J[0] * p.J[1] * p.J[2];
            k_core_out<<<(unsigned)std::min<int64_t>(ceil_div(nJ, 256), 65536), 256, 0, s>>>(p.Gp, core, p.J[0],
                                                                                              p.J[1], p.J[2], p.ldc);
            STS(hipGetLastError());
            STS(sumsq(core, nJ, p.partials, p.scal + 1, s));
        }
        STS(hipMemcpyAsync(&g2, p.scal + 1, 8, hipMemcpyDeviceToHost, s));
        STS(hipStreamSynchronize(s));
        const double fit = 1.0 - std::sqrt(std::max(0.0, nx2 - g2)) / std::sqrt(nx2);
        hist[t - 1] = fit;
        *iters_done = t;
        if (o->tol > 0 && fit - prev < o->tol) break;
        prev = fit;
    }
    const double t3 = now_ms();
    if (stats) {
        stats->prep_ms = t1 - t0;
        stats->init_ms = t2 - t1;
        stats->sweeps_ms = t3 - t2;
        stats->nnz_unique = p.nnz;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
        stats->streamed_bytes = sm.bytes;
        stats->streamed_slabs = sm.slabs;
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

}  // namespace tk
