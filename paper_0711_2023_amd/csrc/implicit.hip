// Multislice Projection without its Grams (tucker_mp_implicit): the
// projections are kept only for the non-empty fibres, and the leading
// subspace of each M_n is found from products with M_n that never form it.
//
// MP's matrix for mode n (Figure 7, the slice products regrouped) is
//   M_n = sum over the two other modes m of T(m)_(n) T(m)_(n)^T,
//   T(m) = X x_m A(m)^T,
// where T(m) is indexed by the two modes other than m, the unfolding's rows
// by i_n and its columns by (i_o, r) with o the third mode. A product splits
// over the slices of mode o:
//   M_n Q = sum_m sum_{i_o} T_{i_o} (T_{i_o}^T Q),   T_{i_o}[i_n][r] = T(m)[..][r].
// A fibre of mode m is a pair (i_hi, i_lo) of the other two coordinates; it
// appears in T(m) as one row of J_m values, and only the fibres that hold a
// nonzero (the fibre list) give nonzero rows. So T(m) is stored compactly:
// row f of Tc(m) is the f-th non-empty fibre, and with o(f), n(f) its
// coordinates in modes o and n,
//   W_{i_o}[r][c] = sum over fibres f with o(f) = i_o of Tc[f][r] Q[n(f)][c]
//   Yf[f][c]      = sum_r Tc[f][r] W_{o(f)}[r][c]
//   (M_n Q)[i][c] = sum over both terms, fibres f with n(f) = i, of Yf[f][c].
// The cost per product is linear in the number of non-empty fibres instead
// of quadratic in I_n: when most fibres are empty (a tensor much sparser than
// its mode sizes squared) the dense projections and the Gram would spend
// nearly all their bytes and flops on zeros.
//
// One workgroup owns a slice i_o of one term: it gathers the slice's fibre
// rows and the matching rows of Q through LDS, accumulates W_{i_o} in
// registers, keeps it in LDS and forms the slice's Yf rows from it, so W
// never goes to memory. A second kernel sums the Yf rows of each i_n (over
// both terms) into the product. Both visit fibres in a fixed order: the
// product is deterministic. Columns go in slabs of 64.
//
// The eigensolver (eig.hip) takes the product as an operator; modes of at
// most 140 rows form M_n explicitly from products with the identity.
// The core G = X x_1 A^T x_2 B^T x_3 C^T comes from Tc(3) (fibres over
// (i_2, i_1)): per slice i_2 the first kernel's W with Q = A gives
// Z[i_2][r][p] = sum_i1 Tc[(i_2, i_1)][r] A[i_1][p], then G from B^T Z.
#include "../../include/tucker.h"
#include "../../include/tucker_implicit.h"
#include "common.h"
#include "guards.h"
#include "timer.h"

#include <hip/hip_ext.h>

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

constexpr int kMaxJi = 128;
constexpr int kGfThreads = 256;
constexpr int kGfCols = 64;    // columns of a slab (one per lane)
constexpr int kGfBatch = 16;   // fibres per batch of a wave
constexpr int kExplicitMax = 140;  // modes up to this size form M_n explicitly

inline int hi_of(int m) { return (m + 2) % 3; }
inline int lo_of(int m) { return (m + 1) % 3; }

// ------------------------------------------------------------------ kernels
template <class A>
__device__ inline A fma_(A a, A b, A c);
template <>
__device__ inline float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ inline double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class A, class T>
__device__ inline A to_acc(T v) { return (A)(float)v; }
template <>
__device__ inline double to_acc<double, double>(double v) { return v; }
template <>
__device__ inline float to_acc<float, double>(double v) { return (float)v; }
template <>
__device__ inline double to_acc<double, float>(float v) { return (double)v; }

// One wave per group (slice i_o) of one term, lane c = column c of the
// slab (Q already offset to it, c < cw). The group's fibres are positions
// [gptr[g], gptr[g+1]) of the grouping, fibre gperm[k] (or k without gperm).
// Lane c keeps column c of W_g = sum_f Tc[f]^T Q[n(f)] in registers (rows
// up to JB >= J; rows beyond J stay zero). Fibres go in batches of kGfBatch:
// the batch's fibre numbers and Q rows are loaded together (independent
// loads in flight at once), its Tc rows staged in the wave's part of LDS and
// read back as broadcasts. The waves of a workgroup run independently (no
// workgroup barrier): a wave's LDS accesses complete in issue order.
// !CORE: second pass over the group, Yf[f * kGfCols + c] = Tc[f] . W_g[:, c].
// CORE: Wout[g * ldw_g + r * ldw_r + c] = W_g[r][c] (zeros for an empty group).
template <class TP, class TQ, class Acc, int JB, bool CORE>
__global__ void __launch_bounds__(kGfThreads) k_gf_wave(const TP *__restrict__ T, int ld, int J,
                                                        const int32_t *__restrict__ gptr,
                                                        const int32_t *__restrict__ gperm,
                                                        const int32_t *__restrict__ fn, const TQ *__restrict__ Q,
                                                        int64_t ldq, int cw, int64_t ngroups, Acc *__restrict__ Yf,
                                                        double *__restrict__ Wout, int64_t ldw_g, int ldw_r) {
    extern __shared__ __attribute__((aligned(16))) char gf_smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * (kGfThreads / 64) + wv;
    if (g >= ngroups) return;
    Acc *sT = reinterpret_cast<Acc *>(gf_smem) + wv * (kGfBatch * JB);  // [kGfBatch][JB]
    const int32_t k0 = gptr[g], k1 = gptr[g + 1];
    if (!CORE && k1 <= k0) return;
    const bool col = lane < cw;
    Acc acc[JB];
#pragma unroll
    for (int r = 0; r < JB; ++r) acc[r] = (Acc)0;
    // stage the batch's Tc rows (fibre of batch slot j held by lane j in fl)
    auto stage = [&](int nc, int32_t fl) {
        for (int e = lane; e < kGfBatch * JB; e += 64) {
            const int j = e / JB, r = e - j * JB;
            const int32_t fj = __shfl(fl, j);
            Acc v = (Acc)0;
            if (j < nc && r < J) v = to_acc<Acc>(T[(int64_t)fj * ld + r]);
            sT[e] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int32_t kb = k0; kb < k1; kb += kGfBatch) {
        const int nc = min(kGfBatch, (int)(k1 - kb));
        int32_t fl = 0, nl = 0;
        if (lane < nc) {
            fl = gperm ? gperm[kb + lane] : kb + lane;
            nl = fn[fl];
        }
        Acc q[kGfBatch];
#pragma unroll
        for (int j = 0; j < kGfBatch; ++j) {
            const int32_t nj = __shfl(nl, j);
            q[j] = (j < nc && col) ? to_acc<Acc>(Q[(int64_t)nj * ldq + lane]) : (Acc)0;
        }
        stage(nc, fl);
#pragma unroll
        for (int j = 0; j < kGfBatch; ++j) {
            if (j < nc) {
                const Acc *t = sT + j * JB;
#pragma unroll
                for (int r = 0; r < JB; ++r) acc[r] = fma_(t[r], q[j], acc[r]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (CORE) {
        if (col)
#pragma unroll
            for (int r = 0; r < JB; ++r)
                if (r < J) Wout[g * ldw_g + (int64_t)r * ldw_r + lane] = (double)acc[r];
        return;
    }
    for (int32_t kb = k0; kb < k1; kb += kGfBatch) {
        const int nc = min(kGfBatch, (int)(k1 - kb));
        int32_t fl = 0;
        if (lane < nc) fl = gperm ? gperm[kb + lane] : kb + lane;
        stage(nc, fl);
#pragma unroll
        for (int j = 0; j < kGfBatch; ++j) {
            if (j < nc) {
                const Acc *t = sT + j * JB;
                Acc y = (Acc)0;
#pragma unroll
                for (int r = 0; r < JB; ++r) y = fma_(t[r], acc[r], y);
                const int32_t fj = __shfl(fl, j);
                if (col) Yf[(int64_t)fj * kGfCols + lane] = y;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Y[i * ldy + c] = sum over the fibres of row i in both terms' groupings of
// Yf_t[f * kGfCols + c] (FP64 sums, fixed order), c < cw.
template <class Acc>
__global__ void __launch_bounds__(256) k_gf_rows(int64_t In, int cw, const int32_t *__restrict__ gp0,
                                                 const int32_t *__restrict__ pm0, const Acc *__restrict__ Y0,
                                                 const int32_t *__restrict__ gp1, const int32_t *__restrict__ pm1,
                                                 const Acc *__restrict__ Y1, double *__restrict__ Y, int64_t ldy) {
    const int c = threadIdx.x & (kGfCols - 1);
    const int64_t i = (int64_t)blockIdx.x * (256 / kGfCols) + threadIdx.x / kGfCols;
    if (i >= In || c >= cw) return;
    double a = 0.0;
    for (int32_t k = gp0[i]; k < gp0[i + 1]; ++k) {
        const int32_t f = pm0 ? pm0[k] : k;
        a += (double)Y0[(int64_t)f * kGfCols + c];
    }
    for (int32_t k = gp1[i]; k < gp1[i + 1]; ++k) {
        const int32_t f = pm1 ? pm1[k] : k;
        a += (double)Y1[(int64_t)f * kGfCols + c];
    }
    Y[i * ldy + c] = a;
}

// hi / lo coordinates of each fibre from its slot.
__global__ void k_fibre_coords(const int32_t *fib, int64_t nf, int32_t Ilo, int32_t *fhi, int32_t *flo) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sl = fib[f];
        fhi[f] = sl / Ilo;
        flo[f] = sl - (sl / Ilo) * Ilo;
    }
}

// gptr[h] = first fibre whose (ascending) hi coordinate is >= h, h <= Ih.
__global__ void k_group_bounds(const int32_t *fhi, int64_t nf, int64_t Ih, int32_t *gptr) {
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h <= Ih; h += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = 0, b = nf;
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if (fhi[mid] < h)
                a = mid + 1;
            else
                b = mid;
        }
        gptr[h] = (int32_t)a;
    }
}

// out[l] = ptr[l * stride] for l <= n.
__global__ void k_stride_gather(const int32_t *ptr, int64_t n, int64_t stride, int32_t *out) {
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l <= n; l += (int64_t)gridDim.x * blockDim.x)
        out[l] = ptr[l * stride];
}

__global__ void k_identity(double *X, int n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
         t += (int64_t)gridDim.x * blockDim.x)
        X[t] = (t / n) == (t % n) ? 1.0 : 0.0;
}

// M = (M + M^T) / 2 (n x n): the products of a reduced-precision operator
// round the two triangles differently.
__global__ void k_symmetrize(double *M, int n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t % n);
        if (i < j) {
            const double v = 0.5 * (M[(int64_t)i * n + j] + M[(int64_t)j * n + i]);
            M[(int64_t)i * n + j] = v;
            M[(int64_t)j * n + i] = v;
        }
    }
}

// core[p][q][r] = G'[q][r][p] (G' = B^T Z, Z[i2][r][p])
__global__ void k_core_from(const double *Gp, double *core, int J0, int J1, int J2) {
    const int64_t tot = (int64_t)J0 * J1 * J2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / ((int64_t)J1 * J2));
        const int rem = (int)(t - (int64_t)p * J1 * J2);
        const int q = rem / J2, r = rem - q * J2;
        core[t] = Gp[((int64_t)q * J2 + r) * J0 + p];
    }
}

__global__ void k_fit_i(const double *nx2, const double *g2, double *fit) {
    const double d = *nx2 - *g2;
    *fit = 1.0 - sqrt(d > 0.0 ? d : 0.0) / sqrt(*nx2);
}

// ------------------------------------------------------------------ plan
struct IPlan {
    int prec = P64;   // element type of the projections
    Tune tune;
    int64_t I[3] = {}, nnz = 0, nslots[3] = {}, cap[3] = {};
    int J[3] = {}, ld[3] = {}, ldc = 0, b[3] = {};
    int64_t nfib[3] = {};
    // device
    int32_t *flags, *nu, *perm, *tmp, *heads, *pos, *counts, *cursor, *scan, *cidx[3];
    double *scal, *partials, *cval;
    int32_t *ptr[3], *lidx[3];
    double *lval64[3];
    float *lval32[3];
    int32_t *fib[3], *fptr[3], *fhi[3], *flo[3], *ghi[3], *glo[3], *plo[3];
    void *T[3];       // compact projections (cap rows of ld)
    float *Tcore;     // mixed: FP32 compact projection of mode 3 for the core (rows of ldc)
    float *Fc;        // mixed: FP32 mode-3 factor padded to ldc
    void *Fp[3];      // padded factor copies (FP64 / FP32 / FP16)
    void *Yf[2];      // per-term fibre rows of a product slab (Acc)
    float *Qc;        // FP32 / BF16 products: the slab of Q in FP32 (rows of 64)
    double *Xblk[3], *theta, *Mg, *Wc, *Gp, *core_split;
    int64_t core_split_elems;
    void *eigw;
    bool blk_ok[3] = {false, false, false};
    int sweep_solves[3] = {0, 0, 0};
    Timer *tm = nullptr;
    int64_t prod_fibres = 0, prod_pairs = 0;  // product kernel launches: fibres, fibres x columns
};

size_t es_of(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }
size_t acc_of(int prec) { return prec == P64 ? 8 : 4; }

void carve(IPlan &p, Arena &ar) {
    const int64_t nnz = std::max<int64_t>(p.nnz, 1);
    int64_t maxslots = 1, maxI = 1, maxcap = 1;
    for (int m = 0; m < 3; ++m) {
        maxslots = std::max(maxslots, p.nslots[m]);
        maxI = std::max(maxI, p.I[m]);
        maxcap = std::max(maxcap, p.cap[m]);
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
    const size_t es = es_of(p.prec);
    for (int m = 0; m < 3; ++m) {
        p.ptr[m] = ar.take<int32_t>(p.nslots[m] + 1);
        p.lidx[m] = ar.take<int32_t>(nnz);
        p.lval64[m] = ar.take<double>(nnz);
        p.lval32[m] = p.prec != P64 ? ar.take<float>(nnz) : nullptr;
        p.fib[m] = ar.take<int32_t>(p.cap[m]);
        p.fptr[m] = ar.take<int32_t>(p.cap[m] + 1);
        p.fhi[m] = ar.take<int32_t>(p.cap[m]);
        p.flo[m] = ar.take<int32_t>(p.cap[m]);
        p.ghi[m] = ar.take<int32_t>(p.I[hi_of(m)] + 1);
        p.glo[m] = ar.take<int32_t>(p.I[lo_of(m)] + 1);
        p.plo[m] = ar.take<int32_t>(p.cap[m]);
        p.T[m] = ar.take<char>(p.cap[m] * p.ld[m] * (int64_t)es);
        p.Fp[m] = ar.take<char>(p.I[m] * p.ld[m] * (int64_t)es);
    }
    p.Tcore = nullptr;
    p.Fc = nullptr;
    if (p.prec == PBF16) {
        p.Tcore = ar.take<float>(p.cap[2] * p.ldc);
        p.Fc = ar.take<float>(p.I[2] * p.ldc);
    }
    for (int t = 0; t < 2; ++t) p.Yf[t] = ar.take<char>(maxcap * kGfCols * (int64_t)acc_of(p.prec));
    p.Qc = p.prec != P64 ? ar.take<float>(maxI * kGfCols) : nullptr;
    size_t ew = 0;
    int bmax = 1;
    for (int n = 0; n < 3; ++n) {
        p.b[n] = eig_block_width((int)p.I[n], p.J[n]);
        bmax = std::max(bmax, p.b[n]);
        p.Xblk[n] = ar.take<double>(p.I[n] * p.b[n]);
        ew = std::max(ew, eig_work_bytes((int)p.I[n], p.b[n]));
    }
    p.eigw = ar.take<char>((int64_t)ew);
    p.theta = ar.take<double>(std::max<int64_t>(bmax, std::min<int64_t>(maxI, kExplicitMax)));
    p.Mg = ar.take<double>((int64_t)kExplicitMax * kExplicitMax);
    const int64_t J0 = p.J[0], J1 = p.J[1], J2 = p.J[2];
    p.Wc = ar.take<double>(p.I[1] * J2 * J0);
    p.Gp = ar.take<double>(J1 * J2 * J0);
    p.core_split_elems = 8 * J1 * J2 * J0;
    p.core_split = ar.take<double>(p.core_split_elems);
}

void plan_init(IPlan &p, const tk_coo *X, const int32_t *J, int precision, const tk_tune *tune) {
    p.prec = precision == TK_FP64 ? P64 : (precision == TK_FP32 ? P32 : PBF16);
    if (tune) {
        if (tune->proj_elems) p.tune.proj_elems = tune->proj_elems;
        if (tune->proj_min_blocks) p.tune.proj_min_blocks = tune->proj_min_blocks;
    }
    p.nnz = X->nnz;
    const int v = (int)(16 / es_of(p.prec));
    for (int n = 0; n < 3; ++n) {
        p.I[n] = X->dims[n];
        p.J[n] = J[n];
        p.ld[n] = (int)ceil_div(J[n], v) * v;
    }
    p.ldc = (int)ceil_div(J[2], 4) * 4;
    for (int m = 0; m < 3; ++m) {
        p.nslots[m] = p.I[hi_of(m)] * p.I[lo_of(m)];
        p.cap[m] = std::max<int64_t>(1, std::min(p.nslots[m], p.nnz));
    }
}

int check(const tk_coo *X, const int32_t *J, const tk_opts *o) {
    if (!X || !J || !o || !X->dims || X->order != 3) return TK_ERR_ARG;
    if (X->nnz < 0 || X->nnz >= (int64_t)INT32_MAX - 1) return TK_ERR_ARG;
    if (X->nnz > 0 && (!X->idx[0] || !X->idx[1] || !X->idx[2] || !X->vals)) return TK_ERR_ARG;
    for (int n = 0; n < 3; ++n) {
        if (X->dims[n] < 1 || X->dims[n] >= INT32_MAX) return TK_ERR_ARG;
        if (J[n] < 1 || J[n] > X->dims[n] || J[n] > kMaxJi) return TK_ERR_ARG;
    }
    for (int m = 0; m < 3; ++m)
        if (X->dims[hi_of(m)] * X->dims[lo_of(m)] >= (int64_t)INT32_MAX) return TK_ERR_ARG;
    if (o->precision != TK_FP64 && o->precision != TK_FP32 && o->precision != TK_MIXED_BF16) return TK_ERR_ARG;
    if (o->init != TK_INIT_RANDOM && o->init != TK_INIT_GIVEN) return TK_ERR_ARG;
    if (o->max_iters < 1 || o->eig_max_iters < 1 || !(o->eig_tol >= 0.0) || std::isnan(o->tol)) return TK_ERR_ARG;
    if (o->hosvd_fit) return TK_ERR_ARG;
    if (o->tune) {
        const tk_tune *t = o->tune;
        auto in = [](int32_t v, int32_t lo, int32_t hi) { return v == 0 || (v >= lo && v <= hi); };
        if (!in(t->proj_elems, 1024, 65536) || !in(t->proj_min_blocks, 64, 16384) || !in(t->gram_items, 64, 16384) ||
            !in(t->gram_min_stages, 1, 64))
            return TK_ERR_ARG;
    }
    return TK_OK;
}

#define IST(call)                         \
    do {                                  \
        hipError_t e_ = (call);           \
        if (e_ != hipSuccess) {           \
            set_hip_error(e_, #call);     \
            return TK_ERR_DEVICE;         \
        }                                 \
    } while (0)

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 65536)); }

// Validation, duplicate summing, the three orderings, their fibre lists and
// groupings, ||X||^2.
int prep(IPlan &p, const tk_coo *X, hipStream_t s, int64_t *nu_out, double *nx2_out) {
    const int64_t dims[3] = {p.I[0], p.I[1], p.I[2]};
    IST(validate(X->idx, X->vals, p.nnz, dims, p.flags, s));
    int32_t flags = 0;
    IST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    IST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    OrderScratch sc{p.counts, p.cursor, p.tmp, p.scan};
    IST(build_order(X->idx, p.nnz, dims, 2, p.ptr[2], p.perm, sc, p.flags, s));
    IST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    IST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    int32_t *cidx[3] = {p.cidx[0], p.cidx[1], p.cidx[2]};
    IST(dedup(X->idx, X->vals, p.nnz, p.perm, p.heads, p.pos, p.scan, cidx, p.cval, p.nu, s));
    int32_t nu = 0;
    IST(hipMemcpyAsync(&nu, p.nu, 4, hipMemcpyDeviceToHost, s));
    IST(hipStreamSynchronize(s));
    IST(sumsq(p.cval, nu, p.partials, p.scal + 0, s));
    const int32_t *cid[3] = {p.cidx[0], p.cidx[1], p.cidx[2]};
    int32_t nfib[3] = {0, 0, 0};
    for (int m = 0; m < 3; ++m) {
        IST(build_order(cid, nu, dims, m, p.ptr[m], p.perm, sc, p.flags, s));
        IST(gather_leaf<double>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval64[m], p.flags, s));
        if (p.lval32[m]) IST(gather_leaf<float>(p.cidx[m], p.cval, p.perm, nu, p.lidx[m], p.lval32[m], p.flags, s));
        IST(fibre_list(p.ptr[m], p.nslots[m], p.cap[m], p.fib[m], p.fptr[m], p.counts, p.cursor, p.scan, p.flags,
                       s));
        IST(hipMemcpyAsync(&nfib[m], p.cursor + p.nslots[m], 4, hipMemcpyDeviceToHost, s));
        IST(hipStreamSynchronize(s));
    }
    double nx2 = 0.0;
    IST(hipMemcpyAsync(&nx2, p.scal + 0, 8, hipMemcpyDeviceToHost, s));
    IST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    IST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    for (int m = 0; m < 3; ++m) {
        p.nfib[m] = nfib[m];
        if (nfib[m] < 0 || nfib[m] > p.cap[m]) return TK_ERR_DEVICE;
    }
    *nu_out = nu;
    *nx2_out = nx2;
    if (!(nx2 > 0.0)) return TK_ERR_EMPTY;
    // fibre coordinates; grouping by the major key (the fibre order itself)
    // and by the minor key: the fibres counting-sorted by the transposed
    // slot i_lo * I_hi + i_hi (one fibre per slot, so the order is fixed),
    // whose slot pointers go to ptr[m] (free once the fibre list exists);
    // the groups start at ptr[m][i_lo * I_hi]
    for (int m = 0; m < 3; ++m) {
        const int64_t nf = p.nfib[m];
        const int64_t Ih = p.I[hi_of(m)], Il = p.I[lo_of(m)];
        k_fibre_coords<<<grid_of(nf), 256, 0, s>>>(p.fib[m], nf, (int32_t)Il, p.fhi[m], p.flo[m]);
        IST(hipGetLastError());
        k_group_bounds<<<grid_of(Ih + 1), 256, 0, s>>>(p.fhi[m], nf, Ih, p.ghi[m]);
        IST(hipGetLastError());
        IST(build_order_keys(p.flo[m], p.fhi[m], p.fhi[m], nf, (int32_t)Ih, p.nslots[m], p.ptr[m], p.plo[m], sc,
                             p.flags, s));
        k_stride_gather<<<grid_of(Il + 1), 256, 0, s>>>(p.ptr[m], Il, Ih, p.glo[m]);
        IST(hipGetLastError());
    }
    IST(hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s));
    IST(hipStreamSynchronize(s));
    if (int r = prep_status(flags)) return r;
    return TK_OK;
}

// Compact projection Tc(m) = rows of X x_m F^T for the non-empty fibres of
// ordering m (the slot form of the projection over the fibre pointers).
hipError_t project_c(IPlan &p, int m, hipStream_t s) {
    const int64_t nf = p.nfib[m];
    const int ld = p.ld[m];
    KernelEvents ke = p.tm ? p.tm->kernel(kProj, m, p.prec) : KernelEvents();
    if (p.prec == P64)
        return project<double, double, double>(p.fptr[m], p.lidx[m], p.lval64[m], (const double *)p.Fp[m], p.I[m],
                                               ld, p.J[m], ld, nf, p.nnz, (double *)p.T[m], s, p.tune, ke);
    if (p.prec == P32)
        return project<float, float, float>(p.fptr[m], p.lidx[m], p.lval32[m], (const float *)p.Fp[m], p.I[m], ld,
                                            p.J[m], ld, nf, p.nnz, (float *)p.T[m], s, p.tune, ke);
    return project<float, f16, bf16>(p.fptr[m], p.lidx[m], p.lval32[m], (const f16 *)p.Fp[m], p.I[m], ld, p.J[m],
                                     ld, nf, p.nnz, (bf16 *)p.T[m], s, p.tune, ke);
}

hipError_t refresh(IPlan &p, int n, const double *F, hipStream_t s) {
    if (p.prec == P64)
        TK_HIP(pad_rows<double>(F, p.I[n], p.J[n], p.ld[n], (double *)p.Fp[n], s));
    else if (p.prec == P32)
        TK_HIP(pad_rows<float>(F, p.I[n], p.J[n], p.ld[n], (float *)p.Fp[n], s));
    else
        TK_HIP(pad_rows<f16>(F, p.I[n], p.J[n], p.ld[n], (f16 *)p.Fp[n], s));
    if (p.Fc && n == 2) TK_HIP(pad_rows<float>(F, p.I[2], p.J[2], p.ldc, p.Fc, s));
    return hipSuccess;
}

// Register rows of a wave's W column: J rounded up to a multiple of 8
// (16 above 64), at most 128.
int jb_of(int J) { return J <= 64 ? (int)ceil_div(J, 8) * 8 : (int)ceil_div(J, 16) * 16; }

template <class K, class... A>
void gf_launch(K kernel, int64_t blocks, size_t lds, hipStream_t s, KernelEvents ke, A... args) {
    lds_limit((const void *)kernel, lds);
    if (ke.start && ke.stop)
        hipExtLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kGfThreads), (uint32_t)lds, s, ke.start, ke.stop,
                              0u, args...);
    else
        kernel<<<(unsigned)blocks, kGfThreads, lds, s>>>(args...);
}

// The wave kernel for J's register rows, one wave per group.
template <class TP, class TQ, class Acc, bool CORE>
hipError_t gf_wave(int J, int64_t ngroups, hipStream_t s, KernelEvents ke, const TP *T, int ld,
                   const int32_t *gptr, const int32_t *gperm, const int32_t *fn, const TQ *Q, int64_t ldq, int cw,
                   Acc *Yf, double *Wout, int64_t ldw_g, int ldw_r) {
    const int JB = jb_of(J);
    const int64_t blocks = ceil_div(ngroups, kGfThreads / 64);
    const size_t lds = (size_t)(kGfThreads / 64) * kGfBatch * JB * sizeof(Acc);
#define TK_GF_CASE(JBV)                                                                                          \
    case JBV:                                                                                                    \
        gf_launch(k_gf_wave<TP, TQ, Acc, JBV, CORE>, blocks, lds, s, ke, T, ld, J, gptr, gperm, fn, Q, ldq, cw, \
                  ngroups, Yf, Wout, ldw_g, ldw_r);                                                              \
        break;
    switch (JB) {
        TK_GF_CASE(8)
        TK_GF_CASE(16)
        TK_GF_CASE(24)
        TK_GF_CASE(32)
        TK_GF_CASE(40)
        TK_GF_CASE(48)
        TK_GF_CASE(56)
        TK_GF_CASE(64)
        TK_GF_CASE(80)
        TK_GF_CASE(96)
        TK_GF_CASE(112)
        TK_GF_CASE(128)
        default:
            return hipErrorInvalidValue;
    }
#undef TK_GF_CASE
    TK_LAUNCHED();
    return hipSuccess;
}

// Qc[i * kGfCols + c] = X[i * ldx + c] (c < cw) in FP32: the gathered rows of
// the FP32 / BF16 products.
__global__ void k_q32(const double *__restrict__ X, int64_t ldx, int64_t n, int cw, float *__restrict__ Qc) {
    const int64_t tot = n * kGfCols;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / kGfCols;
        const int c = (int)(t - i * kGfCols);
        Qc[t] = c < cw ? (float)X[i * ldx + c] : 0.0f;
    }
}

// One Gram term's group kernel over the slices of mode o.
template <class TP, class TQ, class Acc>
hipError_t gf_term(IPlan &p, int m, int n, const TQ *Q, int64_t ldq, int cw, Acc *Yf, hipStream_t s) {
    const int o = 3 - n - m;
    const bool n_hi = hi_of(m) == n;
    const int32_t *gptr = n_hi ? p.glo[m] : p.ghi[m];
    const int32_t *gperm = n_hi ? p.plo[m] : nullptr;
    const int32_t *fn = n_hi ? p.fhi[m] : p.flo[m];
    KernelEvents ke = p.tm ? p.tm->kernel(kGram, n, p.prec) : KernelEvents();
    p.prod_fibres += p.nfib[m];
    p.prod_pairs += p.nfib[m] * cw;
    return gf_wave<TP, TQ, Acc, false>(p.J[m], p.I[o], s, ke, (const TP *)p.T[m], p.ld[m], gptr, gperm, fn, Q, ldq,
                                       cw, Yf, (double *)nullptr, (int64_t)0, 0);
}

template <class TP, class Acc>
hipError_t gf_apply(IPlan &p, int n, const double *X, int64_t ldx, int w, double *Y, int64_t ldy, hipStream_t s) {
    const int m1 = (n + 1) % 3, m2 = (n + 2) % 3;
    for (int c0 = 0; c0 < w; c0 += kGfCols) {
        const int cw = std::min(kGfCols, w - c0);
        if (sizeof(Acc) == 8) {
            TK_HIP((gf_term<TP, double, Acc>(p, m1, n, X + c0, ldx, cw, (Acc *)p.Yf[0], s)));
            TK_HIP((gf_term<TP, double, Acc>(p, m2, n, X + c0, ldx, cw, (Acc *)p.Yf[1], s)));
        } else {
            k_q32<<<grid_of(p.I[n] * kGfCols), 256, 0, s>>>(X + c0, ldx, p.I[n], cw, p.Qc);
            TK_LAUNCHED();
            TK_HIP((gf_term<TP, float, Acc>(p, m1, n, p.Qc, kGfCols, cw, (Acc *)p.Yf[0], s)));
            TK_HIP((gf_term<TP, float, Acc>(p, m2, n, p.Qc, kGfCols, cw, (Acc *)p.Yf[1], s)));
        }
        // rows of n in each term's grouping by n
        const bool h1 = hi_of(m1) == n, h2 = hi_of(m2) == n;
        k_gf_rows<Acc><<<(unsigned)ceil_div(p.I[n], 256 / kGfCols), 256, 0, s>>>(
            p.I[n], cw, h1 ? p.ghi[m1] : p.glo[m1], h1 ? nullptr : p.plo[m1], (const Acc *)p.Yf[0],
            h2 ? p.ghi[m2] : p.glo[m2], h2 ? nullptr : p.plo[m2], (const Acc *)p.Yf[1], Y + c0, ldy);
        TK_LAUNCHED();
    }
    return hipSuccess;
}

struct OpCtx {
    IPlan *p;
    int n;
};

hipError_t op_apply(const void *ctx, const double *X, int64_t ldx, int w, double *Y, int64_t ldy, hipStream_t s) {
    const OpCtx *c = static_cast<const OpCtx *>(ctx);
    IPlan &p = *c->p;
    if (p.prec == P64) return gf_apply<double, double>(p, c->n, X, ldx, w, Y, ldy, s);
    if (p.prec == P32) return gf_apply<float, float>(p, c->n, X, ldx, w, Y, ldy, s);
    return gf_apply<bf16, float>(p, c->n, X, ldx, w, Y, ldy, s);
}

// Leading J_n eigenvectors of M_n into F: through the operator, or from M_n
// formed by products with the identity for small modes.
int run_eig(IPlan &p, int n, double *F, const tk_opts *o, tk_stats *st, int *noconv, hipStream_t s) {
    EigOpts eo;
    eo.max_iters = o->eig_max_iters;
    eo.tol = o->eig_tol > 0 ? o->eig_tol : (p.prec == P64 ? 1e-12 : (p.prec == P32 ? 1e-8 : 1e-4));
    eo.warm = p.blk_ok[n];
    if (eo.warm && p.sweep_solves[n] == 0) eo.warm_degree = eo.degree;
    p.sweep_solves[n] += 1;
    eo.seed = 0x5eed0000ull + (uint64_t)n;
    OpCtx ctx{&p, n};
    EigOp op{op_apply, &ctx};
    const int In = (int)p.I[n];
    double *M = nullptr;
    if (In <= kExplicitMax) {
        k_identity<<<grid_of((int64_t)In * In), 256, 0, s>>>(p.Xblk[n], In);
        IST(hipGetLastError());
        IST(op_apply(&ctx, p.Xblk[n], In, In, p.Mg, In, s));
        if (p.prec != P64) {
            k_symmetrize<<<grid_of((int64_t)In * In), 256, 0, s>>>(p.Mg, In);
            IST(hipGetLastError());
        }
        M = p.Mg;
    } else {
        eo.op = &op;
    }
    int it = 0, nc = 0;
    IST(lead_eig(M, In, p.J[n], p.Xblk[n], F, p.theta, p.eigw, eo, &it, &nc, s));
    if (st) {
        st->eig_iters += it;
        st->eig_noconv += nc;
    }
    if (nc) *noconv = 1;
    p.blk_ok[n] = In > kExplicitMax;
    return TK_OK;
}

// Core from Tc(3): Z[i2][r][p] by the group kernel with Q = A over the
// slices i2 (fibres grouped by the major key), G' = B^T Z, permuted.
hipError_t core_and_fit(IPlan &p, const double *A, const double *B, double *core, hipStream_t s) {
    const int J0 = p.J[0], J1 = p.J[1], J2 = p.J[2];
    const void *Tc = p.prec == PBF16 ? (const void *)p.Tcore : p.T[2];
    const int ldt = p.prec == PBF16 ? p.ldc : p.ld[2];
    for (int c0 = 0; c0 < J0; c0 += kGfCols) {
        const int cw = std::min(kGfCols, J0 - c0);
        if (p.prec == P64)
            TK_HIP((gf_wave<double, double, double, true>(J2, p.I[1], s, KernelEvents(), (const double *)Tc, ldt,
                                                           p.ghi[2], nullptr, p.flo[2], A + c0, (int64_t)J0, cw,
                                                           (double *)nullptr, p.Wc + c0, (int64_t)J2 * J0, J0)));
        else
            TK_HIP((gf_wave<float, double, double, true>(J2, p.I[1], s, KernelEvents(), (const float *)Tc, ldt,
                                                          p.ghi[2], nullptr, p.flo[2], A + c0, (int64_t)J0, cw,
                                                          (double *)nullptr, p.Wc + c0, (int64_t)J2 * J0, J0)));
    }
    GemmArgs h;
    h.M = J1;
    h.N = J2 * J0;
    h.K = (int)p.I[1];
    h.batch = 1;
    h.A = B;
    h.lda = J1;
    h.a_trans = true;
    h.B = p.Wc;
    h.ldb = (int64_t)J2 * J0;
    h.sB = 0;
    h.C = p.Gp;
    h.ldc = (int64_t)J2 * J0;
    h.sC = 0;
    h.prec = P64;
    h.out_type = P64;
    const int tiles = (int)(ceil_div(J1, 64) * ceil_div((int64_t)J2 * J0, 64));
    h.splitk = std::max(1, std::min(8, 256 / std::max(1, tiles)));
    h.split_scratch = p.core_split;
    TK_HIP(gemm(h, s));
    const int64_t nJ = (int64_t)J0 * J1 * J2;
    k_core_from<<<grid_of(nJ), 256, 0, s>>>(p.Gp, core, J0, J1, J2);
    TK_LAUNCHED();
    TK_HIP(sumsq(core, nJ, p.partials, p.scal + 1, s));
    k_fit_i<<<1, 1, 0, s>>>(p.scal + 0, p.scal + 1, p.scal + 2);
    TK_LAUNCHED();
    return hipSuccess;
}

}  // namespace

int mp_implicit_workspace(const tk_coo *X, const int32_t *J, const tk_opts *o, size_t *bytes) {
    if (!bytes) return TK_ERR_ARG;
    int st = check(X, J, o);
    if (st) return st;
    IPlan p;
    plan_init(p, X, J, o->precision, o->tune);
    Arena ar;
    carve(p, ar);
    *bytes = ar.used + 256;
    return TK_OK;
}

int mp_implicit(const tk_coo *X, const int32_t *J, const tk_opts *o, double *core, double *const *F, double *hist,
                int32_t *iters_done, tk_stats *stats, void *ws, size_t wsb, void *stream) {
    int st = check(X, J, o);
    if (st) return st;
    if (!core || !F || !F[0] || !F[1] || !F[2] || !hist || !iters_done) return TK_ERR_ARG;
    IPlan p;
    plan_init(p, X, J, o->precision, o->tune);
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
    Timer tm(o, s);
    if (tm.on) p.tm = &tm;
    const double t0 = now_ms();
    int64_t nu = 0;
    double nx2 = 0.0;
    if ((st = prep(p, X, s, &nu, &nx2))) return st;
    const double t1 = now_ms();
    int noconv = 0;
    for (int n = 1; n < 3; ++n) {
        if (o->init == TK_INIT_RANDOM) IST(random_start_fill(F[n], p.I[n], p.J[n], n, o->seed, s));
        IST(refresh(p, n, F[n], s));
    }
    // projections of the start (untimed, as in the in-core driver)
    Timer *keep = p.tm;
    p.tm = nullptr;
    IST(project_c(p, 1, s));
    IST(project_c(p, 2, s));
    p.tm = keep;
    IST(hipStreamSynchronize(s));
    const double t2 = now_ms();
    double prev = 0.0, g2 = 0.0;
    *iters_done = 0;
    for (int t = 1; t <= o->max_iters; ++t) {
        for (int n = 0; n < 3; ++n) {
            tm.begin(kEig, n, P64);
            if ((st = run_eig(p, n, F[n], o, stats, &noconv, s))) return st;
            tm.end();
            IST(refresh(p, n, F[n], s));
            IST(project_c(p, n, s));
        }
        if (p.Tcore) {
            KernelEvents ke = p.tm ? p.tm->kernel(kProj, 2, P32) : KernelEvents();
            IST((project<float, float, float>(p.fptr[2], p.lidx[2], p.lval32[2], p.Fc, p.I[2], p.ldc, p.J[2], p.ldc,
                                              p.nfib[2], p.nnz, p.Tcore, s, p.tune, ke)));
        }
        tm.begin(kCore, -1, p.prec == P64 ? P64 : P32);
        IST(core_and_fit(p, F[0], F[1], core, s));
        tm.end();
        double gf[2];
        IST(hipMemcpyAsync(gf, p.scal + 1, 16, hipMemcpyDeviceToHost, s));
        IST(hipStreamSynchronize(s));
        tm.collect();
        g2 = gf[0];
        const double fit = gf[1];
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
        tm.report(stats);
        stats->nnz_unique = nu;
        stats->norm_x = std::sqrt(nx2);
        stats->core_norm = std::sqrt(g2);
        stats->product_fibres = p.prod_fibres;
        stats->product_pairs = p.prod_pairs;
    }
    return noconv ? TK_WARN_NOCONV : TK_OK;
}

}  // namespace tk
