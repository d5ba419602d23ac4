// Fibre projection: the n-mode product T = X x_m F^T of a sparse tensor with
// a factor matrix (Section 3, n-mode product equation), evaluated on one of
// the fibre orderings. It is the projection that Multislice Projection
// applies to every slice (Figure 7: the products X_::k B, X_:j: C, ...) and
// the first stage of the HOOI tensor-times-matrix chain (Figure 3: U, V, W).
//
// Output layout: T[slot][r] with slot = i_hi * I_lo + i_lo (the two other
// modes), r < ldT contiguous; r in [J, ldT) is zero padding; every element
// is written exactly once, empty fibres as zeros.
//
// The kernel is bound by HBM writes of T. A workgroup owns a contiguous run
// of slots (about 8192 output elements). It first stages the run's slot
// pointers and its nonzeros (leaf index, value) in LDS with coalesced loads,
// so the dependent chain pointer -> nonzero -> factor row costs two bulk
// loads per workgroup instead of three trips to memory per element. Then
// lanes cover consecutive output elements: lanes in the same slot read the
// same staged nonzeros and consecutive entries of a factor row (coalesced,
// served by L2), and stores write contiguous memory. Each thread takes its
// elements in batches of 8 and issues the factor loads of a batch together. Nonzeros beyond the LDS
// capacity (a run with very long fibres) are read from global memory.
#include "common.h"

namespace tk {

template <class TA>
struct AccOf { typedef float type; };
template <>
struct AccOf<double> { typedef double type; };

constexpr int kProjThreads = 256;
constexpr int kProjU = 8;          // independent elements per thread per batch (general form)
constexpr int kProjUV = 2;         // independent 16-byte chunks per thread per batch (vector form)

template <class TO>
struct Vec16;
template <>
struct Vec16<double> { typedef double __attribute__((ext_vector_type(2))) type; };
template <>
struct Vec16<float> { typedef float __attribute__((ext_vector_type(4))) type; };
template <>
struct Vec16<bf16> { typedef bf16 __attribute__((ext_vector_type(8))) type; };

// Stage the run's slot pointers and nonzeros into LDS: sptr[0..ns], then up to
// cap nonzeros. Returns the number staged.
template <class TV>
__device__ inline int stage_run(const int32_t *__restrict__ ptr, const int32_t *__restrict__ lidx,
                                const TV *__restrict__ lval, int64_t s0, int ns, int cap, int32_t *sptr,
                                int32_t *sidx, TV *sval, int32_t &q0) {
    const int tid = threadIdx.x;
    for (int i = tid; i <= ns; i += kProjThreads) sptr[i] = ptr[s0 + i];
    __syncthreads();
    q0 = sptr[0];
    const int nq = sptr[ns] - q0;
    const int nst = nq < cap ? nq : cap;
    for (int i = tid; i < nst; i += kProjThreads) {
        sidx[i] = lidx[q0 + i];
        sval[i] = lval[q0 + i];
    }
    __syncthreads();
    return nst;
}

template <class TV>
__device__ inline void nz_at(int p, int nst, int32_t q0, const int32_t *sidx, const TV *sval,
                             const int32_t *__restrict__ lidx, const TV *__restrict__ lval, int32_t &id, TV &v) {
    if (p < nst) {
        id = sidx[p];
        v = sval[p];
    } else {
        id = lidx[q0 + p];
        v = lval[q0 + p];
    }
}

// General form: any row stride; lanes cover consecutive elements.
template <class TV, class TF, class TO>
__global__ void __launch_bounds__(kProjThreads) k_project(const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ lidx,
                                                          const TV *__restrict__ lval, const TF *__restrict__ F,
                                                          int32_t ldF, int32_t J, int32_t ldT, int32_t spw,
                                                          int32_t cap,
                                                          int64_t nslots, TO *__restrict__ T) {
    typedef typename AccOf<TV>::type Acc;
    extern __shared__ __attribute__((aligned(16))) int32_t smem[];
    int32_t *sptr = smem, *sidx = smem + ((spw + 4) & ~3);
    TV *sval = reinterpret_cast<TV *>(sidx + ((cap + 3) & ~3));
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * spw;
    const int ns = (int)(s0 + spw <= nslots ? spw : nslots - s0);
    int32_t q0;
    const int nst = stage_run(ptr, lidx, lval, s0, ns, cap, sptr, sidx, sval, q0);
    const int nel = ns * ldT;
    const float rld = 1.0f / (float)ldT;
    TO *out = T + s0 * ldT;
    for (int qb = tid; qb < nel; qb += kProjThreads * kProjU) {
        int r[kProjU], a[kProjU], b[kProjU], id[kProjU];
        Acc acc[kProjU];
        TV v[kProjU];
#pragma unroll
        for (int u = 0; u < kProjU; ++u) {
            const int q = qb + u * kProjThreads;
            int sl = (int)((float)q * rld);
            if (sl * ldT > q) --sl;
            if ((sl + 1) * ldT <= q) ++sl;
            r[u] = q - sl * ldT;
            a[u] = 0;
            b[u] = 0;
            if (q < nel && r[u] < J) {
                a[u] = sptr[sl] - q0;
                b[u] = sptr[sl + 1] - q0;
            }
            id[u] = 0;
            v[u] = 0;
            if (a[u] < b[u]) nz_at(a[u], nst, q0, sidx, sval, lidx, lval, id[u], v[u]);
        }
#pragma unroll
        for (int u = 0; u < kProjU; ++u)
            acc[u] = a[u] < b[u] ? (Acc)v[u] * (Acc)F[(int64_t)id[u] * ldF + r[u]] : (Acc)0;
#pragma unroll
        for (int u = 0; u < kProjU; ++u)
            for (int p = a[u] + 1; p < b[u]; ++p) {
                int32_t i2;
                TV v2;
                nz_at(p, nst, q0, sidx, sval, lidx, lval, i2, v2);
                acc[u] += (Acc)v2 * (Acc)F[(int64_t)i2 * ldF + r[u]];
            }
#pragma unroll
        for (int u = 0; u < kProjU; ++u) {
            const int q = qb + u * kProjThreads;
            if (q < nel) out[q] = (TO)acc[u];
        }
    }
}

// Row strides of T and F equal and a multiple of 16 bytes, F's padding
// columns zero: each thread produces whole 16-byte chunks of T, which never
// cross a slot, from 16-byte loads of F rows and one vector store per chunk.
// SPLIT: T receives each output rounded to TO and Tlo the rounded remainder
// (the value minus its rounded part), so T + Tlo carries about twice the
// significand bits of TO.
template <class TV, class TF, class TO, bool SPLIT = false>
__global__ void __launch_bounds__(kProjThreads) k_project_vec(const int32_t *__restrict__ ptr,
                                                              const int32_t *__restrict__ lidx,
                                                              const TV *__restrict__ lval,
                                                              const TF *__restrict__ F, int32_t J, int32_t ldT,
                                                              int32_t spw, int32_t cap, int64_t nslots,
                                                              TO *__restrict__ T, TO *__restrict__ Tlo = nullptr) {
    typedef typename AccOf<TV>::type Acc;
    typedef typename Vec16<TF>::type FV;
    constexpr int V = 16 / sizeof(TO);            // outputs per chunk
    constexpr int FPV = 16 / sizeof(TF);          // factor entries per 16-byte load
    constexpr int NL = V / FPV;                   // loads per chunk
    constexpr int U = kProjUV;
    extern __shared__ __attribute__((aligned(16))) int32_t smem[];
    int32_t *sptr = smem, *sidx = smem + ((spw + 4) & ~3);
    TV *sval = reinterpret_cast<TV *>(sidx + ((cap + 3) & ~3));
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * spw;
    const int ns = (int)(s0 + spw <= nslots ? spw : nslots - s0);
    int32_t q0;
    const int nst = stage_run(ptr, lidx, lval, s0, ns, cap, sptr, sidx, sval, q0);
    const int cps = ldT / V;  // chunks per slot
    const int nch = ns * cps;
    const float rcps = 1.0f / (float)cps;
    TO *out = T + s0 * ldT;
    for (int cb = tid; cb < nch; cb += kProjThreads * U) {
        int r0[U], a[U], b[U], id[U];
        TV v[U];
        Acc acc[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = cb + u * kProjThreads;
            int sl = (int)((float)c * rcps);
            if (sl * cps > c) --sl;
            if ((sl + 1) * cps <= c) ++sl;
            r0[u] = (c - sl * cps) * V;
            a[u] = 0;
            b[u] = 0;
            if (c < nch && r0[u] < J) {
                a[u] = sptr[sl] - q0;
                b[u] = sptr[sl + 1] - q0;
            }
            id[u] = 0;
            v[u] = 0;
            if (a[u] < b[u]) nz_at(a[u], nst, q0, sidx, sval, lidx, lval, id[u], v[u]);
        }
        FV f[U][NL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int l = 0; l < NL; ++l)
                f[u][l] = a[u] < b[u] ? *reinterpret_cast<const FV *>(F + (int64_t)id[u] * ldT + r0[u] + l * FPV)
                                      : FV(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int l = 0; l < NL; ++l)
#pragma unroll
                for (int t = 0; t < FPV; ++t) acc[u][l * FPV + t] = (Acc)v[u] * (Acc)f[u][l][t];
#pragma unroll
        for (int u = 0; u < U; ++u)
            for (int p = a[u] + 1; p < b[u]; ++p) {
                int32_t i2;
                TV v2;
                nz_at(p, nst, q0, sidx, sval, lidx, lval, i2, v2);
                const FV *row = reinterpret_cast<const FV *>(F + (int64_t)i2 * ldT + r0[u]);
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    const FV g = row[l];
#pragma unroll
                    for (int t = 0; t < FPV; ++t) acc[u][l * FPV + t] += (Acc)v2 * (Acc)g[t];
                }
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = cb + u * kProjThreads;
            if (c < nch) {
                typename Vec16<TO>::type o;
#pragma unroll
                for (int t = 0; t < V; ++t) o[t] = (TO)acc[u][t];
                *reinterpret_cast<typename Vec16<TO>::type *>(out + (int64_t)c * V) = o;
                if (SPLIT) {
                    typename Vec16<TO>::type o2;
#pragma unroll
                    for (int t = 0; t < V; ++t) o2[t] = (TO)(acc[u][t] - (Acc)o[t]);
                    *reinterpret_cast<typename Vec16<TO>::type *>(Tlo + s0 * ldT + (int64_t)c * V) = o2;
                }
            }
        }
    }
}

template <class TO>
__device__ inline TO from_f64(double x) { return (TO)(float)x; }
template <>
__device__ inline double from_f64<double>(double x) { return x; }

template <class TO>
__global__ void k_pad_rows(const double *__restrict__ in, int64_t rows, int J, int ld, TO *__restrict__ out) {
    const int64_t n = rows * ld;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / ld;
        const int r = (int)(q - i * ld);
        out[q] = r < J ? from_f64<TO>(in[i * J + r]) : (TO)0;
    }
}

template <class TO>
hipError_t pad_rows(const double *in, int64_t rows, int J, int ld, TO *out, hipStream_t s) {
    const int64_t n = rows * ld;
    if (n <= 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(ceil_div(n, 256), 4096);
    k_pad_rows<TO><<<(unsigned)g, 256, 0, s>>>(in, rows, J, ld, out);
    TK_LAUNCHED();
    return hipSuccess;
}

template <class TV, class TF, class TO>
hipError_t project(const int32_t *ptr, const int32_t *lidx, const TV *lval, const TF *F, int ldF, int J, int ldT,
                   int64_t nslots, TO *T, hipStream_t s, const Tune &tn) {
    if (nslots <= 0 || ldT <= 0) return hipSuccess;
    // runs of slots: large enough to amortise the staging, small enough that
    // the grid still fills the chip
    int spw = (int)std::min<int64_t>(tn.proj_elems / ldT, ceil_div(nslots, tn.proj_min_blocks));
    if (spw < 1) spw = 1;
    if (spw > 4096) spw = 4096;
    // staged nonzeros: room for 4 per slot on average (at most 4096, so LDS
    // stays under 64 KiB); longer runs read the rest from global memory
    int cap = spw * 4 < 256 ? 256 : spw * 4;
    if (cap > 4096) cap = 4096;
    const size_t lds = sizeof(int32_t) * (((spw + 4) & ~3) + ((cap + 3) & ~3)) + sizeof(TV) * cap;
    const int64_t blocks = ceil_div(nslots, spw);
    const bool vec = ldF == ldT && ldT % (16 / (int)sizeof(TO)) == 0 && ((uintptr_t)F & 15) == 0 &&
                     ((uintptr_t)T & 15) == 0;
    if (vec)
        k_project_vec<TV, TF, TO><<<(unsigned)blocks, kProjThreads, lds, s>>>(ptr, lidx, lval, F, J, ldT, spw, cap,
                                                                             nslots, T);
    else
        k_project<TV, TF, TO><<<(unsigned)blocks, kProjThreads, lds, s>>>(ptr, lidx, lval, F, ldF, J, ldT, spw,
                                                                         cap, nslots, T);
    TK_LAUNCHED();
    return hipSuccess;
}

hipError_t project_split(const int32_t *ptr, const int32_t *lidx, const float *lval, const float *F, int ld, int J,
                         int64_t nslots, bf16 *Thi, bf16 *Tlo, hipStream_t s, const Tune &tn) {
    if (nslots <= 0 || ld <= 0) return hipSuccess;
    if (ld % 8 != 0 || ((uintptr_t)F & 15) != 0 || ((uintptr_t)Thi & 15) != 0 || ((uintptr_t)Tlo & 15) != 0)
        return hipErrorInvalidValue;
    int spw = (int)std::min<int64_t>(tn.proj_elems / ld, ceil_div(nslots, tn.proj_min_blocks));
    if (spw < 1) spw = 1;
    if (spw > 4096) spw = 4096;
    int cap = spw * 4 < 256 ? 256 : spw * 4;
    if (cap > 4096) cap = 4096;
    const size_t lds = sizeof(int32_t) * (((spw + 4) & ~3) + ((cap + 3) & ~3)) + sizeof(float) * cap;
    const int64_t blocks = ceil_div(nslots, spw);
    k_project_vec<float, float, bf16, true><<<(unsigned)blocks, kProjThreads, lds, s>>>(ptr, lidx, lval, F, J, ld,
                                                                                       spw, cap, nslots, Thi, Tlo);
    TK_LAUNCHED();
    return hipSuccess;
}

template hipError_t project<double, double, double>(const int32_t *, const int32_t *, const double *, const double *,
                                                    int, int, int, int64_t, double *, hipStream_t, const Tune &);
template hipError_t project<float, float, float>(const int32_t *, const int32_t *, const float *, const float *, int,
                                                 int, int, int64_t, float *, hipStream_t, const Tune &);
template hipError_t project<float, float, bf16>(const int32_t *, const int32_t *, const float *, const float *, int,
                                                int, int, int64_t, bf16 *, hipStream_t, const Tune &);
template hipError_t project<float, bf16, bf16>(const int32_t *, const int32_t *, const float *, const bf16 *, int,
                                               int, int, int64_t, bf16 *, hipStream_t, const Tune &);
template hipError_t pad_rows<double>(const double *, int64_t, int, int, double *, hipStream_t);
template hipError_t pad_rows<bf16>(const double *, int64_t, int, int, bf16 *, hipStream_t);
template hipError_t pad_rows<float>(const double *, int64_t, int, int, float *, hipStream_t);

}  // namespace tk
