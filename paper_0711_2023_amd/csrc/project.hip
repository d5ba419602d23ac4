// Fibre projection: the n-mode product T = X x_m F^T of a sparse tensor with
// a factor matrix (Section 3, n-mode product equation), evaluated on one of
// the fibre orderings. It is the projection that Multislice Projection
// applies to every slice (Figure 7: the products X_::k B, X_:j: C, ...) and
// the first stage of the HOOI tensor-times-matrix chain (Figure 3: U, V, W).
//
// Output layout: T[slot][r] with slot = i_hi * I_lo + i_lo (the two other
// modes; the other three for a fourth-order tensor), r < ldT contiguous; r in
// [J, ldT) is zero padding. The slot form writes every element exactly once,
// empty fibres as zeros; the fibre-list form (the sweeps of MP and SP) walks
// only the non-empty fibres and writes only their rows, into a buffer whose
// other rows were zeroed once.
//
// The kernel is bound by HBM writes of T. A workgroup owns a contiguous run
// of slots (about 32768 output elements). It first stages the run's slot
// pointers and its nonzeros (leaf index, value) in LDS with coalesced loads,
// so the dependent chain pointer -> nonzero -> factor row costs two bulk
// loads per workgroup instead of three trips to memory per element.
//
// Vector form (padded rows): a thread owns one 16-byte column chunk of the
// output for the whole run and walks the run's slots with a fixed stride, so
// no index division remains in the loop; lanes of one slot read one factor
// row (served by L2) and a wave stores 1 KiB of contiguous output. Factor
// rows are read and T written through buffer descriptors with 32-bit
// offsets, whose range check turns the load of an empty fibre into zeros.
// The loop is bound by vector-ALU issue (a wave64 instruction takes four
// cycles), so the per-nonzero work is kept to the address, the LDS read and
// one fused multiply-add per output; with an FP16 factor copy the
// multiply-add takes the FP16 operand directly (mixed FP16/FP32 FMA).
// Nonzeros beyond the LDS capacity (a run with very long fibres) are read
// from global memory.
#include "common.h"

#include <hip/hip_ext.h>

namespace tk {

template <class TA>
struct AccOf { typedef float type; };
template <>
struct AccOf<double> { typedef double type; };

constexpr int kProjThreads = 256;
constexpr int kProjU = 8;          // independent elements per thread per batch (general form)

template <class T>
struct Vec16 { typedef T __attribute__((ext_vector_type(16 / sizeof(T)))) type; };

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Stage the run's slot pointers into LDS: sptr[0..ns]; returns the pointer of
// the run's first nonzero.
__device__ inline int32_t stage_ptr(const int32_t *__restrict__ ptr, int64_t s0, int ns, int32_t *sptr) {
    for (int i = threadIdx.x; i <= ns; i += kProjThreads) sptr[i] = ptr[s0 + i];
    __syncthreads();
    return sptr[0];
}

// Buffer descriptor over [base, base + bytes): a load at or past the end
// returns zeros and a store there is dropped. The range check covers the
// per-lane offset only, so every offset is passed in the per-lane operand.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr uint32_t kOffNone = 0x80000000u;  // past every projection buffer (all are below 2 GiB)

// Nonzero p of the run (p relative to the run's first): staged copy for
// p < nst, else global memory. The LDS read is issued unconditionally at a
// clamped index and the global read is a distinct (streaming) load, so that
// the LDS read stays an LDS access (a read that may come from either space
// would otherwise become one generic load through the vector memory path).
template <class TV>
__device__ inline void nz_at(int p, int nst, int32_t q0, const int32_t *sidx, const TV *sval,
                             const int32_t *__restrict__ lidx, const TV *__restrict__ lval, int32_t &id, TV &v) {
    const int ps = p < nst ? p : 0;
    id = sidx[ps];
    v = sval[ps];
    if (p >= nst) {
        id = __builtin_nontemporal_load(lidx + q0 + p);
        v = __builtin_nontemporal_load(lval + q0 + p);
    }
}

// General form: any row stride; lanes cover consecutive elements. Slots
// with more than maxlen nonzeros are skipped (not written): the long-row
// workgroups of k_project_gen_fused project them. (The body of workgroup
// blk; k_project and k_project_gen_fused launch it.)
template <class TV, class TF, class TO>
__device__ inline void project_gen_body(int64_t blk, const int32_t *__restrict__ ptr,
                                        const int32_t *__restrict__ lidx, const TV *__restrict__ lval,
                                        const TF *__restrict__ F, int32_t ldF, int32_t J, int32_t ldT, int32_t spw,
                                        int32_t cap, int64_t nslots, TO *__restrict__ T, int32_t maxlen) {
    typedef typename AccOf<TV>::type Acc;
    extern __shared__ __attribute__((aligned(16))) int32_t smem[];
    int32_t *sptr = smem, *sidx = smem + ((spw + 4) & ~3);
    TV *sval = reinterpret_cast<TV *>(sidx + ((cap + 3) & ~3));
    const int tid = threadIdx.x;
    const int64_t s0 = blk * spw;
    const int ns = (int)(s0 + spw <= nslots ? spw : nslots - s0);
    const int32_t q0 = stage_ptr(ptr, s0, ns, sptr);
    const int nq = sptr[ns] - q0;
    const int nst = nq < cap ? nq : cap;
    for (int i = tid; i < nst; i += kProjThreads) {
        sidx[i] = lidx[q0 + i];
        sval[i] = lval[q0 + i];
    }
    __syncthreads();
    const int nel = ns * ldT;
    const float rld = 1.0f / (float)ldT;
    TO *out = T + s0 * ldT;
    for (int qb = tid; qb < nel; qb += kProjThreads * kProjU) {
        int r[kProjU], a[kProjU], b[kProjU], id[kProjU];
        bool skip[kProjU];
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
            skip[u] = q < nel && sptr[sl + 1] - sptr[sl] > maxlen;
            if (q < nel && r[u] < J && !skip[u]) {
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
            if (q < nel && !skip[u]) out[q] = (TO)acc[u];
        }
    }
}

template <class TV, class TF, class TO>
__global__ void __launch_bounds__(kProjThreads) k_project(const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ lidx,
                                                          const TV *__restrict__ lval, const TF *__restrict__ F,
                                                          int32_t ldF, int32_t J, int32_t ldT, int32_t spw,
                                                          int32_t cap, int64_t nslots, TO *__restrict__ T) {
    project_gen_body<TV, TF, TO>(blockIdx.x, ptr, lidx, lval, F, ldF, J, ldT, spw, cap, nslots, T, 0x7fffffff);
}

// A slot the general form skips (more than maxlen nonzeros), by one
// workgroup: G = kProjThreads / ldT groups take its nonzeros round robin,
// each thread one column, and the groups' partial rows are summed in LDS in
// group order (fixed: the same bits on every run).
template <class TV, class TF, class TO>
__device__ inline void project_long_rows_body(int64_t blk, const int32_t *__restrict__ ptr,
                                              const int32_t *__restrict__ ls, const int32_t *__restrict__ lidx,
                                              const TV *__restrict__ lval, const TF *__restrict__ F, int32_t ldF,
                                              int32_t J, int32_t ldT, TO *__restrict__ T) {
    typedef typename AccOf<TV>::type Acc;
    extern __shared__ __attribute__((aligned(16))) char long_rows_smem[];
    Acc *red = reinterpret_cast<Acc *>(long_rows_smem);  // [G][ldT]
    const int64_t slot = ls[blk];
    const int a = ptr[slot], b = ptr[slot + 1];
    const int G = kProjThreads / ldT;
    const int tid = threadIdx.x, g = tid / ldT, c = tid - g * ldT;
    Acc acc = (Acc)0;
    if (g < G && c < J)
        for (int p = a + g; p < b; p += G) acc += (Acc)lval[p] * (Acc)F[(int64_t)lidx[p] * ldF + c];
    if (g < G) red[g * ldT + c] = acc;
    __syncthreads();
    if (tid < ldT) {
        Acc sum = red[tid];
        for (int gg = 1; gg < G; ++gg) sum += red[gg * ldT + tid];
        T[slot * ldT + tid] = (TO)sum;
    }
}

// The general form's workgroups (the first nmain) and one workgroup per long
// slot after them, in one launch.
template <class TV, class TF, class TO>
__global__ void __launch_bounds__(kProjThreads) k_project_gen_fused(const int32_t *__restrict__ ptr,
                                                                    const int32_t *__restrict__ lidx,
                                                                    const TV *__restrict__ lval,
                                                                    const TF *__restrict__ F, int32_t ldF, int32_t J,
                                                                    int32_t ldT, int32_t spw, int32_t cap,
                                                                    int64_t nslots, TO *__restrict__ T,
                                                                    int32_t maxlen, const int32_t *__restrict__ ls,
                                                                    int64_t nmain) {
    if ((int64_t)blockIdx.x < nmain)
        project_gen_body<TV, TF, TO>(blockIdx.x, ptr, lidx, lval, F, ldF, J, ldT, spw, cap, nslots, T, maxlen);
    else
        project_long_rows_body<TV, TF, TO>((int64_t)blockIdx.x - nmain, ptr, ls, lidx, lval, F, ldF, J, ldT, T);
}

// A staged nonzero: leaf index and value side by side (one LDS read).
template <class TV>
struct NzPair;
template <>
struct NzPair<float> { int32_t i; float v; };
template <>
struct NzPair<double> { int32_t i; int32_t pad; double v; };

// Unstaged nonzero p of the run, through descriptors over the run's index and
// value arrays (a buffer load, which cannot merge with the LDS read of the
// staged case).
__device__ inline void nz_global(__amdgpu_buffer_rsrc_t ri, __amdgpu_buffer_rsrc_t rv, int p, NzPair<float> &e) {
    e.i = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ri, (uint32_t)p * 4u, 0, 0);
    e.v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rv, (uint32_t)p * 4u, 0, 0));
}
__device__ inline void nz_global(__amdgpu_buffer_rsrc_t ri, __amdgpu_buffer_rsrc_t rv, int p, NzPair<double> &e) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    e.i = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(ri, (uint32_t)p * 4u, 0, 0);
    e.v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, (uint32_t)p * 8u, 0, 0));
}

__device__ inline float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc[t] (+)= v * F entry t of the 16-byte loads x (FP16 / BF16 / FP32 / FP64 rows).
template <class TF, int NL, class Acc, bool FIRST>
__device__ inline void fma_row(const u32x4 (&x)[NL], Acc v, Acc *acc) {
    constexpr int FPV = 16 / sizeof(TF);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const typename Vec16<TF>::type f = __builtin_bit_cast(typename Vec16<TF>::type, x[l]);
#pragma unroll
        for (int t = 0; t < FPV; ++t)  // the first as a fused product with zero: one mixed FMA for FP16 rows
            acc[l * FPV + t] = fused(v, (Acc)f[t], FIRST ? (Acc)0 : acc[l * FPV + t]);
    }
}

template <int NL>
__device__ inline void load_row(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x4 (&x)[NL]) {
#pragma unroll
    for (int l = 0; l < NL; ++l) x[l] = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16 * l, 0, 0);
}

// Row strides of T and F equal (ldT) and a multiple of 16 bytes of T, F's
// padding columns zero, F below 2 GiB with fewer than 2^24 rows: each thread
// produces whole 16-byte chunks of T. SPLIT: T receives each output rounded
// to TO and Tlo the rounded remainder (the value minus its rounded part), so
// T + Tlo carries about twice the significand bits of TO.
// FIB: the units of a run are the non-empty fibres of the ordering (ptr is
// the fibre pointer list, fib[f] the slot of fibre f, nslots their number)
// and only their rows are written; the rows of empty fibres keep what the
// buffer holds (zeros written once before the first such projection). Else
// the units are all slots and empty ones are written as zeros. Units (fibres
// or slots) with more than maxlen nonzeros are skipped (not written): the
// long-fibre workgroups of k_project_fused project them.
// DUAL (FP32 output): each chunk is also written rounded to BF16 into T2,
// whose rows have stride ld2 (ldT or ldT + 4, a multiple of 8; the same
// fibre's row, its last 4 columns written as zeros when ld2 > ldT), so that
// one pass over the nonzeros serves both an FP32 and a BF16 consumer.
// (The body of workgroup blk; k_project_vec and k_project_fused launch it.)
template <class TV, class TF, class TO, bool SPLIT, bool FIB, bool DUAL>
__device__ inline void project_vec_body(int64_t blk, const int32_t *__restrict__ ptr,
                                        const int32_t *__restrict__ fib, const int32_t *__restrict__ lidx,
                                        const TV *__restrict__ lval, const TF *__restrict__ F, uint32_t Fbytes,
                                        int32_t J, int32_t ldT, int32_t spw, int32_t cap, int64_t nslots,
                                        TO *__restrict__ T, TO *__restrict__ Tlo, bf16 *__restrict__ T2, int32_t ld2,
                                        int32_t maxlen) {
    typedef typename AccOf<TV>::type Acc;
    constexpr int V = 16 / sizeof(TO);              // outputs per chunk
    constexpr int NL = V * (int)sizeof(TF) / 16;    // 16-byte factor loads per chunk
    extern __shared__ __attribute__((aligned(16))) int32_t smem[];
    int32_t *sptr = smem;
    int32_t *sfib = smem + ((spw + 4) & ~3);  // FIB: slots of the run's fibres
    NzPair<TV> *snz = reinterpret_cast<NzPair<TV> *>(smem + ((spw + 4) & ~3) + (FIB ? ((spw + 3) & ~3) : 0));
    const int tid = threadIdx.x;
    const int64_t s0 = blk * spw;
    const int ns = (int)(s0 + spw <= nslots ? spw : nslots - s0);
    // The run's first and end nonzero straight from memory (uniform across
    // the workgroup: the descriptors below must be scalar), so that loading
    // the nonzeros waits for nothing but these; then every staging load of a
    // thread (pointers, fibre slots, nonzeros, SU of each per pass) is in
    // flight before its LDS writes: one or two trips to memory per run
    // instead of one per element a thread stages.
    const int32_t q0 = __builtin_amdgcn_readfirstlane(ptr[s0]);
    const int nq = __builtin_amdgcn_readfirstlane(ptr[s0 + ns] - q0);
    const int nst = nq < cap ? nq : cap;
    constexpr int SU = 4;
    for (int i0 = tid; i0 <= ns || i0 < nst; i0 += SU * kProjThreads) {
        int32_t pv[SU], fv[SU];
        NzPair<TV> e[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = i0 + u * kProjThreads;
            pv[u] = i <= ns ? ptr[s0 + i] : 0;
            fv[u] = FIB && i < ns ? fib[s0 + i] : 0;
            e[u] = NzPair<TV>{};
            if (i < nst) {
                e[u].i = lidx[q0 + i];
                e[u].v = lval[q0 + i];
            }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int i = i0 + u * kProjThreads;
            if (i <= ns) sptr[i] = pv[u];
            if (FIB && i < ns) sfib[i] = fv[u];
            if (i < nst) snz[i] = e[u];
        }
    }
    __syncthreads();
    const int cps = ldT / V;            // chunks per slot
    const int spi = kProjThreads / cps; // slots per pass of the workgroup
    const int tsl = tid / cps, r = tid - tsl * cps;
    if (tsl >= spi) return;
    const bool col_on = r * V < J;
    const uint32_t rowb = (uint32_t)ldT * sizeof(TF), coloff = (uint32_t)r * V * sizeof(TF);
    const __amdgpu_buffer_rsrc_t fr = buf_rsrc(F, Fbytes);
    // output rows of the run: slots [row0, row0 + nrows); under FIB the span
    // of the run's fibres, whose 32-bit byte size the host has checked
    const int64_t row0 = FIB ? (int64_t)__builtin_amdgcn_readfirstlane(sfib[0]) : s0;
    const int64_t nrows = FIB ? (int64_t)__builtin_amdgcn_readfirstlane(sfib[ns - 1]) + 1 - row0 : ns;
    const uint32_t outb = (uint32_t)nrows * (uint32_t)ldT * sizeof(TO);
    const __amdgpu_buffer_rsrc_t orr = buf_rsrc(T + row0 * ldT, outb);
    const __amdgpu_buffer_rsrc_t ri = buf_rsrc(lidx + q0, (uint32_t)nq * 4u);
    const __amdgpu_buffer_rsrc_t rv = buf_rsrc(lval + q0, (uint32_t)nq * (uint32_t)sizeof(TV));
    // the output chunk of unit sl (slot or fibre)
    auto store = [&](int sl, const Acc *acc) {
        const int orow = FIB ? (int)(sfib[sl] - row0) : sl;
        const uint32_t off = (uint32_t)(orow * cps + r) * 16u;
        typename Vec16<TO>::type o;
#pragma unroll
        for (int t = 0; t < V; ++t) o[t] = (TO)acc[t];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, o), orr, off, 0, 0);
        if (SPLIT) {
            typename Vec16<TO>::type o2;
#pragma unroll
            for (int t = 0; t < V; ++t) o2[t] = (TO)(acc[t] - (Acc)o[t]);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, o2), buf_rsrc(Tlo + row0 * ldT, outb), off,
                                                   0, 0);
        }
        if (DUAL) {  // V = 4 FP32 outputs -> 4 BF16 (8 bytes)
            typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            bf16x4 h;
#pragma unroll
            for (int t = 0; t < 4; ++t) h[t] = (bf16)acc[t];
            const uint32_t off2 = ((uint32_t)orow * (uint32_t)ld2 + (uint32_t)r * 4u) * 2u;
            const __amdgpu_buffer_rsrc_t r2 = buf_rsrc(T2 + row0 * ld2, (uint32_t)nrows * (uint32_t)ld2 * 2u);
            if (r == cps - 1 && ld2 > ldT) {
                // the row's last chunk also writes the zero padding columns
                // (4, then 8 per further store): whole rows, with no holes
                // that split the memory lines
                const u32x2 hv = __builtin_bit_cast(u32x2, h);
                __builtin_amdgcn_raw_buffer_store_b128(u32x4{hv[0], hv[1], 0u, 0u}, r2, off2, 0, 0);
                for (uint32_t z = 16u; z < (uint32_t)(ld2 - ldT + 4) * 2u; z += 16u)
                    __builtin_amdgcn_raw_buffer_store_b128(u32x4{0u, 0u, 0u, 0u}, r2, off2 + z, 0, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, h), r2, off2, 0, 0);
            }
        }
    };
    // one unit of the run, with any of its nonzeros read from global memory
    // when they lie beyond the staged ones
    auto one = [&](int sl) {
        // a unit longer than maxlen belongs to a long-fibre workgroup
        // (project_long_body)
        if (sptr[sl + 1] - sptr[sl] > maxlen) return;
        int a = 0, b = 0;
        if (col_on) {
            a = sptr[sl] - q0;
            b = sptr[sl + 1] - q0;
        }
        // first nonzero; an empty fibre loads zeros from past the end of F
        NzPair<TV> e = snz[a < nst ? a : 0];
        if (a < b && a >= nst) nz_global(ri, rv, a, e);
        Acc acc[V];
        {
            u32x4 x[NL];
            load_row<NL>(fr, a < b ? __umul24((uint32_t)e.i, rowb) + coloff : kOffNone, x);
            fma_row<TF, NL, Acc, true>(x, a < b ? (Acc)e.v : (Acc)0, acc);
        }
        if (b <= nst) {
            for (int p = a + 1; p < b; ++p) {
                const NzPair<TV> e2 = snz[p];
                u32x4 x[NL];
                load_row<NL>(fr, __umul24((uint32_t)e2.i, rowb) + coloff, x);
                fma_row<TF, NL, Acc, false>(x, (Acc)e2.v, acc);
            }
        } else {
            for (int p = a + 1; p < b; ++p) {
                NzPair<TV> e2 = snz[p < nst ? p : 0];
                if (p >= nst) nz_global(ri, rv, p, e2);
                u32x4 x[NL];
                load_row<NL>(fr, __umul24((uint32_t)e2.i, rowb) + coloff, x);
                fma_row<TF, NL, Acc, false>(x, (Acc)e2.v, acc);
            }
        }
        store(sl, acc);
    };
    for (int sl = tsl; sl < ns; sl += spi) one(sl);
}

template <class TV, class TF, class TO, bool SPLIT = false, bool FIB = false, bool DUAL = false>
__global__ void __launch_bounds__(kProjThreads) k_project_vec(const int32_t *__restrict__ ptr,
                                                              const int32_t *__restrict__ fib,
                                                              const int32_t *__restrict__ lidx,
                                                              const TV *__restrict__ lval,
                                                              const TF *__restrict__ F, uint32_t Fbytes, int32_t J,
                                                              int32_t ldT, int32_t spw, int32_t cap, int64_t nslots,
                                                              TO *__restrict__ T, TO *__restrict__ Tlo,
                                                              bf16 *__restrict__ T2, int32_t ld2,
                                                              int32_t maxlen) {
    project_vec_body<TV, TF, TO, SPLIT, FIB, DUAL>(blockIdx.x, ptr, fib, lidx, lval, F, Fbytes, J, ldT, spw, cap,
                                                   nslots, T, Tlo, T2, ld2, maxlen);
}

// Threads of a long-fibre workgroup (64 and 128 measured slower on the
// Zipf-skewed 1000^3 tensor: 66-116 and 58-90 us per projection against
// 61-79 us).
constexpr int kLongThreads = 256;

// The fibres the vector kernel skips (more than maxlen nonzeros): one
// workgroup per fibre of the list lf (k_project_fused). Its threads are
// (group, chunk) pairs: the fibre's nonzeros are dealt round robin to
// G = kLongThreads / cps groups, each thread accumulates its 16-byte output
// chunk over its group's nonzeros, and the G partial rows are summed in LDS
// in group order (a fixed order, the same bits on every run), then written
// as the vector kernel writes a row (SPLIT: rounded part and remainder;
// DUAL: also the BF16 copy, its padding columns zero).
template <class TV, class TF, class TO, bool SPLIT, bool DUAL>
__device__ inline void project_long_body(int64_t blk, const int32_t *__restrict__ fptr,
                                         const int32_t *__restrict__ fib, const int32_t *__restrict__ lf,
                                         const int32_t *__restrict__ lidx, const TV *__restrict__ lval,
                                         const TF *__restrict__ F, uint32_t Fbytes, int32_t J, int32_t ldT,
                                         TO *__restrict__ T, TO *__restrict__ Tlo, bf16 *__restrict__ T2,
                                         int32_t ld2) {
    typedef typename AccOf<TV>::type Acc;
    constexpr int V = 16 / sizeof(TO);
    constexpr int NL = V * (int)sizeof(TF) / 16;
    extern __shared__ __attribute__((aligned(16))) char long_smem[];
    Acc *red = reinterpret_cast<Acc *>(long_smem);  // [G][ldT]
    const int f = lf[blk];
    const int a = fptr[f], b = fptr[f + 1];
    const int64_t row = fib ? fib[f] : f;  // a slot list names the rows itself
    const int cps = ldT / V, G = kLongThreads / cps;
    const int tid = threadIdx.x, g = tid / cps, r = tid - g * cps;
    const uint32_t rowb = (uint32_t)ldT * sizeof(TF), coloff = (uint32_t)r * V * sizeof(TF);
    const __amdgpu_buffer_rsrc_t fr = buf_rsrc(F, Fbytes);
    Acc acc[V];
#pragma unroll
    for (int t = 0; t < V; ++t) acc[t] = (Acc)0;
    if (g < G && r * V < J) {
        for (int p = a + g; p < b; p += G) {
            u32x4 x[NL];
            load_row<NL>(fr, __umul24((uint32_t)lidx[p], rowb) + coloff, x);
            fma_row<TF, NL, Acc, false>(x, (Acc)lval[p], acc);
        }
    }
    if (g < G)
#pragma unroll
        for (int t = 0; t < V; ++t) red[g * ldT + r * V + t] = acc[t];
    __syncthreads();
    if (tid >= cps) return;
    Acc sum[V];
#pragma unroll
    for (int t = 0; t < V; ++t) sum[t] = red[tid * V + t];
    for (int gg = 1; gg < G; ++gg)
#pragma unroll
        for (int t = 0; t < V; ++t) sum[t] += red[gg * ldT + tid * V + t];
    typename Vec16<TO>::type o;
#pragma unroll
    for (int t = 0; t < V; ++t) o[t] = (TO)sum[t];
    *reinterpret_cast<typename Vec16<TO>::type *>(T + row * ldT + tid * V) = o;
    if (SPLIT) {
        typename Vec16<TO>::type o2;
#pragma unroll
        for (int t = 0; t < V; ++t) o2[t] = (TO)(sum[t] - (Acc)o[t]);
        *reinterpret_cast<typename Vec16<TO>::type *>(Tlo + row * ldT + tid * V) = o2;
    }
    if (DUAL) {  // V = 4 FP32 outputs -> 4 BF16, the row's last chunk with the padding zeros
        typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 h;
#pragma unroll
        for (int t = 0; t < 4; ++t) h[t] = (bf16)sum[t];
        bf16 *dst = T2 + row * ld2 + tid * 4;
        *reinterpret_cast<bf16x4 *>(dst) = h;
        if (tid == cps - 1)
            for (int c = ldT; c < ld2; c += 4) *reinterpret_cast<bf16x4 *>(T2 + row * ld2 + c) = bf16x4{0, 0, 0, 0};
    }
}

// The vector kernel's workgroups over the fibre list (the first nmain) and
// one workgroup per long fibre after them, in one launch, so that the long
// fibres run beside the tail of the rest instead of after it. Without FIB
// the units are all slots and lf lists long slots (fib null).
static_assert(kLongThreads == kProjThreads, "one launch: the same workgroup size");
template <class TV, class TF, class TO, bool SPLIT = false, bool DUAL = false, bool FIB = true>
__global__ void __launch_bounds__(kProjThreads) k_project_fused(const int32_t *__restrict__ fptr,
                                                                const int32_t *__restrict__ fib,
                                                                const int32_t *__restrict__ lidx,
                                                                const TV *__restrict__ lval,
                                                                const TF *__restrict__ F, uint32_t Fbytes, int32_t J,
                                                                int32_t ldT, int32_t spw, int32_t cap, int64_t nfib,
                                                                TO *__restrict__ T, TO *__restrict__ Tlo,
                                                                bf16 *__restrict__ T2, int32_t ld2, int32_t maxlen,
                                                                const int32_t *__restrict__ lf, int64_t nmain) {
    if ((int64_t)blockIdx.x < nmain)
        project_vec_body<TV, TF, TO, SPLIT, FIB, DUAL>(blockIdx.x, fptr, fib, lidx, lval, F, Fbytes, J, ldT, spw,
                                                       cap, nfib, T, Tlo, T2, ld2, maxlen);
    else
        project_long_body<TV, TF, TO, SPLIT, DUAL>((int64_t)blockIdx.x - nmain, fptr, fib, lf, lidx, lval, F, Fbytes,
                                                   J, ldT, T, Tlo, T2, ld2);
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

// Run length and staging capacity of a projection launch.
struct ProjShape {
    int spw, cap;
    int64_t blocks;
};
static ProjShape proj_shape(int64_t nslots, int ld, const Tune &tn, int cap_max) {
    // runs of slots: large enough to amortise the staging, small enough that
    // the grid still fills the chip
    int spw = (int)std::min<int64_t>(tn.proj_elems / ld, ceil_div(nslots, tn.proj_min_blocks));
    if (spw < 1) spw = 1;
    if (spw > 4096) spw = 4096;
    // staged nonzeros: room for 4 per slot on average; longer runs read the
    // rest from global memory
    int cap = spw * 4 < 256 ? 256 : spw * 4;
    if (cap > cap_max) cap = cap_max;
    return {spw, cap, ceil_div(nslots, spw)};
}

// The vector form's conditions beyond equal, 16-byte padded rows: 32-bit
// buffer offsets for F, the run's output and its nonzeros, 24-bit row
// indices, and a chunk column per thread.
template <class TV, class TF, class TO>
static bool vec_ok(const TF *F, int64_t rowsF, int ld, const void *T, int spw, int64_t nnz) {
    const int V = 16 / (int)sizeof(TO);
    return ld % V == 0 && ld / V <= kProjThreads && ((uintptr_t)F & 15) == 0 && ((uintptr_t)T & 15) == 0 &&
           rowsF < (int64_t(1) << 24) && rowsF * ld * (int64_t)sizeof(TF) < (int64_t(1) << 31) &&
           (int64_t)spw * ld * (int64_t)sizeof(TO) < (int64_t(1) << 31) &&
           nnz * (int64_t)sizeof(TV) < (int64_t(1) << 32);
}

// Launch on s, through the extended launch when the caller asked for the
// kernel's own start / end events.
template <class K, class... A>
static void launch(K kernel, int64_t blocks, size_t lds, hipStream_t s, KernelEvents ke, A... args) {
    if (ke.start && ke.stop)
        hipExtLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kProjThreads), (uint32_t)lds, s, ke.start, ke.stop,
                              0u, args...);
    else
        kernel<<<(unsigned)blocks, kProjThreads, lds, s>>>(args...);
}

// LDS of a long-fibre launch: G partial rows of ldT accumulators.
template <class TV, class TO>
static size_t long_lds(int ldT) {
    const int V = 16 / (int)sizeof(TO), cps = ldT / V;
    return (size_t)(kLongThreads / cps) * ldT * sizeof(typename AccOf<TV>::type);
}

// A fibre list is usable when the whole output fits 32-bit buffer offsets
// (a run's rows may then span any part of it).
template <class TO>
static bool fib_ok(const FibreList &fl, int64_t nslots, int ld) {
    return fl.fib && fl.fptr && nslots * (int64_t)ld * (int64_t)sizeof(TO) < (int64_t(1) << 31);
}

// LDS bytes of a vector launch: staged pointers (and fibre slots), nonzeros.
template <class TV>
static size_t vec_lds(const ProjShape &sh, bool fib) {
    return sizeof(int32_t) * (((sh.spw + 4) & ~3) + (fib ? ((sh.spw + 3) & ~3) : 0)) +
           sizeof(NzPair<TV>) * (size_t)sh.cap;
}

template <class TV, class TF, class TO>
hipError_t project(const int32_t *ptr, const int32_t *lidx, const TV *lval, const TF *F, int64_t rowsF, int ldF,
                   int J, int ldT, int64_t nslots, int64_t nnz, TO *T, hipStream_t s, const Tune &tn,
                   KernelEvents ke, FibreList fl) {
    if (nslots <= 0 || ldT <= 0) return hipSuccess;
    if (ldF == ldT && vec_ok<TV, TF, TO>(F, rowsF, ldT, T, proj_shape(nslots, ldT, tn, 4096).spw, nnz)) {
        // pairs of 16 bytes for FP64 values: at most 2048 staged (32 KiB)
        const int cap_max = sizeof(TV) == 8 ? 2048 : 4096;
        const uint32_t Fb = (uint32_t)(rowsF * ldT * (int64_t)sizeof(TF));
        if (fib_ok<TO>(fl, nslots, ldT)) {
            if (fl.n <= 0) return hipSuccess;  // no nonzeros: every row keeps its zeros
            const ProjShape sh = proj_shape(fl.n, ldT, tn, cap_max);
            if (fl.nlong > 0)
                launch(k_project_fused<TV, TF, TO>, sh.blocks + fl.nlong,
                       std::max(vec_lds<TV>(sh, true), long_lds<TV, TO>(ldT)), s, ke, fl.fptr, fl.fib, lidx, lval, F,
                       Fb, (int32_t)J, (int32_t)ldT, (int32_t)sh.spw, (int32_t)sh.cap, fl.n, T, (TO *)nullptr,
                       (bf16 *)nullptr, (int32_t)0, fl.maxlen, fl.lf, sh.blocks);
            else
                launch(k_project_vec<TV, TF, TO, false, true>, sh.blocks, vec_lds<TV>(sh, true), s, ke, fl.fptr,
                       fl.fib, lidx, lval, F, Fb, (int32_t)J, (int32_t)ldT, (int32_t)sh.spw, (int32_t)sh.cap, fl.n,
                       T, (TO *)nullptr, (bf16 *)nullptr, (int32_t)0, fl.maxlen);
        } else {
            const ProjShape sh = proj_shape(nslots, ldT, tn, cap_max);
            if (fl.nls > 0)  // long slots: their own workgroups in the same launch
                launch(k_project_fused<TV, TF, TO, false, false, false>, sh.blocks + fl.nls,
                       std::max(vec_lds<TV>(sh, false), long_lds<TV, TO>(ldT)), s, ke, ptr, (const int32_t *)nullptr,
                       lidx, lval, F, Fb, (int32_t)J, (int32_t)ldT, (int32_t)sh.spw, (int32_t)sh.cap, nslots, T,
                       (TO *)nullptr, (bf16 *)nullptr, (int32_t)0, fl.slot_maxlen, fl.ls, sh.blocks);
            else
                launch(k_project_vec<TV, TF, TO, false, false>, sh.blocks, vec_lds<TV>(sh, false), s, ke, ptr,
                       (const int32_t *)nullptr, lidx, lval, F, Fb, (int32_t)J, (int32_t)ldT, (int32_t)sh.spw,
                       (int32_t)sh.cap, nslots, T, (TO *)nullptr, (bf16 *)nullptr, (int32_t)0,
                       (int32_t)0x7fffffff);
        }
    } else {
        const ProjShape sh = proj_shape(nslots, ldT, tn, 4096);
        const size_t lds = sizeof(int32_t) * (((sh.spw + 4) & ~3) + ((sh.cap + 3) & ~3)) + sizeof(TV) * sh.cap;
        if (fl.nls > 0 && ldT <= kProjThreads)  // long slots: their own workgroups in the same launch
            launch(k_project_gen_fused<TV, TF, TO>, sh.blocks + fl.nls,
                   std::max(lds, (size_t)(kProjThreads / ldT) * ldT * sizeof(typename AccOf<TV>::type)), s, ke, ptr,
                   lidx, lval, F, (int32_t)ldF, (int32_t)J, (int32_t)ldT, (int32_t)sh.spw, (int32_t)sh.cap, nslots,
                   T, fl.slot_maxlen, fl.ls, sh.blocks);
        else
            launch(k_project<TV, TF, TO>, sh.blocks, lds, s, ke, ptr, lidx, lval, F, (int32_t)ldF, (int32_t)J,
                   (int32_t)ldT, (int32_t)sh.spw, (int32_t)sh.cap, nslots, T);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

bool project_dual_ok(const float *F, int64_t rowsF, int ld, const float *T, const bf16 *T2, int ld2,
                     int64_t nslots, int64_t nnz, const Tune &tn, const FibreList &fl) {
    return nslots > 0 && ld > 0 &&
           vec_ok<float, float, float>(F, rowsF, ld, T, proj_shape(nslots, ld, tn, 4096).spw, nnz) &&
           ((uintptr_t)T2 & 15) == 0 && (ld2 == ld || (ld2 >= ld + 4 && (ld2 - ld - 4) % 8 == 0)) && ld2 % 8 == 0 &&
           fib_ok<float>(fl, nslots, ld) &&
           nslots * (int64_t)ld2 * 2 < (int64_t(1) << 31);
}

hipError_t project_dual(const int32_t *ptr, const int32_t *lidx, const float *lval, const float *F, int64_t rowsF,
                        int ld, int J, int64_t nslots, int64_t nnz, float *T, bf16 *T2, int ld2, hipStream_t s,
                        const Tune &tn, KernelEvents ke, FibreList fl) {
    (void)ptr;
    if (!project_dual_ok(F, rowsF, ld, T, T2, ld2, nslots, nnz, tn, fl)) return hipErrorInvalidValue;
    if (fl.n <= 0) return hipSuccess;  // no nonzeros: every row keeps its zeros
    const uint32_t Fb = (uint32_t)(rowsF * ld * (int64_t)sizeof(float));
    const ProjShape sh = proj_shape(fl.n, ld, tn, 4096);
    if (fl.nlong > 0)
        launch(k_project_fused<float, float, float, false, true>, sh.blocks + fl.nlong,
               std::max(vec_lds<float>(sh, true), long_lds<float, float>(ld)), s, ke, fl.fptr, fl.fib, lidx, lval, F,
               Fb, (int32_t)J, (int32_t)ld, (int32_t)sh.spw, (int32_t)sh.cap, fl.n, T, (float *)nullptr, T2,
               (int32_t)ld2, fl.maxlen, fl.lf, sh.blocks);
    else
        launch(k_project_vec<float, float, float, false, true, true>, sh.blocks, vec_lds<float>(sh, true), s, ke,
               fl.fptr, fl.fib, lidx, lval, F, Fb, (int32_t)J, (int32_t)ld, (int32_t)sh.spw, (int32_t)sh.cap, fl.n,
               T, (float *)nullptr, T2, (int32_t)ld2, fl.maxlen);
    TK_LAUNCHED();
    return hipSuccess;
}

hipError_t project_split(const int32_t *ptr, const int32_t *lidx, const float *lval, const float *F, int64_t rowsF,
                         int ld, int J, int64_t nslots, int64_t nnz, bf16 *Thi, bf16 *Tlo, hipStream_t s,
                         const Tune &tn, KernelEvents ke, FibreList fl) {
    if (nslots <= 0 || ld <= 0) return hipSuccess;
    if (!vec_ok<float, float, bf16>(F, rowsF, ld, Thi, proj_shape(nslots, ld, tn, 4096).spw, nnz) ||
        ((uintptr_t)Tlo & 15) != 0)
        return hipErrorInvalidValue;
    const uint32_t Fb = (uint32_t)(rowsF * ld * (int64_t)sizeof(float));
    if (fib_ok<bf16>(fl, nslots, ld)) {
        if (fl.n <= 0) return hipSuccess;
        const ProjShape sh = proj_shape(fl.n, ld, tn, 4096);
        if (fl.nlong > 0)
            launch(k_project_fused<float, float, bf16, true>, sh.blocks + fl.nlong,
                   std::max(vec_lds<float>(sh, true), long_lds<float, bf16>(ld)), s, ke, fl.fptr, fl.fib, lidx, lval,
                   F, Fb, (int32_t)J, (int32_t)ld, (int32_t)sh.spw, (int32_t)sh.cap, fl.n, Thi, Tlo,
                   (bf16 *)nullptr, (int32_t)0, fl.maxlen, fl.lf, sh.blocks);
        else
            launch(k_project_vec<float, float, bf16, true, true>, sh.blocks, vec_lds<float>(sh, true), s, ke,
                   fl.fptr, fl.fib, lidx, lval, F, Fb, (int32_t)J, (int32_t)ld, (int32_t)sh.spw, (int32_t)sh.cap,
                   fl.n, Thi, Tlo, (bf16 *)nullptr, (int32_t)0, fl.maxlen);
    } else {
        const ProjShape sh = proj_shape(nslots, ld, tn, 4096);
        launch(k_project_vec<float, float, bf16, true, false>, sh.blocks, vec_lds<float>(sh, false), s, ke, ptr,
               (const int32_t *)nullptr, lidx, lval, F, Fb, (int32_t)J, (int32_t)ld, (int32_t)sh.spw,
               (int32_t)sh.cap, nslots, Thi, Tlo, (bf16 *)nullptr, (int32_t)0,
               (int32_t)0x7fffffff);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

#define TK_PROJECT(TV, TF, TO)                                                                                 \
    template hipError_t project<TV, TF, TO>(const int32_t *, const int32_t *, const TV *, const TF *, int64_t, int, \
                                            int, int, int64_t, int64_t, TO *, hipStream_t, const Tune &,       \
                                            KernelEvents, FibreList);
TK_PROJECT(double, double, double)
TK_PROJECT(float, float, float)
TK_PROJECT(float, float, bf16)
TK_PROJECT(float, f16, bf16)
#undef TK_PROJECT
template hipError_t pad_rows<double>(const double *, int64_t, int, int, double *, hipStream_t);
template hipError_t pad_rows<f16>(const double *, int64_t, int, int, f16 *, hipStream_t);
template hipError_t pad_rows<float>(const double *, int64_t, int, int, float *, hipStream_t);

}  // namespace tk
