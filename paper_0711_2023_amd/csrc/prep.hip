// Preparation of a sparse third-order tensor on the GPU: validation, the
// three fibre orderings that replace the paper's per-mode sort and slice
// files (Section 4.3, slice construction; appendix), duplicate summing, the
// squared norm, and the unfolding Gram X_(n) X_(n)^T used by the HO-SVD
// initialisation (Figure 1; Figure 3 initialisation; Figure 7 pseudo HO-SVD,
// whose Gram is exactly twice this one).
//
// Every reduction here is deterministic: integer atomics only count, and
// floating-point sums run in an order fixed by the data.
#include "common.h"
#include "guards.h"

#include <cmath>

namespace tk {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
static int grid_for(int64_t n, int threads = 256) {
    int64_t g = ceil_div(n, threads);
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}
hipError_t fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n), 256, 0, s>>>(p, n, v);
    TK_LAUNCHED();
    return hipSuccess;
}
hipError_t fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_f64<<<grid_for(n), 256, 0, s>>>(p, n, v);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ scan
// Three phases: per-chunk sums, one-block scan of the chunk sums, per-chunk
// exclusive scan plus offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ inline int32_t wave_incl_scan(int32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive block scan of one value per thread (blocks of up to 1024
// threads, 16 waves); returns the block total. The total has a slot of its
// own: with 16 waves every entry of wsum is a wave prefix.
__device__ inline int32_t block_excl_scan(int32_t x, int32_t &excl) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t wtotal;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int32_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < nw; ++i) {
            int32_t t = wsum[i];
            wsum[i] = run;
            run += t;
        }
        wtotal = run;
    }
    __syncthreads();
    excl = inc - x + wsum[w];
    int32_t total = wtotal;
    __syncthreads();
    return total;
}

__global__ void k_chunk_sums(const int32_t *in, int64_t n, int32_t *sums) {
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int32_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) t += in[base + i];
    int32_t ex;
    int32_t tot = block_excl_scan(t, ex);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of sums[0..nb) in place; sums[nb] = total.
__global__ void k_scan_sums(int32_t *sums, int64_t nb) {
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < nb ? sums[i] : 0;
        int32_t ex;
        int32_t tot = block_excl_scan(v, ex);
        if (i < nb) sums[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void k_scan_apply(const int32_t *in, int64_t n, const int32_t *sums, int32_t *out) {
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        t += v[i];
    }
    int32_t ex;
    block_excl_scan(t, ex);
    int32_t run = ex + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        int64_t nb = gridDim.x;
        out[n] = sums[nb];
    }
}

int64_t scan_scratch_ints(int64_t n) { return ceil_div(n > 0 ? n : 1, kScanChunk) + 1; }

hipError_t scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s) {
    if (n <= 0) {
        return fill_i32(out, 1, 0, s);
    }
    int64_t nb = ceil_div(n, kScanChunk);
    k_chunk_sums<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, scratch);
    TK_LAUNCHED();
    k_scan_sums<<<1, 1024, 0, s>>>(scratch, nb);
    TK_LAUNCHED();
    k_scan_apply<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, scratch, out);
    TK_LAUNCHED();
    return hipSuccess;
}

// ---------------------------------------------------------------- fibre lists
// The non-empty fibres of an ordering (slots holding at least one entry), in
// slot order: fib[f] = slot, fptr[f] = its first entry, fptr[F] = the total.
__global__ void k_fibre_flags(const int32_t *__restrict__ ptr, int64_t nslots, int32_t *__restrict__ flag) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nslots; q += (int64_t)gridDim.x * blockDim.x)
        flag[q] = ptr[q + 1] > ptr[q] ? 1 : 0;
}

__global__ void k_fibre_scatter(const int32_t *__restrict__ ptr, const int32_t *__restrict__ pos, int64_t nslots,
                                int64_t cap, int32_t *__restrict__ fib, int32_t *__restrict__ fptr,
                                int32_t *__restrict__ flags) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t q = tid; q < nslots; q += (int64_t)gridDim.x * blockDim.x) {
        if (ptr[q + 1] > ptr[q]) {
            const int32_t f = pos[q];
            if (f >= 0 && (int64_t)f < cap) {
                fib[f] = (int32_t)q;
                fptr[f] = ptr[q];
            } else {
                atomicOr(flags, kFlagOrderCheck);
            }
        }
    }
    if (tid == 0) {
        const int32_t total = pos[nslots];
        if (total >= 0 && (int64_t)total <= cap)
            fptr[total] = ptr[nslots];
        else
            atomicOr(flags, kFlagOrderCheck);
    }
}

hipError_t fibre_list(const int32_t *ptr, int64_t nslots, int64_t cap, int32_t *fib, int32_t *fptr, int32_t *flag_tmp,
                      int32_t *pos_tmp, int32_t *scan_scratch, int32_t *flags, hipStream_t s) {
    if (nslots <= 0) return fill_i32(pos_tmp, 1, 0, s);
    k_fibre_flags<<<grid_for(nslots), 256, 0, s>>>(ptr, nslots, flag_tmp);
    TK_LAUNCHED();
    TK_HIP(scan_exclusive(flag_tmp, pos_tmp, nslots, scan_scratch, s));
    k_fibre_scatter<<<grid_for(nslots), 256, 0, s>>>(ptr, pos_tmp, nslots, cap, fib, fptr, flags);
    TK_LAUNCHED();
    return hipSuccess;
}

__global__ void k_long_flags(const int32_t *__restrict__ fptr, int64_t n, int32_t maxlen, int32_t *__restrict__ flag) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n; f += (int64_t)gridDim.x * blockDim.x)
        flag[f] = fptr[f + 1] - fptr[f] > maxlen ? 1 : 0;
}

__global__ void k_long_scatter(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t n,
                               int64_t cap, int32_t *__restrict__ lf, int32_t *__restrict__ flags) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        if (flag[f]) {
            const int32_t k = pos[f];
            if (k >= 0 && (int64_t)k < cap)
                lf[k] = (int32_t)f;
            else
                atomicOr(flags, kFlagOrderCheck);
        }
    }
}

hipError_t long_fibres(const int32_t *fptr, int64_t n, int32_t maxlen, int64_t cap, int32_t *lf, int32_t *flag_tmp,
                       int32_t *pos_tmp, int32_t *scan_scratch, int32_t *flags, hipStream_t s) {
    if (n <= 0) return fill_i32(pos_tmp, 1, 0, s);
    k_long_flags<<<grid_for(n), 256, 0, s>>>(fptr, n, maxlen, flag_tmp);
    TK_LAUNCHED();
    TK_HIP(scan_exclusive(flag_tmp, pos_tmp, n, scan_scratch, s));
    k_long_scatter<<<grid_for(n), 256, 0, s>>>(flag_tmp, pos_tmp, n, cap, lf, flags);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ validation
__global__ void k_validate(const int32_t *i0, const int32_t *i1, const int32_t *i2, const double *v, int64_t nnz,
                           int32_t I0, int32_t I1, int32_t I2, int32_t *flags) {
    int bad = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        if ((uint32_t)i0[p] >= (uint32_t)I0 || (uint32_t)i1[p] >= (uint32_t)I1 || (uint32_t)i2[p] >= (uint32_t)I2)
            bad |= 1;
        if (!isfinite(v[p])) bad |= 2;
    }
    uint64_t any1 = __ballot(bad & 1), any2 = __ballot(bad & 2);
    if ((threadIdx.x & 63) == 0 && (any1 | any2)) atomicOr(flags, (any1 ? 1 : 0) | (any2 ? 2 : 0));
}

hipError_t validate(const int32_t *const idx[3], const double *vals, int64_t nnz, const int64_t dims[3],
                    int32_t *flags, hipStream_t s) {
    TK_HIP(fill_i32(flags, 1, 0, s));
    if (nnz == 0) return hipSuccess;
    k_validate<<<grid_for(nnz), 256, 0, s>>>(idx[0], idx[1], idx[2], vals, nnz, (int32_t)dims[0], (int32_t)dims[1],
                                              (int32_t)dims[2], flags);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ orderings
__global__ void k_slot_hist(const int32_t *ihi, const int32_t *ilo, int64_t nnz, int32_t Ilo, int32_t *counts) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&counts[ihi[p] * Ilo + ilo[p]], 1);
}

// Entry p goes to ptr[slot] + (its arrival rank in the slot). A position
// outside the slot's range (which a wrong scan would produce) is not
// written; it raises kFlagOrderCheck, as does a scan total other than nnz.
__global__ void k_slot_scatter(const int32_t *ihi, const int32_t *ilo, int64_t nnz, int32_t Ilo, int64_t nslots,
                               const int32_t *ptr, int32_t *cursor, int32_t *tmp, int32_t *flags) {
    const bool total_ok = order_total_ok(ptr[nslots], nnz);
    int bad = total_ok ? 0 : 1;
    if (total_ok) {
        for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
             p += (int64_t)gridDim.x * blockDim.x) {
            int32_t slot = ihi[p] * Ilo + ilo[p];
            int32_t b = ptr[slot], e = ptr[slot + 1];
            int64_t pos = (int64_t)b + atomicAdd(&cursor[slot], 1);
            if (order_pos_ok(pos, b, e, nnz))
                tmp[pos] = (int32_t)p;
            else
                bad = 1;
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, kFlagOrderCheck);
}

// The order inside a slot is fixed by the key (i_m, input position), which
// is unique, so the result does not depend on the atomic order above.
// Skipped entirely when the scatter raised kFlagOrderCheck (tmp is then not
// a permutation).
__global__ void k_slot_rank(const int32_t *ihi, const int32_t *ilo, const int32_t *im, int64_t nnz, int32_t Ilo,
                            const int32_t *ptr, const int32_t *tmp, int32_t *perm, const int32_t *flags) {
    if (*flags & kFlagOrderCheck) return;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = tmp[q];
        int32_t slot = ihi[p] * Ilo + ilo[p];
        int32_t b = ptr[slot], e = ptr[slot + 1];
        int32_t key = im[p];
        int32_t rank = 0;
        for (int32_t r = b; r < e; ++r) {
            int32_t p2 = tmp[r];
            int32_t k2 = im[p2];
            rank += (k2 < key) || (k2 == key && p2 < p);
        }
        perm[b + rank] = p;
    }
}

hipError_t build_order_keys(const int32_t *ihi, const int32_t *ilo, const int32_t *im, int64_t nnz, int32_t Ilo,
                            int64_t nslots, int32_t *ptr, int32_t *perm, OrderScratch sc, int32_t *flags,
                            hipStream_t s) {
    TK_HIP(fill_i32(sc.counts, nslots, 0, s));
    TK_HIP(fill_i32(sc.cursor, nslots, 0, s));
    if (nnz > 0) {
        k_slot_hist<<<grid_for(nnz), 256, 0, s>>>(ihi, ilo, nnz, Ilo, sc.counts);
        TK_LAUNCHED();
    }
    TK_HIP(scan_exclusive(sc.counts, ptr, nslots, sc.scan, s));
    if (nnz > 0) {
        k_slot_scatter<<<grid_for(nnz), 256, 0, s>>>(ihi, ilo, nnz, Ilo, nslots, ptr, sc.cursor, sc.tmp, flags);
        TK_LAUNCHED();
        k_slot_rank<<<grid_for(nnz), 256, 0, s>>>(ihi, ilo, im, nnz, Ilo, ptr, sc.tmp, perm, flags);
        TK_LAUNCHED();
    }
    return hipSuccess;
}

hipError_t build_order(const int32_t *const idx[3], int64_t nnz, const int64_t dims[3], int m, int32_t *ptr,
                       int32_t *perm, OrderScratch sc, int32_t *flags, hipStream_t s) {
    const int hi = (m + 2) % 3, lo = (m + 1) % 3;
    return build_order_keys(idx[hi], idx[lo], idx[m], nnz, (int32_t)dims[lo], dims[hi] * dims[lo], ptr, perm, sc,
                            flags, s);
}


// ------------------------------------------------------------------ duplicates
__global__ void k_heads(const int32_t *i0, const int32_t *i1, const int32_t *i2, const int32_t *perm, int64_t nnz,
                        int32_t *heads) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t h = 1;
        if (q > 0) {
            int32_t p = perm[q], r = perm[q - 1];
            h = (i0[p] != i0[r]) || (i1[p] != i1[r]) || (i2[p] != i2[r]);
        }
        heads[q] = h;
    }
}

__global__ void k_dedup_write(const int32_t *i0, const int32_t *i1, const int32_t *i2, const double *vals,
                              const int32_t *perm, const int32_t *heads, const int32_t *pos, int64_t nnz, int32_t *c0,
                              int32_t *c1, int32_t *c2, double *cval) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        if (!heads[q]) continue;
        int32_t p = perm[q];
        double sum = vals[p];
        for (int64_t r = q + 1; r < nnz && !heads[r]; ++r) sum += vals[perm[r]];
        int32_t u = pos[q];
        c0[u] = i0[p];
        c1[u] = i1[p];
        c2[u] = i2[p];
        cval[u] = sum;
    }
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst) { *dst = *src; }

hipError_t dedup(const int32_t *const idx[3], const double *vals, int64_t nnz, const int32_t *perm, int32_t *heads,
                 int32_t *pos, int32_t *scan_scratch, int32_t *const cidx[3], double *cval, int32_t *nu_dev,
                 hipStream_t s) {
    if (nnz == 0) return fill_i32(nu_dev, 1, 0, s);
    k_heads<<<grid_for(nnz), 256, 0, s>>>(idx[0], idx[1], idx[2], perm, nnz, heads);
    TK_LAUNCHED();
    TK_HIP(scan_exclusive(heads, pos, nnz, scan_scratch, s));
    k_dedup_write<<<grid_for(nnz), 256, 0, s>>>(idx[0], idx[1], idx[2], vals, perm, heads, pos, nnz, cidx[0], cidx[1],
                                                cidx[2], cval);
    TK_LAUNCHED();
    k_copy_i32<<<1, 1, 0, s>>>(pos + nnz, nu_dev);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ order N
// out[p] = a[p] * Ib + b[p]: two coordinates merged into one key digit.
__global__ void k_merge_keys(const int32_t *a, const int32_t *b, int64_t nnz, int32_t Ib, int32_t *out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        out[p] = a[p] * Ib + b[p];
}

hipError_t merge_keys(const int32_t *a, const int32_t *b, int64_t nnz, int32_t Ib, int32_t *out, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    k_merge_keys<<<grid_for(nnz), 256, 0, s>>>(a, b, nnz, Ib, out);
    TK_LAUNCHED();
    return hipSuccess;
}

__global__ void k_validate_n(CoordsN c, const double *v, int64_t nnz, int32_t *flags) {
    int bad = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < c.n; ++k)
            if ((uint32_t)c.i[k][p] >= (uint32_t)c.dim[k]) bad |= 1;
        if (!isfinite(v[p])) bad |= 2;
    }
    uint64_t any1 = __ballot(bad & 1), any2 = __ballot(bad & 2);
    if ((threadIdx.x & 63) == 0 && (any1 | any2)) atomicOr(flags, (any1 ? 1 : 0) | (any2 ? 2 : 0));
}

hipError_t validate_n(CoordsN c, const double *vals, int64_t nnz, int32_t *flags, hipStream_t s) {
    TK_HIP(fill_i32(flags, 1, 0, s));
    if (nnz == 0) return hipSuccess;
    k_validate_n<<<grid_for(nnz), 256, 0, s>>>(c, vals, nnz, flags);
    TK_LAUNCHED();
    return hipSuccess;
}

__global__ void k_heads_n(CoordsN c, const int32_t *perm, int64_t nnz, int32_t *heads) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t h = 1;
        if (q > 0) {
            const int32_t p = perm[q], r = perm[q - 1];
            h = 0;
            for (int k = 0; k < c.n; ++k) h |= c.i[k][p] != c.i[k][r];
        }
        heads[q] = h;
    }
}

__global__ void k_dedup_write_n(CoordsN c, const double *vals, const int32_t *perm, const int32_t *heads,
                                const int32_t *pos, int64_t nnz, CoordsOut out, double *cval) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        if (!heads[q]) continue;
        const int32_t p = perm[q];
        double sum = vals[p];
        for (int64_t r = q + 1; r < nnz && !heads[r]; ++r) sum += vals[perm[r]];
        const int32_t u = pos[q];
        for (int k = 0; k < c.n; ++k) out.i[k][u] = c.i[k][p];
        cval[u] = sum;
    }
}

hipError_t dedup_n(CoordsN c, const double *vals, int64_t nnz, const int32_t *perm, int32_t *heads, int32_t *pos,
                   int32_t *scan_scratch, CoordsOut out, double *cval, int32_t *nu_dev, hipStream_t s) {
    if (nnz == 0) return fill_i32(nu_dev, 1, 0, s);
    k_heads_n<<<grid_for(nnz), 256, 0, s>>>(c, perm, nnz, heads);
    TK_LAUNCHED();
    TK_HIP(scan_exclusive(heads, pos, nnz, scan_scratch, s));
    k_dedup_write_n<<<grid_for(nnz), 256, 0, s>>>(c, vals, perm, heads, pos, nnz, out, cval);
    TK_LAUNCHED();
    k_copy_i32<<<1, 1, 0, s>>>(pos + nnz, nu_dev);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ leaf gather
// Skipped when the ordering failed its checks (perm is then not written).
template <class T>
__global__ void k_gather_leaf(const int32_t *idx_m, const double *vals, const int32_t *perm, int64_t n, int32_t *lidx,
                              T *lval, const int32_t *flags) {
    if (*flags & kFlagOrderCheck) return;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = perm[q];
        lidx[q] = idx_m[p];
        lval[q] = (T)vals[p];
    }
}
template <class T>
hipError_t gather_leaf(const int32_t *idx_m, const double *vals, const int32_t *perm, int64_t n, int32_t *lidx,
                       T *lval, const int32_t *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_gather_leaf<T><<<grid_for(n), 256, 0, s>>>(idx_m, vals, perm, n, lidx, lval, flags);
    TK_LAUNCHED();
    return hipSuccess;
}
template hipError_t gather_leaf<double>(const int32_t *, const double *, const int32_t *, int64_t, int32_t *,
                                        double *, const int32_t *, hipStream_t);
template hipError_t gather_leaf<float>(const int32_t *, const double *, const int32_t *, int64_t, int32_t *, float *,
                                       const int32_t *, hipStream_t);

// ------------------------------------------------------------------ sum of squares
__device__ inline double block_sum_f64(double x) {
    __shared__ double ws[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if (lane == 0) ws[w] = x;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) t += ws[i];
    __syncthreads();
    return t;  // valid in thread 0
}

__global__ void k_sumsq_partial(const double *v, int64_t n, double *partials) {
    double acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += v[i] * v[i];
    double t = block_sum_f64(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}
__global__ void k_sum_final(const double *partials, int np, double *out) {
    double acc = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
    double t = block_sum_f64(acc);
    if (threadIdx.x == 0) *out = t;
}
hipError_t sumsq(const double *v, int64_t n, double *partials, double *out, hipStream_t s) {
    k_sumsq_partial<<<kReduceBlocks, 256, 0, s>>>(v, n, partials);
    TK_LAUNCHED();
    k_sum_final<<<1, 256, 0, s>>>(partials, kReduceBlocks, out);
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ HO-SVD Gram
// A workgroup of W waves owns row i of H = X_(n) X_(n)^T. The mode-n slice i
// (leaf-(n+1) ordering: slots (i, i_{n+2}), leaf index i_{n+1}) is cut into W
// contiguous slot ranges, one per wave, and each wave keeps its own partial
// row in LDS. Each entry x of the slice belongs to the mode-n fibre
// (i_{n+1}, i_{n+2}), whose entries (i', x') in the leaf-n ordering add
// x * x' to H[i][i']. Lanes take 64 slots at a time and make one product per
// round; the lane that made a product adds it to the partial row itself.
// Lanes whose columns share a key (column mod kHosvdTag) within a round add
// in lane order, one pass per depth of collision: the pending lanes post
// their lane id to the key's tag with an LDS atomic minimum, the lane whose
// id stands there adds and resets the tag. The partial rows are summed in
// wave order at the end, so every H[i][i'] is summed in an order fixed by
// the data and W.
constexpr int kHosvdTag = 512;
constexpr int kHosvdMaxWaves = 16;

__global__ void __launch_bounds__(64 * kHosvdMaxWaves)
    k_hosvd_gram(int32_t In, int32_t In1, int32_t In2, const int32_t *ptr_n, const int32_t *lidx_n,
                 const double *lval_n, const int32_t *ptr_s, const int32_t *lidx_s, const double *lval_s, double *H) {
    extern __shared__ double part[];
    const int W = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x;
    double *hrow = part + (int64_t)w * In;
    int32_t *tag = reinterpret_cast<int32_t *>(part + (int64_t)W * In) + w * kHosvdTag;
    for (int c = threadIdx.x; c < W * In; c += blockDim.x) part[c] = 0.0;
    for (int c = lane; c < kHosvdTag; c += 64) tag[c] = 64;
    __syncthreads();
    const int64_t slot0 = (int64_t)i * In2;
    const int64_t lo = (int64_t)In2 * w / W, hi = (int64_t)In2 * (w + 1) / W;
    for (int64_t base = lo; base < hi; base += 64) {
        const int64_t i2 = base + lane;
        int32_t e = 0, e_end = 0;
        if (i2 < hi) {
            e = ptr_s[slot0 + i2];
            e_end = ptr_s[slot0 + i2 + 1];
        }
        int32_t q = 0, q_end = 0;
        double x = 0.0;
        // advance to the first entry with a non-empty fibre
        while (q == q_end && e < e_end) {
            int32_t i1 = lidx_s[e];
            x = lval_s[e];
            int64_t f = i2 * (int64_t)In1 + i1;
            q = ptr_n[f];
            q_end = ptr_n[f + 1];
            ++e;
        }
        while (__ballot(q < q_end)) {
            bool pend = q < q_end;
            int32_t ci = 0;
            double cv = 0.0;
            if (pend) {
                ci = lidx_n[q];
                cv = x * lval_n[q];
                ++q;
                while (q == q_end && e < e_end) {
                    int32_t i1 = lidx_s[e];
                    x = lval_s[e];
                    int64_t f = i2 * (int64_t)In1 + i1;
                    q = ptr_n[f];
                    q_end = ptr_n[f + 1];
                    ++e;
                }
            }
            const int key = ci & (kHosvdTag - 1);
            while (__ballot(pend)) {
                if (pend) atomicMin(&tag[key], lane);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (pend && __hip_atomic_load(&tag[key], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) == lane) {
                    double h = __hip_atomic_load(&hrow[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    __hip_atomic_store(&hrow[ci], h + cv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    __hip_atomic_store(&tag[key], 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    pend = false;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
    }
    __syncthreads();
    double *row = H + (int64_t)i * In;
    for (int c = threadIdx.x; c < In; c += blockDim.x) {
        double s = part[c];
        for (int v = 1; v < W; ++v) s += part[(int64_t)v * In + c];
        row[c] = s;
    }
}

// H <- (H + H^T) / 2, elementwise symmetric result.
__global__ void k_symmetrize(double *H, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * n; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / n, j = t - i * n;
        if (i > j) {
            double a = H[i * n + j], b = H[j * n + i];
            double m = 0.5 * (a + b);
            H[i * n + j] = m;
            H[j * n + i] = m;
        }
    }
}

hipError_t hosvd_gram(int n, const int64_t dims[3], const int32_t *ptr_n, const int32_t *lidx_n,
                      const double *lval_n, const int32_t *ptr_s, const int32_t *lidx_s, const double *lval_s,
                      double *H, hipStream_t s) {
    return hosvd_gram_sized((int32_t)dims[n], (int32_t)dims[(n + 1) % 3], (int32_t)dims[(n + 2) % 3], ptr_n, lidx_n,
                            lval_n, ptr_s, lidx_s, lval_s, H, s);
}

hipError_t hosvd_gram_sized(int32_t In, int32_t In1, int32_t In2, const int32_t *ptr_n, const int32_t *lidx_n,
                            const double *lval_n, const int32_t *ptr_s, const int32_t *lidx_s, const double *lval_s,
                            double *H, hipStream_t s) {
    // About four waves per SIMD over the rows; no more waves than 64-slot
    // batches in a row; the partial rows and tags within the LDS budget.
    const size_t per_wave = sizeof(double) * (size_t)In + sizeof(int32_t) * kHosvdTag;
    int64_t W = std::min<int64_t>({kHosvdMaxWaves, std::max<int64_t>(1, ceil_div(4096, In)),
                                   std::max<int64_t>(1, ceil_div(In2, 64))});
    while (W > 1 && (size_t)W * per_wave > 65536) --W;
    const size_t lds = (size_t)W * per_wave;
    if (lds > 65536) lds_limit((const void *)k_hosvd_gram, lds);
    k_hosvd_gram<<<In, (unsigned)(64 * W), lds, s>>>(In, In1, In2, ptr_n, lidx_n, lval_n, ptr_s, lidx_s, lval_s, H);
    TK_LAUNCHED();
    k_symmetrize<<<grid_for((int64_t)In * In), 256, 0, s>>>(H, In);
    TK_LAUNCHED();
    return hipSuccess;
}

}  // namespace tk
