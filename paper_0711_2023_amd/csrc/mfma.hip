// Dense contractions after the projection, on the matrix cores of gfx950:
//
// * gram(): M_n = sum_t T_t,(n) T_t,(n)^T, the projected-slice Grams of
//   Multislice Projection (Figure 7: each M is a sum over two slice families
//   of (X_s F)(X_s F)^T, i.e. the Gram of the mode-n unfolding of a single-
//   mode projection of X) and the Z_(n) Z_(n)^T of HOOI (Figure 3). Lower-
//   triangular output tiles, split over K; the FP32 (or FP64) partial tiles
//   are summed in FP64 in a fixed order and mirrored into a full symmetric M.
// * gemm(): batched C[b] = sum_k A(i,k) B[b](k,j) for the second stage of
//   HOOI's tensor-times-matrix chain, the core contractions, and the dense
//   products of the eigensolver, with an optional split over K and an FP64
//   epilogue C = alpha*acc + beta*E1 + gamma*E2.
//
// MFMA lane layouts (one wave, lane l):
//   v_mfma_f32_32x32x2f32 : A[i=l%32][k=l/32], B[k=l/32][j=l%32],
//                           D[v] -> row 8*(v/4) + 4*(l/32) + v%4, col l%32
//   v_mfma_f32_32x32x16_bf16: A[i=l%32][k=8*(l/32)+t], B[k=8*(l/32)+t][j=l%32]
//                           (t = 0..7), D as above
//   v_mfma_f64_16x16x4f64 : A[i=l%16][k=l/16], B[k=l/16][j=l%16],
//                           D[v] -> row 4*v + l/16, col l%16
#include "common.h"

#include <algorithm>
#include <cmath>

namespace tk {

// ------------------------------------------------------------------ policies
template <int WT>
struct PolF32 {
    typedef float E;
    typedef float Acc;
    typedef floatx16 Frag;
    static constexpr int BT = 32, NB = WT / BT, KS = 16, KI = 2, LDK = KS + 1, NV = 16;
    __device__ static void mma(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        mma_ld<LDK>(As, Bs, arow, brow, kk, c);
    }
    template <int L>
    __device__ static void mma_ld(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        const int l = threadIdx.x & 63;
        float a = As[(arow + (l & 31)) * L + kk + (l >> 5)];
        float b = Bs[(brow + (l & 31)) * L + kk + (l >> 5)];
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static int orow(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
    __device__ static int ocol(int, int l) { return l & 31; }
};

template <int WT>
struct PolBF16 {
    typedef bf16 E;
    typedef float Acc;
    typedef floatx16 Frag;
    static constexpr int BT = 32, NB = WT / BT, KS = 32, KI = 16, LDK = KS + 8, NV = 16;
    __device__ static void mma(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        mma_ld<LDK>(As, Bs, arow, brow, kk, c);
    }
    template <int L>
    __device__ static void mma_ld(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        const int l = threadIdx.x & 63;
        bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[(arow + (l & 31)) * L + kk + 8 * (l >> 5)]);
        bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[(brow + (l & 31)) * L + kk + 8 * (l >> 5)]);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static int orow(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
    __device__ static int ocol(int, int l) { return l & 31; }
};

template <int WT>
struct PolF64 {
    typedef double E;
    typedef double Acc;
    typedef doublex4 Frag;
    static constexpr int BT = 16, NB = WT / BT, KS = 16, KI = 4, LDK = KS + 1, NV = 4;
    __device__ static void mma(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        mma_ld<LDK>(As, Bs, arow, brow, kk, c);
    }
    template <int L>
    __device__ static void mma_ld(const E *As, const E *Bs, int arow, int brow, int kk, Frag &c) {
        const int l = threadIdx.x & 63;
        double a = As[(arow + (l & 15)) * L + kk + (l >> 4)];
        double b = Bs[(brow + (l & 15)) * L + kk + (l >> 4)];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int orow(int v, int l) { return 4 * v + (l >> 4); }
    __device__ static int ocol(int, int l) { return l & 15; }
};

template <class Frag, int NV>
__device__ inline void frag_zero(Frag &f) {
#pragma unroll
    for (int v = 0; v < NV; ++v) f[v] = 0;
}

template <class E, class S>
__device__ inline E cvt(S x) { return (E)x; }
template <>
__device__ inline bf16 cvt<bf16, double>(double x) { return (bf16)(float)x; }

// ------------------------------------------------------------------ Gram
struct GramTermK {
    const void *base, *base_b;
    int64_t s_row, s_chunk, chunk_len, nchunks;
    int64_t kper;         // K elements per split (multiple of the stage depth)
    int32_t split_begin;  // first split index of this term
};
struct GramKArgs {
    GramTermK t[kGramMaxTerms];
    int32_t nterms;
    int32_t splits_total;
    int32_t npairs;
    int32_t n;
};

__device__ inline void pair_decode(int pair, int &ti, int &tj) {
    int t = (int)((sqrt(8.0 * pair + 1.0) - 1.0) * 0.5);
    while ((t + 1) * (t + 2) / 2 <= pair) ++t;
    while (t * (t + 1) / 2 > pair) --t;
    ti = t;
    tj = pair - t * (t + 1) / 2;
}

// Stage depth per element type: 64 BF16, 32 FP32, 16 FP64 (128 bytes per row).
template <class E> struct GramKS { static constexpr int v = 128 / sizeof(E); };
template <> struct GramKS<bf16> { static constexpr int v = 64; };

template <class P, int WT> struct GramCfg {
    typedef typename P::E E;
    static constexpr int TBK = 2 * WT;            // output tile
    static constexpr int KS = GramKS<E>::v;       // stage depth
    static constexpr int VW = 16 / sizeof(E);     // elements per 16-byte vector
    static constexpr int TPR = KS / VW;           // threads per row per stage (8)
    static constexpr int RPP = 256 / TPR;         // rows per load pass (32)
    static constexpr int PASSES = TBK / RPP;      // load passes per operand
    static constexpr int LDK = sizeof(E) == 2 ? KS + 8 : KS + 1;
};

// One operand row-block of one stage: TBK rows x KS columns, loaded as
// 16-byte vectors (VEC: chunk length, strides and base are multiples of the
// vector) or element by element.
template <class Cfg, bool VEC>
struct StageRegs {
    typename Cfg::E v[Cfg::PASSES][Cfg::VW];
};

template <class Cfg, bool VEC>
__device__ inline void load_stage(StageRegs<Cfg, VEC> &R, const typename Cfg::E *base, const GramTermK &t,
                                  int64_t row0, int n, int64_t k, int64_t kend, int64_t kc, int64_t kr, int rr) {
    typedef typename Cfg::E E;
#pragma unroll
    for (int ps = 0; ps < Cfg::PASSES; ++ps) {
        const int64_t row = row0 + ps * Cfg::RPP + rr;
        if (VEC) {
            if (row < n && k < kend) {
                typedef E __attribute__((ext_vector_type(Cfg::VW))) V;
                V x = *reinterpret_cast<const V *>(base + row * t.s_row + kc * t.s_chunk + kr);
#pragma unroll
                for (int e = 0; e < Cfg::VW; ++e) R.v[ps][e] = x[e];
            } else {
#pragma unroll
                for (int e = 0; e < Cfg::VW; ++e) R.v[ps][e] = (E)0;
            }
        } else {
            int64_t c = kc, r = kr;
#pragma unroll
            for (int e = 0; e < Cfg::VW; ++e) {
                const bool ok = row < n && k + e < kend;
                R.v[ps][e] = ok ? base[row * t.s_row + c * t.s_chunk + r] : (E)0;
                if (++r == t.chunk_len) {
                    r = 0;
                    ++c;
                }
            }
        }
    }
}

template <class Cfg, bool VEC>
__device__ inline void store_stage(const StageRegs<Cfg, VEC> &R, typename Cfg::E *S, int rr, int kv) {
#pragma unroll
    for (int ps = 0; ps < Cfg::PASSES; ++ps) {
        const int row = ps * Cfg::RPP + rr;
        if (sizeof(typename Cfg::E) == 2) {
            typedef typename Cfg::E __attribute__((ext_vector_type(Cfg::VW))) V;
            V x;
#pragma unroll
            for (int e = 0; e < Cfg::VW; ++e) x[e] = R.v[ps][e];
            *reinterpret_cast<V *>(&S[row * Cfg::LDK + kv * Cfg::VW]) = x;
        } else {
#pragma unroll
            for (int e = 0; e < Cfg::VW; ++e) S[row * Cfg::LDK + kv * Cfg::VW + e] = R.v[ps][e];
        }
    }
}

template <class P, int WT, bool VEC>
__global__ void __launch_bounds__(256) k_gram(GramKArgs g, typename P::Acc *partials) {
    typedef GramCfg<P, WT> Cfg;
    typedef typename P::E E;
    constexpr int TBK = Cfg::TBK, KS = Cfg::KS, LDK = Cfg::LDK;
    __shared__ __attribute__((aligned(16))) E As[TBK * LDK];
    __shared__ __attribute__((aligned(16))) E Bs[TBK * LDK];
    // XCD-aware item map: consecutive blocks go to different XCDs, so block
    // g runs on XCD g % 8; all tile pairs of one K-split share one XCD (and
    // its L2) by giving split s to XCD s % 8.
    const int gx = blockIdx.x % 8, gq = blockIdx.x / 8;
    const int rnd = gq / g.npairs, pair = gq - rnd * g.npairs;
    const int sidx = rnd * 8 + gx;
    if (sidx >= g.splits_total) return;
    int term = 0;
    for (int q = 1; q < g.nterms; ++q)
        if (sidx >= g.t[q].split_begin) term = q;
    const GramTermK t = g.t[term];
    const int split = sidx - t.split_begin;
    int ti, tj;
    pair_decode(pair, ti, tj);
    const E *base = reinterpret_cast<const E *>(t.base);
    const E *base_b = reinterpret_cast<const E *>(t.base_b);
    // a diagonal tile of a term with one operand reads its rows once
    const bool diag = ti == tj && base_b == base;
    const int64_t K = t.chunk_len * t.nchunks;
    const int64_t kbeg = (int64_t)split * t.kper;
    const int64_t kend = kbeg + t.kper < K ? kbeg + t.kper : K;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
    const int kv = tid % Cfg::TPR, rr = tid / Cfg::TPR;
    int64_t k = kbeg + kv * Cfg::VW;
    int64_t kc = k / t.chunk_len, kr = k - kc * t.chunk_len;
    const int64_t rowA0 = (int64_t)ti * TBK, rowB0 = (int64_t)tj * TBK;

    typename P::Frag acc[P::NB][P::NB];
#pragma unroll
    for (int a = 0; a < P::NB; ++a)
#pragma unroll
        for (int b = 0; b < P::NB; ++b) frag_zero<typename P::Frag, P::NV>(acc[a][b]);

    StageRegs<Cfg, VEC> ra, rb;
    load_stage<Cfg, VEC>(ra, base, t, rowA0, g.n, k, kend, kc, kr, rr);
    if (!diag) load_stage<Cfg, VEC>(rb, base_b, t, rowB0, g.n, k, kend, kc, kr, rr);
    const E *Bsrc = diag ? As : Bs;
    for (int64_t k0 = kbeg; k0 < kend; k0 += KS) {
        store_stage<Cfg, VEC>(ra, As, rr, kv);
        if (!diag) store_stage<Cfg, VEC>(rb, Bs, rr, kv);
        __syncthreads();
        // prefetch the next stage while the matrix cores work on this one
        k += KS;
        kr += KS;
        while (kr >= t.chunk_len) {
            kr -= t.chunk_len;
            ++kc;
        }
        if (k0 + KS < kend) {
            load_stage<Cfg, VEC>(ra, base, t, rowA0, g.n, k, kend, kc, kr, rr);
            if (!diag) load_stage<Cfg, VEC>(rb, base_b, t, rowB0, g.n, k, kend, kc, kr, rr);
        }
#pragma unroll
        for (int q = 0; q < KS; q += P::KI)
#pragma unroll
            for (int a = 0; a < P::NB; ++a)
#pragma unroll
                for (int b = 0; b < P::NB; ++b)
                    P::template mma_ld<LDK>(As, Bsrc, wr * WT + a * P::BT, wc * WT + b * P::BT, q, acc[a][b]);
        __syncthreads();
    }
    typename P::Acc *out = partials + ((int64_t)pair * g.splits_total + sidx) * TBK * TBK;
#pragma unroll
    for (int a = 0; a < P::NB; ++a)
#pragma unroll
        for (int b = 0; b < P::NB; ++b)
#pragma unroll
            for (int v = 0; v < P::NV; ++v) {
                int r = wr * WT + a * P::BT + P::orow(v, lane);
                int c = wc * WT + b * P::BT + P::ocol(v, lane);
                out[r * TBK + c] = acc[a][b][v];
            }
}

template <class Acc>
__global__ void k_gram_reduce(const Acc *partials, int splits_total, int TBK, int n, int64_t total, double *M) {
    const int64_t tile = (int64_t)TBK * TBK;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int pair = (int)(idx / tile);
        int64_t rc = idx - pair * tile;
        int r = (int)(rc / TBK), c = (int)(rc - (int64_t)r * TBK);
        int ti, tj;
        pair_decode(pair, ti, tj);
        int64_t i = (int64_t)ti * TBK + r, j = (int64_t)tj * TBK + c;
        if (i >= n || j >= n) continue;
        if (ti == tj && c > r) continue;
        double sum = 0.0;
        const Acc *p = partials + (int64_t)pair * splits_total * tile + rc;
        for (int s = 0; s < splits_total; ++s) sum += (double)p[s * tile];
        M[i * n + j] = sum;
        M[j * n + i] = sum;
    }
}

struct GramPlan {
    int TBK, KS, npairs, splits_total;
    int64_t kper[kGramMaxTerms];
    int32_t split_begin[kGramMaxTerms];
    size_t acc_size;
};

static GramPlan gram_plan(int n, int prec, int nterms, const int64_t *K, const Tune &tn) {
    GramPlan p;
    p.TBK = prec == P64 ? 64 : 128;
    p.KS = prec == P64 ? 16 : (prec == P32 ? 32 : 64);
    p.acc_size = prec == P64 ? 8 : 4;
    int nt = (int)ceil_div(n, p.TBK);
    p.npairs = nt * (nt + 1) / 2;
    // about tn.gram_items blocks in flight, at least tn.gram_min_stages stages per block
    int want = (int)std::max<int64_t>(1, ceil_div(tn.gram_items, (int64_t)p.npairs * nterms));
    p.splits_total = 0;
    for (int t = 0; t < nterms; ++t) {
        int64_t Kt = K[t] > 0 ? K[t] : 1;
        int64_t maxs = std::max<int64_t>(1, ceil_div(Kt, (int64_t)p.KS * tn.gram_min_stages));
        int64_t s = std::min<int64_t>(want, maxs);
        int64_t kper = ceil_div(ceil_div(Kt, s), p.KS) * p.KS;
        s = ceil_div(Kt, kper);
        p.kper[t] = kper;
        p.split_begin[t] = p.splits_total;
        p.splits_total += (int)s;
    }
    return p;
}

size_t gram_scratch_bytes(int n, int prec, int nterms, const int64_t *K, const Tune &tn) {
    GramPlan p = gram_plan(n, prec, nterms, K, tn);
    return (size_t)p.npairs * p.splits_total * p.TBK * p.TBK * p.acc_size;
}

template <class P, int WT, class Acc>
static hipError_t launch_gram(const GramKArgs &g, bool vec, unsigned blocks, Acc *scratch, hipStream_t s) {
    if (vec)
        k_gram<P, WT, true><<<blocks, 256, 0, s>>>(g, scratch);
    else
        k_gram<P, WT, false><<<blocks, 256, 0, s>>>(g, scratch);
    TK_LAUNCHED();
    return hipSuccess;
}

hipError_t gram(int n, int prec, int nterms, const GramTerm *terms, double *M, void *scratch, hipStream_t s,
                const Tune &tn) {
    if (nterms < 1 || nterms > kGramMaxTerms) return hipErrorInvalidValue;
    int64_t K[kGramMaxTerms] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < nterms; ++t) K[t] = terms[t].chunk_len * terms[t].nchunks;
    GramPlan p = gram_plan(n, prec, nterms, K, tn);
    GramKArgs g{};
    g.nterms = nterms;
    g.splits_total = p.splits_total;
    g.npairs = p.npairs;
    g.n = n;
    const int es = prec == P64 ? 8 : (prec == P32 ? 4 : 2);
    const int vw = 16 / es;
    bool vec = true;
    for (int t = 0; t < nterms; ++t) {
        g.t[t].base = terms[t].base;
        g.t[t].base_b = terms[t].base_b ? terms[t].base_b : terms[t].base;
        g.t[t].s_row = terms[t].s_row;
        g.t[t].s_chunk = terms[t].s_chunk;
        g.t[t].chunk_len = terms[t].chunk_len;
        g.t[t].nchunks = terms[t].nchunks;
        g.t[t].kper = p.kper[t];
        g.t[t].split_begin = p.split_begin[t];
        vec = vec && terms[t].chunk_len % vw == 0 && terms[t].s_row % vw == 0 &&
              (terms[t].nchunks == 1 || terms[t].s_chunk % vw == 0) &&
              reinterpret_cast<uintptr_t>(terms[t].base) % 16 == 0 &&
              reinterpret_cast<uintptr_t>(g.t[t].base_b) % 16 == 0;
    }
    const unsigned blocks = (unsigned)(8 * p.npairs * ceil_div(p.splits_total, 8));
    const int64_t total = (int64_t)p.npairs * p.TBK * p.TBK;
    const int rblocks = (int)std::min<int64_t>(ceil_div(total, 256), 65536);
    if (prec == P64) {
        TK_HIP((launch_gram<PolF64<32>, 32>(g, vec, blocks, (double *)scratch, s)));
        k_gram_reduce<double><<<rblocks, 256, 0, s>>>((const double *)scratch, p.splits_total, p.TBK, n, total, M);
    } else if (prec == P32) {
        TK_HIP((launch_gram<PolF32<64>, 64>(g, vec, blocks, (float *)scratch, s)));
        k_gram_reduce<float><<<rblocks, 256, 0, s>>>((const float *)scratch, p.splits_total, p.TBK, n, total, M);
    } else {
        TK_HIP((launch_gram<PolBF16<64>, 64>(g, vec, blocks, (float *)scratch, s)));
        k_gram_reduce<float><<<rblocks, 256, 0, s>>>((const float *)scratch, p.splits_total, p.TBK, n, total, M);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

// ------------------------------------------------------------------ GEMM
struct GemmKArgs {
    int M, N, K, batch, splitk;
    const void *A;
    int64_t lda;
    int a_trans;
    const void *B;
    int64_t ldb, sB;
    void *C;
    int64_t ldc, sC;
    double alpha, beta, gamma;
    const double *E1, *E2;
    double *split;
    int64_t kper;
};

template <class P, class TA, class TBm, class TO>
__global__ void __launch_bounds__(256) k_gemm(GemmKArgs g) {
    typedef typename P::E E;
    constexpr int WT = 32, BM = 64, BN = 64;
    constexpr int KS = P::KS, LDK = P::LDK;
    __shared__ E As[BM * LDK];
    __shared__ E Bs[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
    const int n0 = blockIdx.x * BN, m0 = blockIdx.y * BM;
    const int zb = blockIdx.z / g.splitk, split = blockIdx.z - zb * g.splitk;
    const int64_t kbeg = (int64_t)split * g.kper;
    const int64_t kend = kbeg + g.kper < g.K ? kbeg + g.kper : g.K;
    const TA *A = reinterpret_cast<const TA *>(g.A);
    const TBm *B = reinterpret_cast<const TBm *>(g.B) + (int64_t)zb * g.sB;

    typename P::Frag acc[P::NB][P::NB];
#pragma unroll
    for (int a = 0; a < P::NB; ++a)
#pragma unroll
        for (int b = 0; b < P::NB; ++b) frag_zero<typename P::Frag, P::NV>(acc[a][b]);

    for (int64_t k0 = kbeg; k0 < kend; k0 += KS) {
        // A tile: BM rows x KS
        if (g.a_trans) {
            // A(i,k) = A[k*lda + i]: i fastest
            for (int e = tid; e < BM * KS; e += 256) {
                int ii = e % BM, kk = e / BM;
                int64_t i = m0 + ii, k = k0 + kk;
                E v = (i < g.M && k < kend) ? cvt<E>(A[k * g.lda + i]) : (E)0;
                As[ii * LDK + kk] = v;
            }
        } else {
            for (int e = tid; e < BM * KS; e += 256) {
                int kk = e % KS, ii = e / KS;
                int64_t i = m0 + ii, k = k0 + kk;
                E v = (i < g.M && k < kend) ? cvt<E>(A[i * g.lda + k]) : (E)0;
                As[ii * LDK + kk] = v;
            }
        }
        // B tile: BN cols x KS, B(k,j) = B[k*ldb + j]: j fastest
        for (int e = tid; e < BN * KS; e += 256) {
            int jj = e % BN, kk = e / BN;
            int64_t j = n0 + jj, k = k0 + kk;
            E v = (j < g.N && k < kend) ? cvt<E>(B[k * g.ldb + j]) : (E)0;
            Bs[jj * LDK + kk] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KS; q += P::KI)
#pragma unroll
            for (int a = 0; a < P::NB; ++a)
#pragma unroll
                for (int b = 0; b < P::NB; ++b)
                    P::mma(As, Bs, wr * WT + a * P::BT, wc * WT + b * P::BT, q, acc[a][b]);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < P::NB; ++a)
#pragma unroll
        for (int b = 0; b < P::NB; ++b)
#pragma unroll
            for (int v = 0; v < P::NV; ++v) {
                int64_t i = m0 + wr * WT + a * P::BT + P::orow(v, lane);
                int64_t j = n0 + wc * WT + b * P::BT + P::ocol(v, lane);
                if (i >= g.M || j >= g.N) continue;
                double x = (double)acc[a][b][v];
                if (g.splitk > 1) {
                    g.split[(((int64_t)split * g.batch + zb) * g.M + i) * g.N + j] = x;
                } else {
                    int64_t o = (int64_t)zb * g.sC + i * g.ldc + j;
                    double y = g.alpha * x;
                    if (g.E1) y += g.beta * g.E1[o];
                    if (g.E2) y += g.gamma * g.E2[o];
                    reinterpret_cast<TO *>(g.C)[o] = cvt<TO>(y);
                }
            }
}

template <class TO>
__global__ void k_gemm_split_reduce(GemmKArgs g) {
    const int64_t per = (int64_t)g.M * g.N, total = per * g.batch;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t zb = t / per, r = t - zb * per, i = r / g.N, j = r - i * g.N;
        double x = 0.0;
        for (int s = 0; s < g.splitk; ++s) x += g.split[((int64_t)s * g.batch + zb) * per + r];
        int64_t o = zb * g.sC + i * g.ldc + j;
        double y = g.alpha * x;
        if (g.E1) y += g.beta * g.E1[o];
        if (g.E2) y += g.gamma * g.E2[o];
        reinterpret_cast<TO *>(g.C)[o] = cvt<TO>(y);
    }
}

template <class P, class TA, class TBm, class TO>
static hipError_t launch_gemm(const GemmArgs &a, hipStream_t s) {
    GemmKArgs g;
    g.M = a.M;
    g.N = a.N;
    g.K = a.K;
    g.batch = a.batch;
    g.splitk = a.splitk < 1 ? 1 : a.splitk;
    g.A = a.A;
    g.lda = a.lda;
    g.a_trans = a.a_trans ? 1 : 0;
    g.B = a.B;
    g.ldb = a.ldb;
    g.sB = a.sB;
    g.C = a.C;
    g.ldc = a.ldc;
    g.sC = a.sC;
    g.alpha = a.alpha;
    g.beta = a.beta;
    g.gamma = a.gamma;
    g.E1 = a.E1;
    g.E2 = a.E2;
    g.split = a.split_scratch;
    g.kper = ceil_div(ceil_div(a.K, g.splitk), P::KS) * P::KS;
    if (g.splitk > 1) g.splitk = (int)ceil_div(a.K, g.kper);
    dim3 grid((unsigned)ceil_div(a.N, 64), (unsigned)ceil_div(a.M, 64), (unsigned)(a.batch * g.splitk));
    k_gemm<P, TA, TBm, TO><<<grid, 256, 0, s>>>(g);
    TK_LAUNCHED();
    if (g.splitk > 1) {
        int64_t total = (int64_t)a.M * a.N * a.batch;
        int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 65536);
        k_gemm_split_reduce<TO><<<blocks, 256, 0, s>>>(g);
        TK_LAUNCHED();
    }
    return hipSuccess;
}

// prec selects the MFMA kind; A/B element types follow it except for the
// FP64 kind, whose B operand may be FP32 (projections feeding the core).
hipError_t gemm(const GemmArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
    switch (a.prec) {
        case P64:
            if (a.out_type == P64) return launch_gemm<PolF64<32>, double, double, double>(a, s);
            return hipErrorInvalidValue;
        case 3:  // FP64 MFMA, A double, B float, out double
            return launch_gemm<PolF64<32>, double, float, double>(a, s);
        case P32:
            if (a.out_type == P32) return launch_gemm<PolF32<32>, float, float, float>(a, s);
            if (a.out_type == P64) return launch_gemm<PolF32<32>, float, float, double>(a, s);
            return hipErrorInvalidValue;
        case PBF16:
            if (a.out_type == P32) return launch_gemm<PolBF16<32>, bf16, bf16, float>(a, s);
            if (a.out_type == PBF16) return launch_gemm<PolBF16<32>, bf16, bf16, bf16>(a, s);
            return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace tk
