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
constexpr int kGramWideMin = 768;  // BF16 Grams of at least this order use 256-row tiles
constexpr int kGramRing = 4;       // stages in flight in k_gram_dl
constexpr int kGramDlWaves = 8;    // waves of a k_gram_dl workgroup (8: 64 x 128 each; 4: 128 x 128)

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

template <class P, int TBK_, int NT> struct GramCfg {
    typedef typename P::E E;
    static constexpr int TBK = TBK_;              // output tile
    static constexpr int KS = GramKS<E>::v;       // stage depth
    static constexpr int VW = 16 / sizeof(E);     // elements per 16-byte vector
    static constexpr int TPR = KS / VW;           // threads per row per stage (8)
    static constexpr int RPP = NT / TPR;          // rows per load pass (32 for 256 threads)
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

// WR x WC waves, each computing a WTR x WTC part of the TBK x TBK output
// tile (TBK = WR WTR = WC WTC); both operand row blocks of a stage in LDS
// (gram_lds_bytes).
template <class P, int WTR, int WTC, int WR, int WC, bool VEC>
__global__ void __launch_bounds__(64 * WR * WC) k_gram(GramKArgs g, typename P::Acc *partials) {
    constexpr int NT = 64 * WR * WC, TBK0 = WR * WTR;
    static_assert(WC * WTC == TBK0, "square output tiles");
    typedef GramCfg<P, TBK0, NT> Cfg;
    typedef typename P::E E;
    constexpr int TBK = Cfg::TBK, KS = Cfg::KS, LDK = Cfg::LDK;
    constexpr int NBR = WTR / P::BT, NBC = WTC / P::BT;
    extern __shared__ __attribute__((aligned(16))) char gram_smem[];
    E *As = reinterpret_cast<E *>(gram_smem), *Bs = As + TBK * LDK;
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

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w / WC, wc = w % WC;
    const int kv = tid % Cfg::TPR, rr = tid / Cfg::TPR;
    int64_t k = kbeg + kv * Cfg::VW;
    int64_t kc = k / t.chunk_len, kr = k - kc * t.chunk_len;
    const int64_t rowA0 = (int64_t)ti * TBK, rowB0 = (int64_t)tj * TBK;

    typename P::Frag acc[NBR][NBC];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) frag_zero<typename P::Frag, P::NV>(acc[a][b]);

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
            for (int a = 0; a < NBR; ++a)
#pragma unroll
                for (int b = 0; b < NBC; ++b)
                    P::template mma_ld<LDK>(As, Bsrc, wr * WTR + a * P::BT, wc * WTC + b * P::BT, q, acc[a][b]);
        __syncthreads();
    }
    typename P::Acc *out = partials + ((int64_t)pair * g.splits_total + sidx) * TBK * TBK;
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b)
#pragma unroll
            for (int v = 0; v < P::NV; ++v) {
                int r = wr * WTR + a * P::BT + P::orow(v, lane);
                int c = wc * WTC + b * P::BT + P::ocol(v, lane);
                out[r * TBK + c] = acc[a][b][v];
            }
}

// LDS of a k_gram launch: both operand row blocks of one stage.
template <class P, int TBK>
constexpr size_t gram_lds_bytes() {
    return 2 * (size_t)TBK * GramCfg<P, TBK, 256>::LDK * sizeof(typename P::E);
}

// BF16 Gram with 256-row output tiles whose operand stages go from memory
// straight into LDS (buffer loads with the LDS destination: no staging
// registers), in a ring of four stages, so that the loads of a stage are
// issued three stages ahead of the matrix-core work on it and a stage costs
// one workgroup barrier. Stages are 32 K columns deep; an operand stage is
// 256 LDS rows of 64 bytes, each filled by one 16-row wave load, the four
// 16-byte chunks of row r at slots c ^ gram_dl_swz(r), so that fragment
// reads of consecutive rows fall on distinct banks. Elements past the
// split, the term or the order read as zeros (the load's offset is made out
// of range). kGramDlWaves waves (eight, each 64 x 128 as in
// k_gram<PolBF16, 64, 128, 4, 2>; four of 128 x 128 read half the fragment
// bytes per matrix-core step but ran 4 % slower); the same items, partial
// tiles and reduction as k_gram.
constexpr int kGramDlKS = 32, kGramDlRowB = 64, kGramDlStage = 256 * kGramDlRowB;
constexpr uint32_t kGramDlOob = 0x80000000u;

// Slot permutation of the chunks of LDS row r: chunk c sits at slot
// c ^ gram_dl_swz(r). Any 8 aligned consecutive rows (two 16-byte units per
// row in 128 bytes) and any 16 aligned consecutive rows (four per row in
// 256 bytes) then read one chunk index from distinct units.
__device__ inline int gram_dl_swz(int r) { return ((r >> 2) & 1) | ((((r >> 1) ^ (r >> 3)) & 1) << 1); }

struct GramDlLane {
    __amdgpu_buffer_rsrc_t ra, rb;
    uint32_t rowA[4], rowB[4];  // element offsets of the lane's rows (one per wave load of an operand)
    bool okA[4], okB[4];
    int64_t k, kc, kr, kend, chunk_len, s_chunk;
};

template <int SLOT>
__device__ inline char *gram_dl_slot(bool b);

__shared__ __attribute__((aligned(16))) char gram_dl_a0[kGramDlStage], gram_dl_b0[kGramDlStage];
__shared__ __attribute__((aligned(16))) char gram_dl_a1[kGramDlStage], gram_dl_b1[kGramDlStage];
__shared__ __attribute__((aligned(16))) char gram_dl_a2[kGramDlStage], gram_dl_b2[kGramDlStage];
__shared__ __attribute__((aligned(16))) char gram_dl_a3[kGramDlStage], gram_dl_b3[kGramDlStage];
template <> __device__ inline char *gram_dl_slot<0>(bool b) { return b ? gram_dl_b0 : gram_dl_a0; }
template <> __device__ inline char *gram_dl_slot<1>(bool b) { return b ? gram_dl_b1 : gram_dl_a1; }
template <> __device__ inline char *gram_dl_slot<2>(bool b) { return b ? gram_dl_b2 : gram_dl_a2; }
template <> __device__ inline char *gram_dl_slot<3>(bool b) { return b ? gram_dl_b3 : gram_dl_a3; }

// The lane's loads of the next stage into ring slot SLOT: 16 / NW wave loads
// of 16 rows per operand (rows 16 (w + NW h) of the tile), then the K
// position moves on by one stage.
template <int SLOT, int NW>
__device__ inline void gram_dl_issue(GramDlLane &L, bool diag, int w) {
    typedef __attribute__((address_space(3))) void lds_void;
    constexpr int H = 16 / NW;
    const bool kin = L.k < L.kend;
    const uint32_t koff = (uint32_t)(L.kc * L.s_chunk + L.kr);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        char *dst = gram_dl_slot<SLOT>(false) + (16 * (w + NW * h)) * kGramDlRowB;
        const uint32_t off = kin && L.okA[h] ? (L.rowA[h] + koff) * 2u : kGramDlOob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(L.ra, (lds_void *)dst, 16, off, 0, 0, 0);
    }
    if (!diag) {
#pragma unroll
        for (int h = 0; h < H; ++h) {
            char *dst = gram_dl_slot<SLOT>(true) + (16 * (w + NW * h)) * kGramDlRowB;
            const uint32_t off = kin && L.okB[h] ? (L.rowB[h] + koff) * 2u : kGramDlOob;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(L.rb, (lds_void *)dst, 16, off, 0, 0, 0);
        }
    }
    L.k += kGramDlKS;
    L.kr += kGramDlKS;
    while (L.kr >= L.chunk_len) {
        L.kr -= L.chunk_len;
        ++L.kc;
    }
}

// The fragments of one 16-deep step, read in one asm block that waits for
// them itself (the compiler would otherwise make every LDS read wait for all
// buffer loads in flight, as it cannot tell the ring slots apart).
__device__ inline void gram_dl_frags(const uint32_t (&ad)[6], bf16x8 (&f)[6]) {
    asm volatile(
        "ds_read_b128 %0, %6\n\t"
        "ds_read_b128 %1, %7\n\t"
        "ds_read_b128 %2, %8\n\t"
        "ds_read_b128 %3, %9\n\t"
        "ds_read_b128 %4, %10\n\t"
        "ds_read_b128 %5, %11\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(f[0]), "=&v"(f[1]), "=&v"(f[2]), "=&v"(f[3]), "=&v"(f[4]), "=&v"(f[5])
        : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5])
        : "memory");
}
__device__ inline void gram_dl_frags(const uint32_t (&ad)[8], bf16x8 (&f)[8]) {
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %9\n\t"
        "ds_read_b128 %2, %10\n\t"
        "ds_read_b128 %3, %11\n\t"
        "ds_read_b128 %4, %12\n\t"
        "ds_read_b128 %5, %13\n\t"
        "ds_read_b128 %6, %14\n\t"
        "ds_read_b128 %7, %15\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(f[0]), "=&v"(f[1]), "=&v"(f[2]), "=&v"(f[3]), "=&v"(f[4]), "=&v"(f[5]), "=&v"(f[6]), "=&v"(f[7])
        : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]), "v"(ad[6]), "v"(ad[7])
        : "memory");
}

__device__ inline uint32_t lds_addr(const char *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)p;
}

// One stage of matrix-core work on ring slot SLOT: the wave's WTR x 128
// part of the tile (NBR x 4 fragments of 32 x 32), rows from wr WTR,
// columns from wc 128.
template <int SLOT, int NBR>
__device__ inline void gram_dl_mma(floatx16 (&acc)[NBR][4], bool diag, int wr, int wc, int lane) {
    const uint32_t A = lds_addr(gram_dl_slot<SLOT>(false));
    const uint32_t B = diag ? A : lds_addr(gram_dl_slot<SLOT>(true));
#pragma unroll
    for (int q = 0; q < kGramDlKS / 16; ++q) {
        const int ch = 2 * q + (lane >> 5);
        uint32_t ad[NBR + 4];
#pragma unroll
        for (int a = 0; a < NBR; ++a) {
            const int r = wr * 32 * NBR + a * 32 + (lane & 31);
            ad[a] = A + r * kGramDlRowB + ((ch ^ gram_dl_swz(r)) << 4);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = wc * 128 + b * 32 + (lane & 31);
            ad[NBR + b] = B + r * kGramDlRowB + ((ch ^ gram_dl_swz(r)) << 4);
        }
        bf16x8 f[NBR + 4];
        gram_dl_frags(ad, f);
#pragma unroll
        for (int a = 0; a < NBR; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f[a], f[NBR + b], acc[a][b], 0, 0, 0);
    }
}

// Wait until at most n (0, 2, 4, 6, 8, 12 or 16) of the wave's buffer loads
// are in flight.
__device__ inline void gram_dl_wait(int n) {
    // s_waitcnt immediates: vmcnt n (bits 3:0 and 15:14), expcnt and lgkmcnt
    // not waited on
    switch (n) {
        case 0: __builtin_amdgcn_s_waitcnt(0x0f70); break;
        case 2: __builtin_amdgcn_s_waitcnt(0x0f72); break;
        case 4: __builtin_amdgcn_s_waitcnt(0x0f74); break;
        case 6: __builtin_amdgcn_s_waitcnt(0x0f76); break;
        case 8: __builtin_amdgcn_s_waitcnt(0x0f78); break;
        case 12: __builtin_amdgcn_s_waitcnt(0x0f7c); break;
        default: __builtin_amdgcn_s_waitcnt(0x4f70); break;
    }
}

template <int SLOT, int NW, int NBR>
__device__ inline void gram_dl_step(GramDlLane &L, floatx16 (&acc)[NBR][4], int s, int nst, int lps, bool diag,
                                    int w, int wr, int wc, int lane) {
    // this wave's loads of stage s have landed once only the later issued
    // stages (at most two) are in flight
    const int issued = s + kGramRing - 1 < nst ? s + kGramRing - 1 : nst;
    gram_dl_wait((issued - s - 1) * lps);
    // a bare barrier: every LDS read of the wave has completed (the reads
    // wait for themselves) and its loads of stage s have landed; after it no
    // wave reads the slot of stage s - 1, which the next loads refill
    asm volatile("s_barrier" ::: "memory");
    if (s + kGramRing - 1 < nst) gram_dl_issue<(SLOT + kGramRing - 1) % kGramRing, NW>(L, diag, w);
    gram_dl_mma<SLOT, NBR>(acc, diag, wr, wc, lane);
}

// NW waves as NW / 2 x 2, each computing a (512 / NW) x 128 part of the tile.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_gram_dl(GramKArgs g, float *partials) {
    constexpr int NBR = 16 / NW, H = 16 / NW;
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
    const bool diag = ti == tj && t.base_b == t.base;
    const int64_t K = t.chunk_len * t.nchunks;
    const int64_t kbeg = (int64_t)split * t.kper;
    const int64_t kend = kbeg + t.kper < K ? kbeg + t.kper : K;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
    // the operand's extent in bytes (the host has checked it is below 2^31)
    const uint32_t nbytes =
        (uint32_t)((((int64_t)g.n - 1) * t.s_row + (t.nchunks - 1) * t.s_chunk + t.chunk_len) * 2);
    GramDlLane L;
    L.ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(t.base), (short)0, (int)nbytes, 0x00020000);
    L.rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(t.base_b), (short)0, (int)nbytes, 0x00020000);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int64_t ra = (int64_t)ti * 256 + 16 * (w + NW * h) + (lane >> 2);
        const int64_t rb = (int64_t)tj * 256 + 16 * (w + NW * h) + (lane >> 2);
        L.okA[h] = ra < g.n;
        L.okB[h] = rb < g.n;
        L.rowA[h] = (uint32_t)((L.okA[h] ? ra : 0) * t.s_row);
        L.rowB[h] = (uint32_t)((L.okB[h] ? rb : 0) * t.s_row);
    }
    // the lane's chunk of each row: its slot lane % 4 of row lane / 4 (mod
    // 16) holds chunk c
    const int c = (lane & 3) ^ gram_dl_swz(lane >> 2);
    L.k = kbeg + 8 * c;
    L.kend = kend;
    L.chunk_len = t.chunk_len;
    L.s_chunk = t.s_chunk;
    L.kc = L.k / t.chunk_len;
    L.kr = L.k - L.kc * t.chunk_len;
    const int nst = (int)((kend - kbeg + kGramDlKS - 1) / kGramDlKS);
    const int lps = diag ? H : 2 * H;

    floatx16 acc[NBR][4];
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) frag_zero<floatx16, 16>(acc[a][b]);
    if (nst > 0) gram_dl_issue<0, NW>(L, diag, w);
    if (nst > 1) gram_dl_issue<1, NW>(L, diag, w);
    if (nst > 2) gram_dl_issue<2, NW>(L, diag, w);
    for (int s = 0; s < nst; s += kGramRing) {
        gram_dl_step<0, NW, NBR>(L, acc, s, nst, lps, diag, w, wr, wc, lane);
        if (s + 1 < nst) gram_dl_step<1, NW, NBR>(L, acc, s + 1, nst, lps, diag, w, wr, wc, lane);
        if (s + 2 < nst) gram_dl_step<2, NW, NBR>(L, acc, s + 2, nst, lps, diag, w, wr, wc, lane);
        if (s + 3 < nst) gram_dl_step<3, NW, NBR>(L, acc, s + 3, nst, lps, diag, w, wr, wc, lane);
    }
    float *out = partials + ((int64_t)pair * g.splits_total + sidx) * 256 * 256;
#pragma unroll
    for (int a = 0; a < NBR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = wr * 32 * NBR + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int cc = wc * 128 + b * 32 + (lane & 31);
                out[r * 256 + cc] = acc[a][b][v];
            }
}

// The split partials of every tile pair summed into M, both triangles. A
// workgroup takes one 32 x 32 block of a tile: each thread sums four of its
// elements over the splits in split order (FP64, from zero), writes them to
// the block's own place in rows of 32, and the block goes through LDS to be
// written to its mirror in rows of 32 as well. Of a diagonal tile only the
// blocks on and below the diagonal are read, and each element above the
// diagonal takes its mirror's sum, so M is symmetric bit for bit.
constexpr int kGramRedB = 32;
template <class Acc>
__global__ void __launch_bounds__(256) k_gram_reduce(const Acc *partials, int splits_total, int TBK, int n,
                                                     double *M) {
    __shared__ double blk[kGramRedB][kGramRedB + 1];
    const int nb = TBK / kGramRedB;
    const int pair = blockIdx.x / (nb * nb), q = blockIdx.x - pair * nb * nb;
    const int br = q / nb, bc = q - br * nb;
    int ti, tj;
    pair_decode(pair, ti, tj);
    const bool dtile = ti == tj;
    if (dtile && bc > br) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t tile = (int64_t)TBK * TBK;
    const Acc *p = partials + (int64_t)pair * splits_total * tile + (int64_t)(br * kGramRedB) * TBK + bc * kGramRedB;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < splits_total; ++s) {
        const Acc *ps = p + s * tile;
#pragma unroll
        for (int e = 0; e < 4; ++e) sum[e] += (double)ps[(ty + 8 * e) * TBK + tx];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) blk[ty + 8 * e][tx] = sum[e];
    __syncthreads();
    const int64_t I0 = (int64_t)ti * TBK + br * kGramRedB, J0 = (int64_t)tj * TBK + bc * kGramRedB;
    if (dtile && br == bc) {  // a block on the diagonal: both triangles from the lower one
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = ty + 8 * e, c = tx;
            if (I0 + r < n && J0 + c < n) M[(I0 + r) * n + J0 + c] = c <= r ? blk[r][c] : blk[c][r];
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = ty + 8 * e, c = tx;
        if (I0 + r < n && J0 + c < n) M[(I0 + r) * n + J0 + c] = blk[r][c];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = ty + 8 * e, r = tx;
        if (J0 + c < n && I0 + r < n) M[(J0 + c) * n + I0 + r] = blk[r][c];
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
    // BF16 operands of a large Gram: 256-row tiles (eight waves, one
    // workgroup per CU), which read each operand byte half as often as
    // 128-row tiles; else 128 (64 for FP64)
    p.TBK = prec == P64 ? 64 : (prec == PBF16 && n >= kGramWideMin ? 256 : 128);
    p.KS = prec == P64 ? 16 : (prec == P32 ? 32 : 64);
    p.acc_size = prec == P64 ? 8 : 4;
    int nt = (int)ceil_div(n, p.TBK);
    p.npairs = nt * (nt + 1) / 2;
    // about tn.gram_items blocks in flight (a quarter for 256-row tiles, one
    // workgroup per CU: rounded down, so that they fit one round), at least
    // tn.gram_min_stages stages per block
    int want = p.TBK == 256 ? (int)std::max<int64_t>(1, (tn.gram_items / 4) / ((int64_t)p.npairs * nterms))
                            : (int)std::max<int64_t>(1, ceil_div(tn.gram_items, (int64_t)p.npairs * nterms));
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

template <class P, int WTR, int WTC, int WR, int WC, class Acc>
static hipError_t launch_gram(const GramKArgs &g, bool vec, unsigned blocks, Acc *scratch, hipStream_t s) {
    constexpr size_t lds = gram_lds_bytes<P, WR * WTR>();
    if (vec) {
        lds_limit((const void *)k_gram<P, WTR, WTC, WR, WC, true>, lds);
        k_gram<P, WTR, WTC, WR, WC, true><<<blocks, 64 * WR * WC, lds, s>>>(g, scratch);
    } else {
        lds_limit((const void *)k_gram<P, WTR, WTC, WR, WC, false>, lds);
        k_gram<P, WTR, WTC, WR, WC, false><<<blocks, 64 * WR * WC, lds, s>>>(g, scratch);
    }
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
    const unsigned rblocks = (unsigned)(p.npairs * (p.TBK / kGramRedB) * (p.TBK / kGramRedB));
    if (prec == P64) {
        TK_HIP((launch_gram<PolF64<32>, 32, 32, 2, 2>(g, vec, blocks, (double *)scratch, s)));
        k_gram_reduce<double><<<rblocks, 256, 0, s>>>((const double *)scratch, p.splits_total, p.TBK, n, M);
    } else if (prec == P32) {
        TK_HIP((launch_gram<PolF32<64>, 64, 64, 2, 2>(g, vec, blocks, (float *)scratch, s)));
        k_gram_reduce<float><<<rblocks, 256, 0, s>>>((const float *)scratch, p.splits_total, p.TBK, n, M);
    } else {
        // direct LDS staging where every operand's extent fits the 32-bit
        // offsets of a buffer load
        bool dl = vec && p.TBK == 256;
        for (int t = 0; t < nterms && dl; ++t)
            dl = (((int64_t)n - 1) * g.t[t].s_row + (g.t[t].nchunks - 1) * g.t[t].s_chunk + g.t[t].chunk_len) * 2 <
                 (int64_t(1) << 31);
        if (dl) {
            k_gram_dl<kGramDlWaves><<<blocks, 64 * kGramDlWaves, 0, s>>>(g, (float *)scratch);
            TK_LAUNCHED();
        } else if (p.TBK == 256)
            TK_HIP((launch_gram<PolBF16<64>, 64, 128, 4, 2>(g, vec, blocks, (float *)scratch, s)));
        else
            TK_HIP((launch_gram<PolBF16<64>, 64, 64, 2, 2>(g, vec, blocks, (float *)scratch, s)));
        k_gram_reduce<float><<<rblocks, 256, 0, s>>>((const float *)scratch, p.splits_total, p.TBK, n, M);
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

// K stage of k_gemm: the policy's. Each stage's loads go into registers
// while the matrix cores work on the previous stage (the batched second
// stage of HOOI's chain and the core contractions, 64 x 64 outputs over
// K = 1000, are bound by those loads' latency). Stages of two and four
// times the depth (more loads in flight, more registers, fewer waves per
// SIMD) measured slower.
template <class P> struct GemmStage {
    static constexpr int KS = P::KS;
    static constexpr int LDK = P::LDK;
};
template <class P>
constexpr size_t gemm_lds_bytes() {
    return (size_t)2 * 64 * GemmStage<P>::LDK * sizeof(typename P::E);
}

template <class P, class TA, class TBm, class TO>
__global__ void __launch_bounds__(256) k_gemm(GemmKArgs g) {
    typedef typename P::E E;
    constexpr int WT = 32, BM = 64, BN = 64;
    constexpr int KS = GemmStage<P>::KS, LDK = GemmStage<P>::LDK;
    constexpr int NA = BM * KS / 256, NBL = BN * KS / 256;  // elements per thread and stage
    extern __shared__ __attribute__((aligned(16))) char gemm_smem[];
    E *As = reinterpret_cast<E *>(gemm_smem), *Bs = As + BM * LDK;
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

    // element u of the thread's share of a stage: A tile BM rows x KS (i
    // fastest when A is stored transposed, else k), B tile BN cols x KS (j
    // fastest)
    E ra[NA], rb[NBL];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256;
            int ii, kk;
            if (g.a_trans) {
                ii = e % BM;
                kk = e / BM;
            } else {
                kk = e % KS;
                ii = e / KS;
            }
            const int64_t i = m0 + ii, k = k0 + kk;
            ra[u] = (i < g.M && k < kend) ? cvt<E>(g.a_trans ? A[k * g.lda + i] : A[i * g.lda + k]) : (E)0;
        }
#pragma unroll
        for (int u = 0; u < NBL; ++u) {
            const int e = tid + u * 256;
            const int jj = e % BN, kk = e / BN;
            const int64_t j = n0 + jj, k = k0 + kk;
            rb[u] = (j < g.N && k < kend) ? cvt<E>(B[k * g.ldb + j]) : (E)0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + u * 256;
            const int ii = g.a_trans ? e % BM : e / KS, kk = g.a_trans ? e / BM : e % KS;
            As[ii * LDK + kk] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < NBL; ++u) {
            const int e = tid + u * 256;
            Bs[(e % BN) * LDK + e / BN] = rb[u];
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += KS) {
        store();
        __syncthreads();
        // the next stage's loads in flight while the matrix cores work
        if (k0 + KS < kend) load(k0 + KS);
#pragma unroll 1
        for (int q = 0; q < KS; q += P::KI)
#pragma unroll
            for (int a = 0; a < P::NB; ++a)
#pragma unroll
                for (int b = 0; b < P::NB; ++b)
                    P::template mma_ld<LDK>(As, Bs, wr * WT + a * P::BT, wc * WT + b * P::BT, q, acc[a][b]);
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
    g.kper = ceil_div(ceil_div(a.K, g.splitk), GemmStage<P>::KS) * GemmStage<P>::KS;
    if (g.splitk > 1) g.splitk = (int)ceil_div(a.K, g.kper);
    dim3 grid((unsigned)ceil_div(a.N, 64), (unsigned)ceil_div(a.M, 64), (unsigned)(a.batch * g.splitk));
    lds_limit((const void *)k_gemm<P, TA, TBm, TO>, gemm_lds_bytes<P>());
    k_gemm<P, TA, TBm, TO><<<grid, 256, gemm_lds_bytes<P>(), s>>>(g);
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
