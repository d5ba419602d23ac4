// "J leading eigenvectors" of a symmetric positive semi-definite Gram M
// (every figure of Section 4), in FP64.
//
// For M = S S^T (all Grams here) the leading eigenvectors of M M^T, as SP and
// MP write them, are those of M, in the same order; the solver works on M.
//
// Small matrices (n <= kDirectMax) are diagonalised exactly by parallel
// cyclic Jacobi in one workgroup. Larger ones use block subspace iteration
// with b = J + p columns:
//   Rayleigh-Ritz (H = X^T M X, Jacobi) -> Ritz vectors, values, residuals;
//   leading Ritz pairs with tiny residuals are locked (kept out of the
//   filter, which would otherwise let an isolated large eigenvalue swamp the
//   block);
//   a Chebyshev filter of degree d on the remaining columns damps [0, mu]
//   (mu = smallest Ritz value of the block) and amplifies the top;
//   the filtered columns are re-orthogonalised against the locked ones and
//   orthonormalised by shifted CholeskyQR (one shifted pass, one plain).
// It stops when a residual estimate of the error of the sum of the J
// leading Ritz values, sum_j r_j^2 / (theta_j - mu) (the quadratic bound of
// a Ritz value by its residual r_j and its distance to the rest of the
// block's spectrum), is at most tol times the sum; when that sum changes by
// at most tol (relative) across a filter of full degree; or when all J are
// locked. A warm start (the previous sweep's factors) is often converged on
// arrival, so its filter starts at a low degree that doubles per step up to
// the full one.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace tk {

constexpr int kDirectMax = 140;   // Jacobi on M itself up to this size
constexpr int kJacobiVLds = 100;  // H and V both in LDS up to this size
constexpr int kMaxBlock = 140;    // H in LDS up to this size
constexpr int kJacobiThreads = 1024;

// p extra columns: a wider block converges in fewer filter steps but each
// Rayleigh-Ritz and CholeskyQR step costs more; on flat spectra (uniform
// data, n = 1000, J = 50) six took the least time of 4, 6, 8, 12, 16 and 25.
int eig_block_width(int n, int J) {
    if (n <= kDirectMax) return n;
    int p = std::min(32, std::max(6, J / 8));
    int b = std::min(J + p, kMaxBlock);
    b = std::min(b, n);
    return std::max(b, J);
}

void lds_limit(const void *fn, size_t bytes) {
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> given;
    std::lock_guard<std::mutex> g(mu);
    size_t &v = given[fn];
    if (bytes > v) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        v = bytes;
    }
}

// Per-thread pinned host buffer for the solver's small read-backs (1024
// doubles, allocated on a thread's first solve and kept for its life), or
// null when pinned memory is not to be had.
static double *pinned_scratch() {
    thread_local double *p = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void **)&p, sizeof(double) * 1024, hipHostMallocDefault) != hipSuccess) p = nullptr;
    }
    return p;
}

// Wait for the stream's work by polling (the solver's host decisions follow
// each wait at once; polling returns sooner than a blocking wait), then a
// blocking wait if it takes longer than about a tenth of a second.
static hipError_t wait_stream(hipStream_t s) {
    for (int i = 0; i < 100000; ++i) {
        const hipError_t e = hipStreamQuery(s);
        if (e != hipErrorNotReady) return e;
    }
    return hipStreamSynchronize(s);
}

// ------------------------------------------------------------------ small kernels
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// Deterministic pseudo-normal numbers (Box-Muller on a counter hash).
__device__ inline double hash_normal(uint64_t seed, uint64_t ctr) {
    uint64_t a = mix64(seed ^ mix64(2 * ctr)), b = mix64(seed ^ mix64(2 * ctr + 1));
    double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void k_random_cols(double *X, int64_t n, int ld, int c0, int c1, uint64_t seed) {
    const int w = c1 - c0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * w; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / w;
        int j = c0 + (int)(t - i * w);
        X[i * ld + j] = hash_normal(seed, (uint64_t)i * 1000003ull + (uint64_t)j);
    }
}

// Column norms of X[:, c0:c1] (one block per column), then scale to unit
// norm; a column whose norm is below 1e-13 of the largest is replaced by a
// pseudo-random one (rank-deficient blocks).
__global__ void k_colnorm(const double *X, int64_t n, int ld, int c0, double *norms) {
    const int j = c0 + blockIdx.x;
    double acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double v = X[i * ld + j];
        acc += v * v;
    }
    __shared__ double ws[16];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i];
        norms[blockIdx.x] = sqrt(t);
    }
}
// X[:, c0 + j] = src[:, c0 + j] / norms[j] (both leading dimension ld; src may be X).
__global__ void k_colscale(const double *src, double *X, int64_t n, int ld, int c0, int w, const double *norms,
                           uint64_t seed) {
    __shared__ double mx;
    if (threadIdx.x == 0) {
        double m = 0;
        for (int j = 0; j < w; ++j) m = fmax(m, norms[j]);
        mx = m;
    }
    __syncthreads();
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * w; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / w;
        int jj = (int)(t - i * w);
        double nv = norms[jj];
        if (nv > 1e-13 * mx && nv > 0)
            X[i * ld + c0 + jj] = src[i * ld + c0 + jj] / nv;
        else
            X[i * ld + c0 + jj] = hash_normal(seed, (uint64_t)i * 1000003ull + (uint64_t)(c0 + jj)) / sqrt((double)n);
    }
}

// Upper Cholesky factor R of S + shift*trace(S)*I (S is w x w with leading
// dimension lds) and its inverse, in one workgroup with everything in LDS.
// Right-looking elimination with one barrier per column: the trailing update
// of step k uses row k unscaled (A_ij -= A_ki A_kj / A_kk) and row k is scaled
// by 1/sqrt(A_kk) during step k+1, when no thread reads it. Non-positive
// pivots are clamped to a tiny positive value (the caller's block then keeps
// a direction it cannot resolve instead of failing). The inverse is formed
// column by column (one thread per column) into the strictly lower triangle,
// transposed, with its diagonal kept apart.
__global__ void __launch_bounds__(1024) k_chol_inv(const double *S, int lds, int w, double shift, double *Rinv) {
    extern __shared__ double A[];  // w*w, then w for the inverse's diagonal
    double *dinv = A + (size_t)w * w;
    __shared__ double tr;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int t = tid; t < w * w; t += nth) {
        int i = t / w, j = t - i * w;
        A[t] = 0.5 * (S[i * lds + j] + S[j * lds + i]);
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0;
        for (int i = 0; i < w; ++i) s += A[i * w + i];
        tr = s;
    }
    __syncthreads();
    const double add = shift * tr;
    for (int i = tid; i < w; i += nth) A[i * w + i] += add;
    __syncthreads();
    const double tiny = 1e-300 + 1e-30 * (tr > 0 ? tr : 1.0);
    for (int k = 0; k < w; ++k) {
        if (k > 0) {
            // scale row k-1 by the square root of its (clamped) pivot; no
            // thread reads row k-1 during this step
            const double pk = fmax(A[(k - 1) * w + (k - 1)], tiny);
            const double sq = sqrt(pk);
            for (int j = k + tid; j < w; j += nth) A[(k - 1) * w + j] /= sq;
        }
        const double rd = 1.0 / fmax(A[k * w + k], tiny);
        // trailing upper triangle (i, j), k < i <= j: thread (g, c) with
        // g < groups = nth / w takes column k+1+c and rows k+1+g, k+1+g+groups, ...
        // (w <= 140 < nth)
        const int groups = nth / w;
        const int g = tid / w, c = tid - g * w;
        if (g < groups) {
            const int j = k + 1 + c;
            if (j < w) {
                const double akj = A[k * w + j] * rd;
                for (int i = k + 1 + g; i <= j; i += groups) A[i * w + j] -= A[k * w + i] * akj;
            }
        }
        __syncthreads();
    }
    for (int k = tid; k < w; k += nth) A[k * w + k] = sqrt(fmax(A[k * w + k], tiny));
    __syncthreads();
    // R is now the upper triangle of A. Its inverse is upper triangular too;
    // row i of it needs only rows below i: Rinv[i][j] = (delta_ij - sum_{k=i+1..j}
    // R[i][k] Rinv[k][j]) / R[i][i], parallel over j. Rinv[i][j] (i < j) is
    // kept at A[j][i] (strictly lower triangle, transposed), its diagonal in dinv.
    for (int j = tid; j < w; j += nth) dinv[j] = 1.0 / A[j * w + j];
    __syncthreads();
    // Each dot product is split over 4 consecutive lanes and combined with
    // two shuffles (groups of 4 lanes are always wholly active).
    for (int i = w - 2; i >= 0; --i) {
        const double rii = dinv[i];
        const int ncol = w - 1 - i;
        for (int t = tid; t < ncol * 4; t += nth) {
            const int j = i + 1 + (t >> 2), part = t & 3;
            double v = 0.0;
            for (int k = i + 1 + part; k < j; k += 4) v -= A[i * w + k] * A[j * w + k];
            if (part == 0) v -= A[i * w + j] * dinv[j];  // k = j term
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            if (part == 0) A[j * w + i] = v * rii;
        }
        __syncthreads();
    }
    for (int t = tid; t < w * w; t += nth) {
        int i = t / w, j = t - i * w;
        double v = 0;
        if (i == j)
            v = dinv[j];
        else if (i < j)
            v = A[j * w + i];
        Rinv[t] = v;
    }
}

// Blocked form of the same factor and inverse for w <= kCholBlkMax, on the
// matrix padded to W = 16 * ceil(w / 16) with an identity block (which stays
// decoupled). Each step factors a 16 x 16 diagonal block in the registers of
// one wave (lane i holds row i; column entries of other rows are fetched
// with readlane, so the serial column chain has no LDS round trips) and
// inverts it there, then the panel below (times the block inverse, transposed)
// and the trailing lower tiles (L_ib L_jb^T subtracted) are FP64 MFMA
// products. The inverse of L is completed by block forward substitution,
// Li_ib,jb = -Li_ib,ib sum_kb L_ib,kb Li_kb,jb, one block row at a time, and
// R^-1 = (L^-1)^T is written out. Same pivot clamping as k_chol_inv.
constexpr int kCholBlkMax = 96;
constexpr int kCholBlkThreads = 256;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x of lane l (l uniform across the wave)
__device__ inline double read_lane(double x, int l) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ void __launch_bounds__(kCholBlkThreads) k_chol_inv_blk(const double *S, int lds, int w, double shift,
                                                                  double *Rinv) {
    extern __shared__ double sm[];
    const int W = (w + 15) & ~15, NB = W / 16;
    double *A = sm;                   // W x W: lower factor L, built in place
    double *Li = sm + (size_t)W * W;  // W x W: L^-1 (lower)
    double *scr = Li + (size_t)W * W; // one 16 x 16 tile per wave
    __shared__ double tr;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = kCholBlkThreads / 64;
    const int l16 = lane & 15, l4 = lane >> 4;
    for (int t = tid; t < W * W; t += kCholBlkThreads) {
        const int i = t / W, j = t - i * W;
        A[t] = (i < w && j < w) ? 0.5 * (S[(int64_t)i * lds + j] + S[(int64_t)j * lds + i]) : (i == j ? 1.0 : 0.0);
        Li[t] = 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double sum = 0;
        for (int i = 0; i < w; ++i) sum += A[i * W + i];
        tr = sum;
    }
    __syncthreads();
    const double add = shift * tr;
    for (int i = tid; i < w; i += kCholBlkThreads) A[i * W + i] += add;
    __syncthreads();
    const double tiny = 1e-300 + 1e-30 * (tr > 0 ? tr : 1.0);
    for (int kb = 0; kb < NB; ++kb) {
        const int o = kb * 16;
        if (wid == 0) {
            double r[16], li[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) r[j] = lane < 16 ? A[(o + lane) * W + o + j] : 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const double d = fmax(read_lane(r[c], c), tiny);
                const double l = sqrt(d), rl = 1.0 / l;
                r[c] = lane > c ? r[c] * rl : (lane == c ? l : r[c]);
#pragma unroll
                for (int j = c + 1; j < 16; ++j) {
                    const double ljc = read_lane(r[c], j);
                    if (lane >= j) r[j] -= r[c] * ljc;
                }
            }
            // lane j builds column j of the block's inverse
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                double acc = lane == i ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < i; ++k) acc -= read_lane(r[k], i) * li[k];
                li[i] = lane <= i ? acc / read_lane(r[i], i) : 0.0;
            }
            if (lane < 16) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j <= lane) A[(o + lane) * W + o + j] = r[j];
                    Li[(o + j) * W + o + lane] = li[j];
                }
            }
        }
        __syncthreads();
        // panel: L_ib,kb = A_ib,kb Li_kb,kb^T
        for (int ib = kb + 1 + wid; ib < NB; ib += nw) {
            doublex4 acc = {0, 0, 0, 0};
            for (int kc = 0; kc < 4; ++kc) {
                const double a = A[(ib * 16 + l16) * W + o + kc * 4 + l4];
                const double b = Li[(o + l16) * W + o + kc * 4 + l4];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            for (int v = 0; v < 4; ++v) A[(ib * 16 + 4 * v + l4) * W + o + l16] = acc[v];
        }
        __syncthreads();
        // trailing lower tiles: A_ib,jb -= L_ib,kb L_jb,kb^T (kb < jb <= ib)
        const int nt = NB - kb - 1;
        for (int t = wid; t < nt * (nt + 1) / 2; t += nw) {
            int x = t, rr = 0;
            while (x > rr) {
                x -= rr + 1;
                ++rr;
            }
            const int ib = kb + 1 + rr, jb = kb + 1 + x;
            doublex4 acc;
            for (int v = 0; v < 4; ++v) acc[v] = A[(ib * 16 + 4 * v + l4) * W + jb * 16 + l16];
            for (int kc = 0; kc < 4; ++kc) {
                const double a = A[(ib * 16 + l16) * W + o + kc * 4 + l4];
                const double b = A[(jb * 16 + l16) * W + o + kc * 4 + l4];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, b, acc, 0, 0, 0);
            }
            for (int v = 0; v < 4; ++v) A[(ib * 16 + 4 * v + l4) * W + jb * 16 + l16] = acc[v];
        }
        __syncthreads();
    }
    double *sc = scr + wid * 256;
    for (int ib = 1; ib < NB; ++ib) {
        for (int jb = wid; jb < ib; jb += nw) {
            doublex4 acc = {0, 0, 0, 0};
            for (int kb = jb; kb < ib; ++kb)
                for (int kc = 0; kc < 4; ++kc) {
                    const double a = A[(ib * 16 + l16) * W + kb * 16 + kc * 4 + l4];
                    const double b = Li[(kb * 16 + kc * 4 + l4) * W + jb * 16 + l16];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
            wave_sync();
            for (int v = 0; v < 4; ++v) sc[(4 * v + l4) * 16 + l16] = acc[v];
            wave_sync();
            doublex4 acc2 = {0, 0, 0, 0};
            for (int kc = 0; kc < 4; ++kc) {
                const double a = Li[(ib * 16 + l16) * W + ib * 16 + kc * 4 + l4];
                const double b = sc[(kc * 4 + l4) * 16 + l16];
                acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc2, 0, 0, 0);
            }
            for (int v = 0; v < 4; ++v) Li[(ib * 16 + 4 * v + l4) * W + jb * 16 + l16] = -acc2[v];
        }
        __syncthreads();
    }
    for (int t = tid; t < w * w; t += kCholBlkThreads) {
        const int i = t / w, j = t - i * w;
        Rinv[t] = (i <= j) ? Li[j * W + i] : 0.0;
    }
}

// Parallel cyclic Jacobi on the symmetric b x b matrix Hin (leading
// dimension ldh). Sixteen waves: a round is bound by its LDS traffic and two
// barriers, and 1024 threads give a 62 x 62 sweep in 100 us where 512 took
// 119 us (same rotations, same bits). Outputs the eigenvalues in descending order (theta) and
// the matching eigenvectors as columns of Vout (b x b row-major).
// With max_sweeps > 1 the matrix counts as diagonal, and no further sweep is
// made, once its off-diagonal squares sum to at most off2 times all squares;
// the test comes before each sweep, so an input that is already diagonal
// enough costs none. A single-sweep call makes no test.
template <bool V_LDS>
__global__ void __launch_bounds__(kJacobiThreads) k_jacobi(const double *Hin, int ldh, int b, int max_sweeps,
                                                           double off2, double *theta, double *Vout,
                                                           double *Vglob) {
    extern __shared__ double sm[];
    double *H = sm;
    double *V = V_LDS ? sm + (size_t)b * b : Vglob;
    const int m = b + (b & 1), half = m / 2;
    __shared__ double cs[(kMaxBlock + 1) / 2], sn[(kMaxBlock + 1) / 2];
    __shared__ int pp[(kMaxBlock + 1) / 2], qq[(kMaxBlock + 1) / 2];
    __shared__ double red[32];
    __shared__ double hmax;
    __shared__ int done, any_rot;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int t = tid; t < b * b; t += nth) {
        int i = t / b, j = t - i * b;
        H[t] = 0.5 * (Hin[(int64_t)i * ldh + j] + Hin[(int64_t)j * ldh + i]);
        V[t] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double m0 = 0;
        for (int i = 0; i < b; ++i) m0 = fmax(m0, fabs(H[i * b + i]));
        hmax = m0;
    }
    // static thread maps (no divisions inside the rounds):
    // blocks (k1, k2) of the pair grid: k2 = tid % half fixed, k1 = tid / half + s*bstep
    const int bstep = nth / half > 0 ? nth / half : 1;
    const int bk2 = tid % half, bk1 = tid / half;
    const bool bact = tid < bstep * half;
    // V rows: pair k = tid % half fixed, row = tid / half + s*bstep
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (max_sweeps > 1) {
            double off = 0, dia = 0;
            for (int t = tid; t < b * b; t += nth) {
                int i = t / b, j = t - i * b;
                double v = H[t] * H[t];
                if (i == j)
                    dia += v;
                else
                    off += v;
            }
            for (int d = 32; d >= 1; d >>= 1) {
                off += __shfl_xor(off, d, 64);
                dia += __shfl_xor(dia, d, 64);
            }
            if ((tid & 63) == 0) {
                red[tid >> 6] = off;
                red[16 + (tid >> 6)] = dia;
            }
            __syncthreads();
            if (tid == 0) {
                double o = 0, dd = 0;
                for (int i = 0; i < (nth >> 6); ++i) {
                    o += red[i];
                    dd += red[16 + i];
                }
                done = (o <= off2 * (o + dd)) || (dd == 0.0);
            }
            __syncthreads();
            if (done) break;
        }
        if (tid == 0) any_rot = 0;
        int nrot = 0;
        for (int r = 0; r < m - 1; ++r) {
            for (int k = tid; k < half; k += nth) {
                // round r of the round-robin schedule: pair 0 is (0, 1 + r),
                // pair k is (1 + (k + r) mod (m - 1), 1 + (m - 1 - k + r) mod
                // (m - 1)); both sums lie below 2 (m - 1), so one conditional
                // subtraction takes the remainder
                int a, c;
                if (k == 0) {
                    a = 0;
                    c = 1 + r;
                } else {
                    int x = k + r, y = m - 1 - k + r;
                    if (x >= m - 1) x -= m - 1;
                    if (y >= m - 1) y -= m - 1;
                    a = 1 + x;
                    c = 1 + y;
                }
                int p = a < c ? a : c, q = a < c ? c : a;
                double cc = 1.0, ss = 0.0;
                if (q < b) {
                    double apq = H[p * b + q], app = H[p * b + p], aqq = H[q * b + q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-16 * hmax) {
                        nrot = 1;
                        double tau = (aqq - app) / (2.0 * apq);
                        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        if (fabs(tau) > 1e150) t = 0.5 / tau;
                        cc = rsqrt(1.0 + t * t);
                        ss = t * cc;
                    }
                }
                cs[k] = cc;
                sn[k] = ss;
                pp[k] = p;
                qq[k] = q;
            }
            __syncthreads();
            // H <- G^T H G on 2x2 blocks (pair k1 rows, pair k2 columns)
            if (bact) {
                const int k2 = bk2;
                const int p2 = pp[k2], q2 = qq[k2];
                const double c2 = cs[k2], s2 = sn[k2];
                for (int k1 = bk1; k1 < half; k1 += bstep) {
                    const int p1 = pp[k1], q1 = qq[k1];
                    if (q1 >= b || q2 >= b) {  // a pair with the padding index of odd b
                        // the idle real index x of the dummy pair meets the
                        // rotation of the other pair on one side only
                        if (q1 >= b && q2 < b) {
                            const int x = p1;
                            double hp = H[x * b + p2], hq = H[x * b + q2];
                            double np_ = c2 * hp - s2 * hq, nq = s2 * hp + c2 * hq;
                            H[x * b + p2] = np_;
                            H[x * b + q2] = nq;
                            H[p2 * b + x] = np_;
                            H[q2 * b + x] = nq;
                        }
                        continue;
                    }
                    const double c1 = cs[k1], s1 = sn[k1];
                    double a = H[p1 * b + p2], bb = H[p1 * b + q2], c = H[q1 * b + p2], d = H[q1 * b + q2];
                    double za, zb, zc, zd;
                    if (k1 == k2) {
                        const double t1 = c1 != 0.0 ? s1 / c1 : 0.0;
                        za = a - t1 * bb;
                        zd = d + t1 * bb;
                        zb = 0.0;
                        zc = 0.0;
                        if (s1 == 0.0) {
                            za = a;
                            zd = d;
                            zb = bb;
                            zc = c;
                        }
                    } else {
                        double ya = c1 * a - s1 * c, yb = c1 * bb - s1 * d;
                        double yc = s1 * a + c1 * c, yd = s1 * bb + c1 * d;
                        za = c2 * ya - s2 * yb;
                        zb = s2 * ya + c2 * yb;
                        zc = c2 * yc - s2 * yd;
                        zd = s2 * yc + c2 * yd;
                    }
                    H[p1 * b + p2] = za;
                    H[p1 * b + q2] = zb;
                    H[q1 * b + p2] = zc;
                    H[q1 * b + q2] = zd;
                }
                // V <- V G: rows bk1, bk1 + bstep, ... of pair k2
                if (q2 < b) {
                    for (int row = bk1; row < b; row += bstep) {
                        double vp = V[row * b + p2], vq = V[row * b + q2];
                        V[row * b + p2] = c2 * vp - s2 * vq;
                        V[row * b + q2] = s2 * vp + c2 * vq;
                    }
                }
            }
            __syncthreads();
        }
        if (nrot) any_rot = 1;
        __syncthreads();
        if (!any_rot) break;
    }
    // sort by eigenvalue, descending (ties by index)
    for (int i = tid; i < b; i += nth) {
        double di = H[i * b + i];
        int rank = 0;
        for (int j = 0; j < b; ++j) {
            double dj = H[j * b + j];
            rank += (dj > di) || (dj == di && j < i);
        }
        theta[rank] = di;
        for (int r = 0; r < b; ++r) Vout[r * b + rank] = V[r * b + i];
    }
}

// Residual norms ||W[:,j] - theta_j X[:,j]|| (one block per column).
__global__ void k_resid(const double *W, const double *X, const double *theta, int64_t n, int b, double *res) {
    const int j = blockIdx.x;
    const double th = theta[j];
    double acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double r = W[i * b + j] - th * X[i * b + j];
        acc += r * r;
    }
    __shared__ double ws[16];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i];
        res[j] = sqrt(t);
    }
}

// F[:, j] = sign_j * X[:, j] for j < J, sign making the largest-magnitude
// entry (first one on ties) positive. One block per column.
__global__ void k_extract(const double *X, int64_t n, int ldx, int J, double *F, const int *colmap) {
    const int j = blockIdx.x;
    const int src = colmap ? colmap[j] : j;
    double best = -1;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double a = fabs(X[i * ldx + src]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    __shared__ double sb[256];
    __shared__ int64_t si[256];
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int d = blockDim.x / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) {
            double o = sb[threadIdx.x + d];
            int64_t oi = si[threadIdx.x + d];
            if (o > sb[threadIdx.x] || (o == sb[threadIdx.x] && oi < si[threadIdx.x])) {
                sb[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const double sgn = X[si[0] * ldx + src] < 0 ? -1.0 : 1.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) F[i * J + j] = sgn * X[i * ldx + src];
}

// M <- M - sum_l theta_l x_l x_l^T over the columns X[:, c0:c0+k] (leading
// dimension ldx); symmetric bit for bit (theta * (x_r x_c)).
__global__ void k_deflate(double *M, int64_t n, const double *X, int ldx, int c0, int k, const double *theta) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * n; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = t / n, c = t - r * n;
        double acc = 0;
        for (int l = 0; l < k; ++l) acc += theta[l] * (X[r * ldx + c0 + l] * X[c * ldx + c0 + l]);
        M[t] -= acc;
    }
}

template <class TO>
__global__ void k_convert(const double *in, TO *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (TO)(float)in[i];
}
template <>
__global__ void k_convert<double>(const double *in, double *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}
template <class TO>
hipError_t convert_f64(const double *in, TO *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = std::min<int64_t>(ceil_div(n, 256), 65536);
    k_convert<TO><<<(unsigned)g, 256, 0, s>>>(in, out, n);
    TK_LAUNCHED();
    return hipSuccess;
}
template hipError_t convert_f64<float>(const double *, float *, int64_t, hipStream_t);
template hipError_t convert_f64<double>(const double *, double *, int64_t, hipStream_t);
template hipError_t convert_f64<bf16>(const double *, bf16 *, int64_t, hipStream_t);

// ------------------------------------------------------------------ skinny FP64 products
// C (M x N, row-major, ldc) = alpha * op(A) B + beta * E1 + gamma * E2 with
// op(A) = A (M x K, row-major, lda) or A^T (A stored K x M), B K x N
// (row-major, ldb), N <= kSkinnyN, and E1, E2 laid out as C. Every product of
// the eigensolver has this shape: M X (n x n times n x w), X^T Y (w x n times
// n x w) and X V (n x w times w x w).
//
// FP64 MFMA 16x16x4 (lane l holds A[l%16][l/16] and B[l/16][l%16]; result v
// lands in row 4v + l/16, column l%16). A workgroup owns a strip of 16 rows,
// all columns, and one K range; its four waves interleave over that range in
// steps of 4 (so the waves of a workgroup read the same cache lines) and are
// combined in LDS in a fixed order. With S > 1 K ranges, the workgroups write
// partial strips and a second kernel sums them in a fixed order, so results
// do not depend on scheduling.
constexpr int kSkinnyN = 144;

struct SkinnyArgs {
    int M, N, K;
    const double *A;
    int64_t lda;
    int at;
    const double *B;
    int64_t ldb;
    double *C;
    int64_t ldc;
    double alpha, beta, gamma;
    const double *E1, *E2;
    int S, Kc;
    double *part;
};

__device__ inline void skinny_out(const SkinnyArgs &g, int i, int j, double acc) {
    const int64_t o = (int64_t)i * g.ldc + j;
    double r = g.alpha * acc;
    if (g.E1) r += g.beta * g.E1[o];
    if (g.E2) r += g.gamma * g.E2[o];
    g.C[o] = r;
}

template <int NT>
__global__ void __launch_bounds__(256) k_skinny(SkinnyArgs g) {
    extern __shared__ double red[];  // [4][16][NT*16]
    constexpr int NC = NT * 16;
    const int strip = blockIdx.x / g.S, sp = blockIdx.x - strip * g.S;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = strip * 16 + (l & 15), kq = l >> 4;
    const int kb = sp * g.Kc, ke = min(g.K, kb + g.Kc);
    doublex4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = doublex4{0, 0, 0, 0};
#pragma unroll 2
    for (int k0 = kb + 4 * wave; k0 < ke; k0 += 16) {
        const int k = k0 + kq;
        const bool kin = k < ke;
        double a = 0.0;
        if (kin && i < g.M) a = g.at ? g.A[(int64_t)k * g.lda + i] : g.A[(int64_t)i * g.lda + k];
        double bv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = t * 16 + (l & 15);
            bv[t] = (kin && j < g.N) ? g.B[(int64_t)k * g.ldb + j] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[t], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 16 + 4 * v + (l >> 4)) * NC + t * 16 + (l & 15)] = acc[t][v];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * NC; e += 256) {
        const double sum = ((red[e] + red[16 * NC + e]) + red[32 * NC + e]) + red[48 * NC + e];
        const int r = e / NC, j = e - r * NC;
        if (g.S == 1) {
            if (strip * 16 + r < g.M && j < g.N) skinny_out(g, strip * 16 + r, j, sum);
        } else {
            g.part[((int64_t)(strip * g.S + sp) * 16 + r) * NC + j] = sum;
        }
    }
}

// Short K (<= kSkinnyWideMaxK): TPW adjacent 16 x 16 tiles of one 16-row strip
// of C per workgroup of 16 waves, which interleave over K in steps of 4
// (consecutive waves read consecutive K) and are summed in LDS in a fixed
// order. No partial strips and no second launch.
constexpr int kSkinnyWideMaxK = 2048;
constexpr int kSkinnyWideWaves = 16;
template <int TPW, bool AT>
__global__ void __launch_bounds__(64 * kSkinnyWideWaves) k_skinny_wide(SkinnyArgs g, int NG) {
    extern __shared__ double red[];  // [waves][TPW][256]
    constexpr int U = 4;             // K steps whose loads are in flight together
    constexpr int STEP = 4 * kSkinnyWideWaves;
    const int strip = blockIdx.x / NG, t0 = (blockIdx.x - strip * NG) * TPW;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = strip * 16 + (l & 15), kq = l >> 4;
    // out-of-range rows, columns and K steps load from a valid address and are
    // zeroed afterwards, so the loads carry no branches and can all be in flight
    const bool iok = i < g.M;
    const int ic = iok ? i : g.M - 1;
    bool jok[TPW];
    int jc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int j = (t0 + u) * 16 + (l & 15);
        jok[u] = j < g.N;
        jc[u] = jok[u] ? j : g.N - 1;
    }
    doublex4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = doublex4{0, 0, 0, 0};
    for (int k0 = 4 * wave; k0 < g.K; k0 += STEP * U) {
        double a[U], bv[U][TPW];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = k0 + q * STEP + kq;
            const bool kin = k < g.K;
            const int kc = kin ? k : g.K - 1;
            const double av = AT ? g.A[(int64_t)kc * g.lda + ic] : g.A[(int64_t)ic * g.lda + kc];
            a[q] = av * ((kin && iok) ? 1.0 : 0.0);  // a product, not a select: keeps the load unpredicated
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const double b = g.B[(int64_t)kc * g.ldb + jc[u]];
                bv[q][u] = b * ((kin && jok[u]) ? 1.0 : 0.0);
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int u = 0; u < TPW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], bv[q][u], acc[u], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * TPW + u) * 256 + (4 * v + (l >> 4)) * 16 + (l & 15)] = acc[u][v];
    __syncthreads();
    for (int e = threadIdx.x; e < TPW * 256; e += 64 * kSkinnyWideWaves) {
        const int u = e >> 8, q = e & 255, r = q >> 4, c = q & 15;
        double sum = 0.0;
        for (int w = 0; w < kSkinnyWideWaves; ++w) sum += red[(w * TPW + u) * 256 + q];
        const int jj = (t0 + u) * 16 + c;
        if (strip * 16 + r < g.M && jj < g.N) skinny_out(g, strip * 16 + r, jj, sum);
    }
}
constexpr int kSkinnyTPW = 1;  // 2 and 4 (fewer re-reads of A, fewer workgroups) measured slower

__global__ void k_skinny_reduce(SkinnyArgs g, int NC) {
    const int64_t total = (int64_t)g.M * g.N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / g.N), j = (int)(e - (int64_t)i * g.N);
        const int strip = i >> 4, r = i & 15;
        const double *p = g.part + ((int64_t)strip * g.S * 16 + r) * NC + j;
        double sum = 0.0;
        for (int q = 0; q < g.S; ++q) sum += p[(int64_t)q * 16 * NC];
        skinny_out(g, i, j, sum);
    }
}

// Narrow products (N <= 8 columns, A row-major): the N columns of B are
// staged in LDS once per workgroup ([K][NB], zero beyond N), then each wave
// takes whole rows of A, lanes striding over K with coalesced row reads,
// and reduces its N sums across the wave (fixed order). Power steps and
// products with few active columns read all of A for a handful of columns;
// this spends them over many workgroups instead of one 16-row strip each.
constexpr int kNarrowRows = 8;  // rows per workgroup (two per wave)
template <int NB>
__global__ void __launch_bounds__(256) k_narrow(SkinnyArgs g) {
    extern __shared__ double xs[];  // [K][NB]
    for (int t = threadIdx.x; t < g.K * NB; t += 256) {
        const int k = t / NB, j = t - k * NB;
        xs[t] = j < g.N ? g.B[(int64_t)k * g.ldb + j] : 0.0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int rr = 0; rr < kNarrowRows / 4; ++rr) {
        const int i = blockIdx.x * kNarrowRows + wave * (kNarrowRows / 4) + rr;
        if (i >= g.M) break;
        const double *arow = g.A + (int64_t)i * g.lda;
        double acc[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j] = 0.0;
        for (int k = l; k < g.K; k += 64) {
            const double a = arow[k];
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[j] = __builtin_fma(a, xs[k * NB + j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            for (int d = 32; d >= 1; d >>= 1) acc[j] += __shfl_xor(acc[j], d, 64);
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (l == j && j < g.N) skinny_out(g, i, j, acc[j]);
    }
}

template <int NB>
static void narrow_launch(const SkinnyArgs &g, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)g.K * NB;
    lds_limit((const void *)k_narrow<NB>, lds);
    k_narrow<NB><<<(unsigned)ceil_div(g.M, kNarrowRows), 256, lds, s>>>(g);
}

// The narrow form applies (row-major A, at most 8 columns whose K x 8 block
// fits 64 KiB of LDS).
static int narrow_width(const SkinnyArgs &g) {
    if (g.at || g.N > 8 || g.K < 64) return 0;
    const int nb = g.N <= 1 ? 1 : (g.N <= 2 ? 2 : (g.N <= 4 ? 4 : 8));
    return (int64_t)g.K * nb * 8 <= 65536 ? nb : 0;
}

// K ranges: enough workgroups to cover the chip (about 512), each range at
// least 64 long and a multiple of 16.
static void skinny_split(int M, int K, int *S, int *Kc) {
    const int strips = (M + 15) / 16;
    int s = std::max(1, std::min(512 / std::max(1, strips), K / 64));
    int kc = (int)ceil_div(K, s);
    kc = (int)ceil_div(kc, 16) * 16;
    *S = (int)ceil_div(K, std::max(kc, 1));
    *Kc = kc;
}
static int64_t skinny_part_elems(int M, int N, int K) {
    int S, Kc;
    skinny_split(M, K, &S, &Kc);
    if (S <= 1) return 0;
    return (int64_t)((M + 15) / 16) * S * 16 * ((N + 15) / 16 * 16);
}

template <int NT>
static void skinny_launch(const SkinnyArgs &g, hipStream_t s) {
    const int strips = (g.M + 15) / 16;
    const size_t lds = sizeof(double) * 4 * 16 * NT * 16;
    lds_limit((const void *)k_skinny<NT>, lds);
    k_skinny<NT><<<(unsigned)(strips * g.S), 256, lds, s>>>(g);
}

static hipError_t skinny(SkinnyArgs g, double *part, int64_t part_elems, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.N > kSkinnyN) return hipErrorInvalidValue;
    const int NT = (g.N + 15) / 16;
    if (g.K <= 0) {  // empty sum: the epilogue alone (the reduction over S = 0 parts)
        g.S = 0;
        g.part = nullptr;
        const int64_t total = (int64_t)g.M * g.N;
        k_skinny_reduce<<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 2048), 256, 0, s>>>(g, NT * 16);
        TK_LAUNCHED();
        return hipSuccess;
    }
    if (const int nb = narrow_width(g)) {
        g.S = 1;
        g.Kc = g.K;
        g.part = nullptr;
        switch (nb) {
            case 1: narrow_launch<1>(g, s); break;
            case 2: narrow_launch<2>(g, s); break;
            case 4: narrow_launch<4>(g, s); break;
            default: narrow_launch<8>(g, s); break;
        }
        TK_LAUNCHED();
        return hipSuccess;
    }
    if (g.K <= kSkinnyWideMaxK) {
        g.S = 1;
        g.Kc = g.K;
        g.part = nullptr;
        const int NG = (NT + kSkinnyTPW - 1) / kSkinnyTPW;
        const size_t lds = sizeof(double) * kSkinnyWideWaves * kSkinnyTPW * 256;
        const unsigned grid = (unsigned)(((g.M + 15) / 16) * NG);
        if (g.at) {
            lds_limit((const void *)k_skinny_wide<kSkinnyTPW, true>, lds);
            k_skinny_wide<kSkinnyTPW, true><<<grid, 64 * kSkinnyWideWaves, lds, s>>>(g, NG);
        } else {
            lds_limit((const void *)k_skinny_wide<kSkinnyTPW, false>, lds);
            k_skinny_wide<kSkinnyTPW, false><<<grid, 64 * kSkinnyWideWaves, lds, s>>>(g, NG);
        }
        TK_LAUNCHED();
        return hipSuccess;
    }
    skinny_split(g.M, g.K, &g.S, &g.Kc);
    g.part = part;
    if (g.S > 1 && skinny_part_elems(g.M, g.N, g.K) > part_elems) return hipErrorInvalidValue;
    switch (NT) {
        case 1: skinny_launch<1>(g, s); break;
        case 2: skinny_launch<2>(g, s); break;
        case 3: skinny_launch<3>(g, s); break;
        case 4: skinny_launch<4>(g, s); break;
        case 5: skinny_launch<5>(g, s); break;
        case 6: skinny_launch<6>(g, s); break;
        case 7: skinny_launch<7>(g, s); break;
        case 8: skinny_launch<8>(g, s); break;
        default: skinny_launch<9>(g, s); break;
    }
    TK_LAUNCHED();
    if (g.S > 1) {
        const int64_t total = (int64_t)g.M * g.N;
        k_skinny_reduce<<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 2048), 256, 0, s>>>(g, NT * 16);
        TK_LAUNCHED();
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ workspace
struct EigLayout {
    double *W, *Y0, *Y1, *Y2, *S, *V, *Vg, *Rinv, *theta, *res, *norms, *split, *thall;
    double *Yop, *Cop, *thl;  // operator solves: A X, locked-part coefficients, locked Ritz values
    double *lz;               // Lanczos coefficients of the spectrum bound (alphas, betas)
    int *colmap;
    int64_t split_elems;
};
static EigLayout eig_layout(Arena &ar, int n, int b) {
    EigLayout L;
    int64_t nb = (int64_t)n * b;
    L.W = ar.take<double>(nb);
    L.Y0 = ar.take<double>(nb);
    L.Y1 = ar.take<double>(nb);
    L.Y2 = ar.take<double>(nb);
    L.S = ar.take<double>((int64_t)b * b);
    L.V = ar.take<double>((int64_t)b * b);
    L.Vg = ar.take<double>((int64_t)b * b);
    L.Rinv = ar.take<double>((int64_t)b * b);
    L.theta = ar.take<double>(2 * (int64_t)b);  // Ritz values, then the residual norms: one read-back
    L.res = L.theta + b;
    L.norms = ar.take<double>(b);
    L.thall = ar.take<double>(b);
    L.colmap = ar.take<int>(b);
    L.Yop = ar.take<double>(nb);
    L.Cop = ar.take<double>((int64_t)b * b);
    L.thl = ar.take<double>(b);
    L.lz = ar.take<double>(64);
    // split-K partial strips: (strips x K ranges) <= 512 for every product
    // (see skinny_split), each 16 rows by at most b columns rounded up to 16
    L.split_elems = (int64_t)512 * 16 * (ceil_div(b, 16) * 16);
    L.split = ar.take<double>(L.split_elems);
    return L;
}
size_t eig_work_bytes(int n, int b) {
    Arena ar;
    eig_layout(ar, n, b);
    return ar.used + 256;
}

// ------------------------------------------------------------------ host helpers
static hipError_t jacobi(const double *H, int ldh, int b, double *theta, double *Vout, double *Vg, hipStream_t s,
                         int sweeps = 30, double off2 = 1e-26) {
    if (b <= kJacobiVLds) {
        size_t lds = sizeof(double) * 2 * (size_t)b * b;
        lds_limit((const void *)k_jacobi<true>, lds);
        k_jacobi<true><<<1, kJacobiThreads, lds, s>>>(H, ldh, b, sweeps, off2, theta, Vout, Vg);
    } else {
        size_t lds = sizeof(double) * (size_t)b * b;
        lds_limit((const void *)k_jacobi<false>, lds);
        k_jacobi<false><<<1, kJacobiThreads, lds, s>>>(H, ldh, b, sweeps, off2, theta, Vout, Vg);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

// C (ldc, column offset in pointer) = alpha * op(A) B (+ beta E1 + gamma E2)
static hipError_t dgemm(int M, int N, int K, const double *A, int64_t lda, bool at, const double *B, int64_t ldb,
                        double *C, int64_t ldc, double alpha, double beta, const double *E1, double gamma,
                        const double *E2, double *split, int64_t split_elems, hipStream_t s) {
    SkinnyArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.at = at ? 1 : 0;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    g.alpha = alpha;
    g.beta = beta;
    g.gamma = gamma;
    g.E1 = beta != 0.0 ? E1 : nullptr;
    g.E2 = gamma != 0.0 ? E2 : nullptr;
    g.S = 1;
    g.Kc = K;
    g.part = nullptr;
    return skinny(g, split, split_elems, s);
}

// C[i][j] *= d[i] for the Lk x w matrix C.
__global__ void k_rowscale(double *C, int rows, int w, const double *d) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows * w; t += gridDim.x * blockDim.x) C[t] *= d[t / w];
}

// Y = alpha (P - D) + beta E1 + gamma E2 elementwise over n x w (Y, D, E1,
// E2 with row stride ldy, P with stride ldp; D is Y itself or absent).
__global__ void k_comb(double *Y, int64_t ldy, const double *P, int64_t ldp, int64_t n, int w, double alpha,
                       double beta, const double *E1, double gamma, const double *E2, int has_d) {
    const int64_t tot = n * w;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / w;
        const int j = (int)(t - i * w);
        double v = P[i * ldp + j];
        if (has_d) v -= Y[i * ldy + j];
        v *= alpha;
        if (E1) v += beta * E1[i * ldy + j];
        if (E2) v += gamma * E2[i * ldy + j];
        Y[i * ldy + j] = v;
    }
}

// Products with the solve's matrix: Y = alpha A X + beta E1 + gamma E2,
// from the explicit (deflated) M, or from the operator with the locked pairs
// (columns [0, Lk) of XL, Ritz values in thl) taken out:
// A' X = A X - XL diag(thl) XL^T X.
struct MProd {
    const double *M;
    int n;
    const EigOp *op;
    EigLayout *L;
    const double *XL;  // locked columns (row stride b)
    int b;
    hipStream_t s;
    hipError_t operator()(const double *X, int64_t ldx, int w, double *Y, int64_t ldy, double alpha, double beta,
                          const double *E1, double gamma, const double *E2, int Lk) const {
        // M is symmetric bit for bit (the Grams write both triangles from
        // one sum; deflation keeps it), so it can be read as its own
        // transpose: a wave's 16 x 4 operand load then spans 16 consecutive
        // columns of 4 rows (4 cache lines) instead of 16 rows (16 lines),
        // and every product term, and so the result, is the same. Products
        // of at most 8 columns keep the row-major narrow kernel.
        if (!op)
            return dgemm(n, w, n, M, n, w > 8, X, ldx, Y, ldy, alpha, beta, E1, gamma, E2, L->split, L->split_elems,
                         s);
        TK_HIP(op->apply(op->ctx, X, ldx, w, L->Yop, w, s));
        if (Lk > 0) {
            TK_HIP(dgemm(Lk, w, n, XL, b, true, X, ldx, L->Cop, w, 1.0, 0.0, nullptr, 0.0, nullptr, L->split,
                         L->split_elems, s));
            k_rowscale<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div((int64_t)Lk * w, 256), 1024)), 256, 0,
                         s>>>(L->Cop, Lk, w, L->thl);
            TK_LAUNCHED();
            TK_HIP(dgemm(n, w, Lk, XL, b, false, L->Cop, w, Y, ldy, 1.0, 0.0, nullptr, 0.0, nullptr, L->split,
                         L->split_elems, s));
        }
        k_comb<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)n * w, 256), 65536), 256, 0, s>>>(
            Y, ldy, L->Yop, w, n, w, alpha, beta, beta != 0.0 ? E1 : nullptr, gamma, gamma != 0.0 ? E2 : nullptr,
            Lk > 0 ? 1 : 0);
        TK_LAUNCHED();
        return hipSuccess;
    }
};

// Lanczos steps on column 0 of the n x b buffers (scalars on the device):
// w -= alpha v + beta_prev vprev; next v = w / beta (zero for beta = 0).
// Sum over a 1024-thread workgroup in a fixed order (red: 16 doubles).
__device__ inline double block_sum(double x, double *red) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    return t;
}
// One Lanczos step after w = A v, in one workgroup: alpha = v.w;
// w -= alpha v + beta_prev vprev; beta = ||w||; vnext = w / beta (vnext may
// be vprev's buffer: it is written after every read of vprev).
__global__ void __launch_bounds__(1024) k_lz_step(double *w, const double *v, const double *vprev, double *vnext,
                                                  int64_t n, int ld, double *alpha_out, const double *beta_prev,
                                                  double *beta_out) {
    __shared__ double red[16];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a += v[i * ld] * w[i * ld];
    a = block_sum(a, red);
    const double bp = beta_prev ? *beta_prev : 0.0;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = w[i * ld] - (a * v[i * ld] + (beta_prev ? bp * vprev[i * ld] : 0.0));
        w[i * ld] = x;
        q += x * x;
    }
    const double bt = sqrt(block_sum(q, red));
    const double inv = bt > 0.0 ? 1.0 / bt : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) vnext[i * ld] = w[i * ld] * inv;
    if (threadIdx.x == 0) {
        *alpha_out = a;
        *beta_out = bt;
    }
}
__global__ void k_lz_next(const double *w, double *v, int64_t n, int ld, const double *beta) {
    const double bt = *beta, inv = bt > 0.0 ? 1.0 / bt : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i * ld] = w[i * ld] * inv;
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..k)
// and off-diagonal e[0..k-1), by bisection on the Sturm count (the number of
// eigenvalues below x is the number of negative pivots of T - x I).
static double tridiag_max(const double *a, const double *e, int k) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = a[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), std::fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == k)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

// Upper estimate of the largest eigenvalue: k Lanczos steps from column 0 of
// x0 (row stride b), the largest eigenvalue of the tridiagonal plus the last
// residual norm (the bound Chebyshev-filtered subspace iteration uses for the
// top of the spectrum: Zhou and Saad, J. Comput. Phys. 2007). Uses column 0
// of Y0, Y1 and Y2.
static hipError_t lanczos_bound(const MProd &mp, int64_t n, int b, const double *x0, int k, EigLayout &L,
                                double *bound, int *products, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 256), 4096);
    double *vprev = L.Y0, *v = L.Y1, *w = L.Y2;
    double *al = L.lz, *be = L.lz + 32;
    k_colnorm<<<1, 256, 0, s>>>(x0, n, b, 0, be + 31);
    TK_LAUNCHED();
    k_lz_next<<<g, 256, 0, s>>>(x0, v, n, b, be + 31);
    TK_LAUNCHED();
    for (int j = 0; j < k; ++j) {
        TK_HIP(mp(v, b, 1, w, b, 1.0, 0.0, nullptr, 0.0, nullptr, 0));
        k_lz_step<<<1, 1024, 0, s>>>(w, v, vprev, vprev, n, b, al + j, j > 0 ? be + j - 1 : nullptr, be + j);
        TK_LAUNCHED();
        std::swap(vprev, v);  // v: the new vector; vprev: the old v
    }
    double hb[64];
    double *h = pinned_scratch() ? pinned_scratch() + 512 : hb;
    TK_HIP(hipMemcpyAsync(h, L.lz, sizeof(double) * 64, hipMemcpyDeviceToHost, s));
    TK_HIP(wait_stream(s));
    *bound = tridiag_max(h, h + 32, k) + std::fabs(h[32 + k - 1]);
    *products += k;
    return hipSuccess;
}

// Orthonormalise columns [c0, c0+w) of X (n x b, row-major) in place:
// column scaling, one shifted CholeskyQR pass, one plain pass.
static hipError_t project_out(const double *X, int64_t n, int b, int c0, double *Xa, int lda, int w, EigLayout &L,
                              hipStream_t s) {
    // Xa -= X[:, :c0] (X[:, :c0]^T Xa), Xa the n x w active columns (leading dimension lda)
    TK_HIP(dgemm(c0, w, (int)n, X, b, true, Xa, lda, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                 L.split_elems, s));
    TK_HIP(dgemm((int)n, w, c0, X, b, false, L.S, w, Xa, lda, -1.0, 1.0, Xa, 0.0, nullptr, L.split, L.split_elems,
                 s));
    return hipSuccess;
}

// Orthonormalise columns [c0, c0+w) of X (n x b, row-major) against the
// columns [0, c0), which are orthonormal already, and among themselves,
// taking them from src (same layout; src may be X): column scaling into X
// (collapsed columns replaced by pseudo-random ones), then two passes of
// (projection against [0, c0), CholeskyQR), the first shifted. The first
// pass writes its result to the scratch Y0 and the second back to X, so no
// copy is needed.
hipError_t chol_inv_upper(const double *S, int w, double shift, double *Rinv, hipStream_t s) {
    if (w <= kCholBlkMax) {
        const int W = (w + 15) & ~15;
        const size_t lds = sizeof(double) * (2 * (size_t)W * W + (kCholBlkThreads / 64) * 256);
        lds_limit((const void *)k_chol_inv_blk, lds);
        k_chol_inv_blk<<<1, kCholBlkThreads, lds, s>>>(S, w, w, shift, Rinv);
    } else {
        const size_t lds = sizeof(double) * ((size_t)w * w + w);
        lds_limit((const void *)k_chol_inv, lds);
        k_chol_inv<<<1, 1024, lds, s>>>(S, w, w, shift, Rinv);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

static hipError_t orthonormalise(const double *src, double *X, int64_t n, int b, int c0, int w, EigLayout &L,
                                 uint64_t seed, hipStream_t s) {
    if (w <= 0) return hipSuccess;
    k_colnorm<<<w, 256, 0, s>>>(src, n, b, c0, L.norms);
    TK_LAUNCHED();
    k_colscale<<<(unsigned)std::min<int64_t>(ceil_div(n * w, 256), 65536), 256, 0, s>>>(src, X, n, b, c0, w,
                                                                                          L.norms, seed);
    TK_LAUNCHED();
    const double u = 1.1102230246251565e-16;
    for (int pass = 0; pass < 2; ++pass) {
        // pass 0: X[:, c0:] -> Y0 (leading dimension w); pass 1: Y0 -> X[:, c0:]
        double *in = pass == 0 ? X + c0 : L.Y0;
        const int ldi = pass == 0 ? b : w;
        double *out = pass == 0 ? L.Y0 : X + c0;
        const int ldo = pass == 0 ? w : b;
        if (c0 > 0) TK_HIP(project_out(X, n, b, c0, in, ldi, w, L, s));
        double shift = pass == 0 ? 11.0 * ((double)n * w + (double)w * (w + 1)) * u / w : 0.0;
        TK_HIP(dgemm(w, w, (int)n, in, ldi, true, in, ldi, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                     L.split_elems, s));
        TK_HIP(chol_inv_upper(L.S, w, shift, L.Rinv, s));
        TK_HIP(dgemm((int)n, w, w, in, ldi, false, L.Rinv, w, out, ldo, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                     L.split_elems, s));
    }
    return hipSuccess;
}

// Column 0 of X <- normalised M^steps x0 (products alternate between X and
// Y0, ending in X), then theta[0] = x^T M x, the Rayleigh quotient that the
// deflation and the output use.
static hipError_t power_lock(const MProd &mp, int n, int b, double *X, int steps, double theta_est, EigLayout &L,
                             hipStream_t s) {
    // each product is scaled by 1 / (the current estimate of the leading
    // eigenvalue), which keeps the vector's norm near one; it is normalised
    // every eighth step and after the last
    const double inv = theta_est > 0.0 ? 1.0 / theta_est : 1.0;
    double *src = X, *dst = L.Y0;
    if (steps & 1) {  // an odd count ends in Y0: start from a copy there
        TK_HIP(hipMemcpy2DAsync(L.Y0, sizeof(double) * b, X, sizeof(double) * b, sizeof(double), n,
                                hipMemcpyDeviceToDevice, s));
        src = L.Y0;
        dst = X;
    }
    for (int k = 0; k < steps; ++k) {
        TK_HIP(mp(src, b, 1, dst, b, inv, 0.0, nullptr, 0.0, nullptr, 0));
        if ((k & 7) == 7 || k == steps - 1) {
            k_colnorm<<<1, 256, 0, s>>>(dst, n, b, 0, L.norms);
            TK_LAUNCHED();
            k_colscale<<<(unsigned)std::min<int64_t>(ceil_div(n, 256), 65536), 256, 0, s>>>(dst, dst, n, b, 0, 1,
                                                                                             L.norms, 0x9e3779b9ull + k);
            TK_LAUNCHED();
        }
        std::swap(src, dst);
    }
    // src == X now; theta = x^T (M x)
    TK_HIP(mp(X, b, 1, L.Y1, b, 1.0, 0.0, nullptr, 0.0, nullptr, 0));
    TK_HIP(dgemm(1, 1, n, X, b, true, L.Y1, b, L.theta, 1, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems,
                 s));
    return hipSuccess;
}

// ------------------------------------------------------------------ shared with the learned start
hipError_t skinny_gemm(int M, int N, int K, const double *A, int64_t lda, bool at, const double *B, int64_t ldb,
                       double *C, int64_t ldc, double alpha, double beta, const double *E1, double *part,
                       int64_t part_elems, hipStream_t s) {
    return dgemm(M, N, K, A, lda, at, B, ldb, C, ldc, alpha, beta, E1, 0.0, nullptr, part, part_elems, s);
}
int64_t skinny_part_bound(int max_n) { return (int64_t)512 * 16 * (ceil_div(max_n, 16) * 16); }



hipError_t canonical_cols(const double *X, int64_t n, int ldx, int J, double *F, hipStream_t s) {
    k_extract<<<J, 256, 0, s>>>(X, n, ldx, J, F, nullptr);
    TK_LAUNCHED();
    return hipSuccess;
}

hipError_t eig_seed_block(double *X, int n, int J, const double *U, void *work, uint64_t seed, hipStream_t s) {
    const int b = eig_block_width(n, J);
    Arena ar;
    ar.base = reinterpret_cast<char *>(work);
    EigLayout L = eig_layout(ar, n, b);
    TK_HIP(hipMemcpy2DAsync(X, sizeof(double) * b, U, sizeof(double) * J, sizeof(double) * J, n,
                            hipMemcpyDeviceToDevice, s));
    if (b > J) {
        k_random_cols<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)n * (b - J), 256), 65536), 256, 0, s>>>(
            X, n, b, J, b, seed);
        TK_LAUNCHED();
        TK_HIP(orthonormalise(X, X, n, b, J, b - J, L, seed + 1, s));
    }
    return hipSuccess;
}

hipError_t lead_eig(double *M, int n, int J, double *X, double *F, double *theta_dev, void *work,
                    const EigOpts &o, int *iters, int *noconv, hipStream_t s) {
    *iters = 0;
    *noconv = 0;
    const int b = eig_block_width(n, J);
    Arena ar;
    ar.base = reinterpret_cast<char *>(work);
    EigLayout L = eig_layout(ar, n, b);
    if (o.op && n <= kDirectMax) return hipErrorInvalidValue;  // small solves need M explicitly
    if (n <= kDirectMax) {
        TK_HIP(jacobi(M, n, n, L.theta, L.V, L.Vg, s, o.direct_sweeps));
        k_extract<<<J, 256, 0, s>>>(L.V, n, n, J, F, nullptr);
        TK_LAUNCHED();
        TK_HIP(hipMemcpyAsync(theta_dev, L.theta, sizeof(double) * J, hipMemcpyDeviceToDevice, s));
        *iters = 1;
        return hipSuccess;
    }
    const int64_t nb = (int64_t)n * b;
    if (!o.warm) {
        k_random_cols<<<(unsigned)std::min<int64_t>(ceil_div(nb, 256), 65536), 256, 0, s>>>(X, n, b, 0, b, o.seed);
        TK_LAUNCHED();
        TK_HIP(orthonormalise(X, X, n, b, 0, b, L, o.seed + 1, s));
    }
    // Locked (converged leading) Ritz pairs occupy X[:, :Lk]; they are
    // deflated out of M, so the filter and the Rayleigh-Ritz steps only see
    // the active columns X[:, Lk:b].
    std::vector<double> h(2 * (size_t)b), thL;
    double Eold = -1.0;
    int matvecs = 0, Lk = 0;
    int deg_cap = o.warm ? std::max(1, std::min(o.warm_degree, o.degree)) : o.degree;
    bool full_step = false;  // the last filter had the full degree
    double *Xc = X;
    double *Md = M;  // deflated in place (an operator solve deflates in its products instead)
    const MProd mprod{Md, n, o.op, &L, X, b, s};
    // An upper bound of the spectrum for the degree of the first filters of a
    // cold start: the Ritz values of a random block can sit far below the top
    // of a flat spectrum, and a degree set by them alone would amplify the
    // top directions beyond what the block's orthonormalisation resolves.
    double bup = 0.0;
    if (!o.warm) TK_HIP(lanczos_bound(mprod, n, b, X, std::min(8, n), L, &bup, &matvecs, s));
    std::vector<double> tha;
    // Intermediate Rayleigh-Ritz steps use one Jacobi sweep: an approximate
    // rotation is enough to pick the leading directions of the block (it is
    // inexact only among nearly tied Ritz pairs, and locking still requires
    // a true residual below its threshold); the step after the energy test
    // has passed diagonalises fully and provides the output.
    // The full diagonalisation only needs the J - Lk leading active columns:
    // the stop rule has judged exactly those (their residuals), and the
    // extra columns of the block serve the filter alone.
    bool final_rr = false;
    // The closing step rotates only inside the wanted columns: the span it
    // returns, and the fit that depends on it alone, are fixed before it, and
    // the trace of its Ritz values is exact at any rotation. Each Ritz value
    // moves by about the square of the remaining off-diagonal over its gap, so
    // an off-diagonal norm of 1e-4 tol relative to the whole (squared: off2)
    // suffices; FP64 solves keep the rounding-level limit.
    const double jt = 1e-4 * o.tol, final_off2 = std::max(1e-26, jt * jt);
    for (int outer = 0;; ++outer) {
        if (final_rr && J == Lk) break;  // every wanted pair is locked
        const int w = final_rr ? J - Lk : b - Lk;
        double *Xa = Xc + Lk, *Wa = L.W + Lk;
        // Rayleigh-Ritz on the active columns
        TK_HIP(mprod(Xa, b, w, Wa, b, 1.0, 0.0, nullptr, 0.0, nullptr, Lk));
        ++matvecs;
        TK_HIP(dgemm(w, w, n, Xa, b, true, Wa, b, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems, s));
        TK_HIP(jacobi(L.S, w, w, L.theta, L.V, L.Vg, s, final_rr ? 30 : 1, final_off2));
        TK_HIP(dgemm(n, w, w, Xa, b, false, L.V, w, L.Y0, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems,
                     s));
        TK_HIP(dgemm(n, w, w, Wa, b, false, L.V, w, L.Y1, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems,
                     s));
        // the Ritz vectors replace the block; M times them (Y1) serves only the
        // residuals, which read it in place
        TK_HIP(hipMemcpy2DAsync(Xa, sizeof(double) * b, L.Y0, sizeof(double) * w, sizeof(double) * w, n,
                                hipMemcpyDeviceToDevice, s));
        k_resid<<<w, 256, 0, s>>>(L.Y1, L.Y0, L.theta, n, w, L.res);
        TK_LAUNCHED();
        if (double *pin = pinned_scratch()) {
            TK_HIP(hipMemcpyAsync(pin, L.theta, sizeof(double) * 2 * b, hipMemcpyDeviceToHost, s));
            TK_HIP(wait_stream(s));
            std::copy(pin, pin + 2 * b, h.begin());
        } else {
            TK_HIP(hipMemcpyAsync(h.data(), L.theta, sizeof(double) * 2 * b, hipMemcpyDeviceToHost, s));
            TK_HIP(hipStreamSynchronize(s));
        }
        tha.assign(h.data(), h.data() + w);
        const double *res = h.data() + b;
        double E = 0;
        for (double v : thL) E += v;
        for (int j = 0; j < J - Lk; ++j) E += tha[j];
        const double thmax = std::max(thL.empty() ? 0.0 : thL[0], tha[0]);
        // residual estimate of the error of E: each wanted Ritz value is off
        // by about its squared residual over its distance to the unwanted
        // spectrum, whose top is estimated by the first unwanted Ritz value
        // (not the block's last one, which can sit far lower and understate
        // the error tenfold on clustered spectra)
        double errE = 0.0;
        bool est_ok = w > J - Lk;
        for (int j = 0; est_ok && j < J - Lk; ++j) {
            const double gap = tha[j] - tha[J - Lk];
            if (!(gap > 1e-12 * thmax)) est_ok = false;
            else errE += res[j] * res[j] / gap;
        }
        bool conv = (est_ok && errE <= o.tol * std::fabs(E)) ||
                    (full_step && Eold >= 0 && std::fabs(E - Eold) <= o.tol * std::fabs(E)) || !(thmax > 0.0);
        // newly converged leading pairs
        int newl = 0;
        const double lock_tol = 1e-11 * std::max(thmax, 1e-300);
        while (Lk + newl < J && res[newl] <= lock_tol) ++newl;
        if (Lk + newl == J) conv = true;
        if (final_rr) break;
        if (conv || matvecs >= o.max_iters) {
            if (!conv) *noconv = 1;
            final_rr = true;  // one more Rayleigh-Ritz, diagonalised fully
            continue;
        }
        Eold = E;
        // A leading Ritz value far above the next one (the mean term of
        // nonnegative data is one) caps the filter degree through the
        // amplification limit below until it is locked. Lock it first with
        // single-vector power steps, whose error shrinks by theta_2/theta_1
        // per product, as many as its residual needs to reach lock_tol.
        // (Warm starts only: from a random block the first Ritz pair is too
        // rough for the step count.)
        if (o.warm && Lk == 0 && newl == 0 && J > 1 && w > 2 && tha[1] > 0.0 && tha[0] > 4.0 * tha[1] &&
            res[0] > lock_tol) {
            const double rate = tha[1] / tha[0];
            const int steps = std::min(60, 2 + (int)std::ceil(std::log(lock_tol / res[0]) / std::log(rate)));
            TK_HIP(power_lock(mprod, n, b, Xc, steps, tha[0], L, s));
            double th1 = 0.0, *pin = pinned_scratch();
            TK_HIP(hipMemcpyAsync(pin ? pin + 600 : &th1, L.theta, sizeof(double), hipMemcpyDeviceToHost, s));
            TK_HIP(wait_stream(s));
            if (pin) th1 = pin[600];
            matvecs += steps + 1;
            tha[0] = th1;
            newl = 1;
        }
        if (newl > 0) {
            if (o.op) {
                TK_HIP(hipMemcpyAsync(L.thl + Lk, L.theta, sizeof(double) * newl, hipMemcpyDeviceToDevice, s));
            } else {
                k_deflate<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)n * n, 256), 65536), 256, 0, s>>>(
                    Md, n, Xc, b, Lk, newl, L.theta);
                TK_LAUNCHED();
            }
            for (int j = 0; j < newl; ++j) thL.push_back(tha[j]);
            Lk += newl;
        }
        // Chebyshev filter on the active columns with the deflated matrix:
        // damp [0, mu] (mu = smallest active Ritz value), scale by the top
        const int wa = b - Lk;
        double *Xf = Xc + Lk;
        double mu = tha[w - 1], top = tha[newl];
        if (!(mu > 0.0) || !(top > mu * (1.0 + 1e-12))) mu = 0.0;  // no interval: power step
        double *Ya = L.Y0 + Lk, *Yb = L.Y1 + Lk, *Yc = L.Y2 + Lk;
        double *cur = Ya;
        if (mu <= 0.0) {
            TK_HIP(mprod(Xf, b, wa, Ya, b, 1.0 / std::max(top, 1e-300), 0.0, nullptr, 0.0, nullptr, Lk));
            ++matvecs;
            full_step = true;
        } else {
            const double c = 0.5 * mu, e = 0.5 * mu, t = (top - c) / e;
            // The filter scales the block's top by T_d(t) relative to its
            // bottom; rounding-level parts along a not yet locked outlier grow
            // by the same factor. Keeping T_d(t) <= 1e8 keeps the filtered
            // block well within what shifted CholeskyQR orthonormalises.
            // (before any pair is locked the degree also respects the
            // spectrum bound, which the top active Ritz value may understate)
            const double tb = Lk == 0 && bup > top ? (bup - c) / e : t;
            const int dmax = (int)std::floor(std::acosh(1e8) / std::acosh(std::max(tb, 1.0 + 1e-12)));
            const int degree = std::max(1, std::min(deg_cap, dmax));
            full_step = deg_cap >= o.degree || degree == dmax;
            double sig = 1.0 / t;
            TK_HIP(mprod(Xf, b, wa, Ya, b, sig / e, -c * sig / e, Xf, 0.0, nullptr, Lk));
            ++matvecs;
            const double *prev = Xf;
            double *bufs[3] = {Ya, Yb, Yc};
            int ci = 0;
            for (int k = 1; k < degree; ++k) {
                const double sig2 = 1.0 / (2.0 * t - sig);
                const double al = 2.0 * sig2 / e;
                int ni = (ci + 1) % 3;
                if (bufs[ni] == prev) ni = (ni + 1) % 3;
                double *nxt = bufs[ni];
                TK_HIP(mprod(cur, b, wa, nxt, b, al, -c * al, cur, -sig * sig2, prev, Lk));
                ++matvecs;
                prev = cur;
                cur = nxt;
                ci = ni;
                sig = sig2;
            }
        }
        deg_cap = std::min(o.degree, 2 * deg_cap);
        // orthonormalise against the locked vectors and among themselves,
        // reading the filtered columns where the filter left them
        TK_HIP(orthonormalise(cur - Lk, Xc, n, b, Lk, wa, L, o.seed + 17 * (outer + 2), s));
    }
    *iters = matvecs;
    // the J leading pairs: locked ones, then the leading active ones; order
    // them by value (locking order is almost always already descending)
    std::vector<double> all(thL);
    for (int j = 0; (int)all.size() < J; ++j) all.push_back(tha[j]);
    std::vector<int> perm(J);
    for (int j = 0; j < J; ++j) perm[j] = j;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return all[a] > all[c]; });
    // uploaded from the thread's pinned buffer (its region is written again
    // only after this thread's next solve has waited on its stream), so no
    // wait here; from pageable vectors with a wait when there is none
    double *pin = pinned_scratch();
    double *sorted = pin ? pin + 640 : all.data();
    int *pm = pin ? reinterpret_cast<int *>(pin + 640 + kMaxBlock) : perm.data();
    std::vector<double> sv(J);
    for (int j = 0; j < J; ++j) sv[j] = all[perm[j]];
    for (int j = 0; j < J; ++j) {
        sorted[j] = sv[j];
        pm[j] = perm[j];
    }
    TK_HIP(hipMemcpyAsync(L.colmap, pm, sizeof(int) * J, hipMemcpyHostToDevice, s));
    TK_HIP(hipMemcpyAsync(theta_dev, sorted, sizeof(double) * J, hipMemcpyHostToDevice, s));
    k_extract<<<J, 256, 0, s>>>(Xc, n, b, J, F, L.colmap);
    TK_LAUNCHED();
    if (!pin) TK_HIP(hipStreamSynchronize(s));  // host vectors above go out of scope
    return hipSuccess;
}

}  // namespace tk
