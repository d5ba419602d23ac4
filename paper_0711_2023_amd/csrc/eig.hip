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
//   orthonormalised by shifted CholeskyQR (one shifted pass, two plain).
// It stops when the sum of the J leading Ritz values changes by at most
// tol (relative) between Rayleigh-Ritz steps, or when all J are locked.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tk {

constexpr int kDirectMax = 140;   // Jacobi on M itself up to this size
constexpr int kJacobiVLds = 100;  // H and V both in LDS up to this size
constexpr int kMaxBlock = 140;    // H in LDS up to this size

int eig_block_width(int n, int J) {
    if (n <= kDirectMax) return n;
    int p = std::min(32, std::max(8, J / 2));
    int b = std::min(J + p, kMaxBlock);
    b = std::min(b, n);
    return std::max(b, J);
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
__global__ void k_colscale(double *X, int64_t n, int ld, int c0, int w, const double *norms, uint64_t seed) {
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
            X[i * ld + c0 + jj] /= nv;
        else
            X[i * ld + c0 + jj] = hash_normal(seed, (uint64_t)i * 1000003ull + (uint64_t)(c0 + jj)) / sqrt((double)n);
    }
}

// Upper Cholesky factor of S + shift*trace(S)/w*I (S is w x w with leading
// dimension lds) and its inverse, in one workgroup. Non-positive pivots are
// clamped to a tiny positive value (the caller's block then keeps a
// direction it cannot resolve instead of failing).
__global__ void __launch_bounds__(256) k_chol_inv(const double *S, int lds, int w, double shift, double *Rinv) {
    extern __shared__ double A[];  // w*w
    __shared__ double tr;
    const int tid = threadIdx.x;
    for (int t = tid; t < w * w; t += blockDim.x) {
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
    for (int i = tid; i < w; i += blockDim.x) A[i * w + i] += add;
    __syncthreads();
    const double tiny = 1e-300 + 1e-30 * (tr > 0 ? tr : 1.0);
    for (int k = 0; k < w; ++k) {
        if (tid == 0) {
            double d = A[k * w + k];
            A[k * w + k] = sqrt(d > tiny ? d : tiny);
        }
        __syncthreads();
        const double dk = A[k * w + k];
        for (int j = k + 1 + tid; j < w; j += blockDim.x) A[k * w + j] /= dk;
        __syncthreads();
        const int m = w - k - 1;
        for (int t = tid; t < m * m; t += blockDim.x) {
            int i = k + 1 + t / m, j = k + 1 + t % m;
            if (j >= i) A[i * w + j] -= A[k * w + i] * A[k * w + j];
        }
        __syncthreads();
    }
    // inverse of the upper triangle, one column per thread
    for (int j = tid; j < w; j += blockDim.x) {
        for (int i = w - 1; i >= 0; --i) {
            double v = 0;
            if (i <= j) {
                v = (i == j) ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) v -= A[i * w + k] * Rinv[k * w + j];
                v /= A[i * w + i];
            }
            Rinv[i * w + j] = v;
        }
    }
}

// Parallel cyclic Jacobi on the symmetric b x b matrix Hin (leading
// dimension ldh). Outputs the eigenvalues in descending order (theta) and
// the matching eigenvectors as columns of Vout (b x b row-major).
template <bool V_LDS>
__global__ void __launch_bounds__(1024) k_jacobi(const double *Hin, int ldh, int b, int max_sweeps, double *theta,
                                                 double *Vout, double *Vglob) {
    extern __shared__ double sm[];
    double *H = sm;
    double *V = V_LDS ? sm + (size_t)b * b : Vglob;
    const int m = b + (b & 1), half = m / 2;
    double *cs = (V_LDS ? sm + 2 * (size_t)b * b : sm + (size_t)b * b);
    double *sn = cs + half;
    int *pp = reinterpret_cast<int *>(sn + half);
    int *qq = pp + half;
    __shared__ double red[32];
    __shared__ int done;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int t = tid; t < b * b; t += nth) {
        int i = t / b, j = t - i * b;
        H[t] = 0.5 * (Hin[(int64_t)i * ldh + j] + Hin[(int64_t)j * ldh + i]);
        V[t] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        for (int r = 0; r < m - 1; ++r) {
            for (int k = tid; k < half; k += nth) {
                int a, c;
                if (k == 0) {
                    a = 0;
                    c = 1 + (r % (m - 1));
                } else {
                    a = 1 + ((k + r) % (m - 1));
                    c = 1 + ((m - 1 - k + r) % (m - 1));
                }
                int p = a < c ? a : c, q = a < c ? c : a;
                double cc = 1.0, ss = 0.0;
                if (q < b) {
                    double apq = H[p * b + q], app = H[p * b + p], aqq = H[q * b + q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
                        double tau = (aqq - app) / (2.0 * apq);
                        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        if (fabs(tau) > 1e150) t = 0.5 / tau;
                        cc = 1.0 / sqrt(1.0 + t * t);
                        ss = t * cc;
                    }
                }
                cs[k] = cc;
                sn[k] = ss;
                pp[k] = p;
                qq[k] = q;
            }
            __syncthreads();
            // H <- G^T H G on 2x2 blocks (pair K1 rows, pair K2 columns)
            for (int t = tid; t < half * half; t += nth) {
                int k1 = t / half, k2 = t - k1 * half;
                int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
                if (q1 >= b || q2 >= b) {
                    // a dummy index: only one real row/column pair to rotate
                    // (handled below by the single-sided pass)
                    continue;
                }
                double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
                double a = H[p1 * b + p2], bb = H[p1 * b + q2], c = H[q1 * b + p2], d = H[q1 * b + q2];
                double ya = c1 * a - s1 * c, yb = c1 * bb - s1 * d;
                double yc = s1 * a + c1 * c, yd = s1 * bb + c1 * d;
                double za = c2 * ya - s2 * yb, zb = s2 * ya + c2 * yb;
                double zc = c2 * yc - s2 * yd, zd = s2 * yc + c2 * yd;
                if (k1 == k2 && s1 != 0.0) {
                    za = a - (s1 / c1) * bb;
                    zd = d + (s1 / c1) * bb;
                    zb = 0.0;
                    zc = 0.0;
                }
                H[p1 * b + p2] = za;
                H[p1 * b + q2] = zb;
                H[q1 * b + p2] = zc;
                H[q1 * b + q2] = zd;
            }
            // rows/columns paired with the dummy index are not rotated, but
            // they still meet rotations of the other pairs on one side
            if (m != b) {
                for (int t = tid; t < half; t += nth) {
                    int kd = -1;
                    for (int k = 0; k < half; ++k)
                        if (qq[k] >= b) kd = k;
                    if (kd < 0 || t == kd) continue;
                    int x = pp[kd];  // the idle real index
                    int p = pp[t], q = qq[t];
                    double c = cs[t], s = sn[t];
                    // row x, columns p, q (H G) and column x, rows p, q (G^T H)
                    double hp = H[x * b + p], hq = H[x * b + q];
                    double np = c * hp - s * hq, nq = s * hp + c * hq;
                    H[x * b + p] = np;
                    H[x * b + q] = nq;
                    H[p * b + x] = np;
                    H[q * b + x] = nq;
                }
            }
            // V <- V G
            for (int t = tid; t < b * half; t += nth) {
                int row = t / half, k = t - row * half;
                int p = pp[k], q = qq[k];
                if (q >= b) continue;
                double c = cs[k], s = sn[k];
                double vp = V[row * b + p], vq = V[row * b + q];
                V[row * b + p] = c * vp - s * vq;
                V[row * b + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        // convergence: off-diagonal mass relative to the diagonal
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
            done = (o <= 1e-30 * dd) || (dd == 0.0);
        }
        __syncthreads();
        if (done) break;
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
__global__ void k_extract(const double *X, int64_t n, int ldx, int J, double *F) {
    const int j = blockIdx.x;
    double best = -1;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double a = fabs(X[i * ldx + j]);
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
    const double sgn = X[si[0] * ldx + j] < 0 ? -1.0 : 1.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) F[i * J + j] = sgn * X[i * ldx + j];
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

// ------------------------------------------------------------------ workspace
struct EigLayout {
    double *W, *Y0, *Y1, *Y2, *S, *V, *Vg, *Rinv, *theta, *res, *norms, *split;
    int64_t split_elems;
};
static int splitk_for(int64_t K, int64_t tiles) {
    int64_t want = std::max<int64_t>(1, 256 / std::max<int64_t>(1, tiles));
    int64_t maxs = std::max<int64_t>(1, K / 64);
    return (int)std::min<int64_t>(want, maxs);
}
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
    L.theta = ar.take<double>(b);
    L.res = ar.take<double>(b);
    L.norms = ar.take<double>(b);
    // split-K partial sums: M*X (K = n) and X^T Y (K = n)
    int64_t t_mx = ceil_div(n, 64) * ceil_div(b, 64);
    int64_t s1 = (int64_t)splitk_for(n, t_mx) * nb;
    int64_t s2 = (int64_t)splitk_for(n, ceil_div(b, 64) * ceil_div(b, 64)) * b * b;
    L.split_elems = std::max(s1, s2);
    L.split = ar.take<double>(L.split_elems);
    return L;
}
size_t eig_work_bytes(int n, int b) {
    Arena ar;
    eig_layout(ar, n, b);
    return ar.used + 256;
}

// ------------------------------------------------------------------ host helpers
static hipError_t jacobi(const double *H, int ldh, int b, double *theta, double *Vout, double *Vg, hipStream_t s) {
    const int half = (b + 1) / 2;
    size_t small = sizeof(double) * 2 * half + sizeof(int) * 2 * half;
    if (b <= kJacobiVLds) {
        size_t lds = sizeof(double) * 2 * (size_t)b * b + small;
        hipFuncSetAttribute((const void *)k_jacobi<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_jacobi<true><<<1, 1024, lds, s>>>(H, ldh, b, 30, theta, Vout, Vg);
    } else {
        size_t lds = sizeof(double) * (size_t)b * b + small;
        hipFuncSetAttribute((const void *)k_jacobi<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_jacobi<false><<<1, 1024, lds, s>>>(H, ldh, b, 30, theta, Vout, Vg);
    }
    TK_LAUNCHED();
    return hipSuccess;
}

// C (ldc, column offset in pointer) = alpha * A B (+ beta E1 + gamma E2)
static hipError_t dgemm(int M, int N, int K, const double *A, int64_t lda, bool at, const double *B, int64_t ldb,
                        double *C, int64_t ldc, double alpha, double beta, const double *E1, double gamma,
                        const double *E2, double *split, int64_t split_elems, hipStream_t s) {
    GemmArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.batch = 1;
    g.A = A;
    g.lda = lda;
    g.a_trans = at;
    g.B = B;
    g.ldb = ldb;
    g.sB = 0;
    g.C = C;
    g.ldc = ldc;
    g.sC = 0;
    g.prec = P64;
    g.out_type = P64;
    g.alpha = alpha;
    g.beta = beta;
    g.gamma = gamma;
    g.E1 = E1;
    g.E2 = E2;
    int64_t tiles = ceil_div(M, 64) * ceil_div(N, 64);
    int sk = splitk_for(K, tiles);
    while (sk > 1 && (int64_t)sk * M * N > split_elems) --sk;
    g.splitk = sk;
    g.split_scratch = split;
    return gemm(g, s);
}

// Orthonormalise columns [c0, c0+w) of X (n x b, row-major) in place:
// column scaling, one shifted CholeskyQR pass, two plain passes.
static hipError_t orthonormalise(double *X, int64_t n, int b, int c0, int w, EigLayout &L, uint64_t seed,
                                 hipStream_t s) {
    if (w <= 0) return hipSuccess;
    k_colnorm<<<w, 256, 0, s>>>(X, n, b, c0, L.norms);
    TK_LAUNCHED();
    k_colscale<<<(unsigned)std::min<int64_t>(ceil_div(n * w, 256), 65536), 256, 0, s>>>(X, n, b, c0, w, L.norms,
                                                                                          seed);
    TK_LAUNCHED();
    const double u = 1.1102230246251565e-16;
    for (int pass = 0; pass < 3; ++pass) {
        double shift = pass == 0 ? 11.0 * ((double)n * w + (double)w * (w + 1)) * u / w : 0.0;
        // S = Xa^T Xa
        TK_HIP(dgemm(w, w, (int)n, X + c0, b, true, X + c0, b, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                     L.split_elems, s));
        size_t lds = sizeof(double) * (size_t)w * w;
        hipFuncSetAttribute((const void *)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_chol_inv<<<1, 256, lds, s>>>(L.S, w, w, shift, L.Rinv);
        TK_LAUNCHED();
        // Y0[:, :w] = Xa Rinv, then copy back into X[:, c0:c0+w]
        TK_HIP(dgemm((int)n, w, w, X + c0, b, false, L.Rinv, w, L.Y0, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                     L.split_elems, s));
        TK_HIP(hipMemcpy2DAsync(X + c0, sizeof(double) * b, L.Y0, sizeof(double) * w, sizeof(double) * w, n,
                                hipMemcpyDeviceToDevice, s));
    }
    return hipSuccess;
}

hipError_t lead_eig(const double *M, int n, int J, double *X, double *F, double *theta_dev, void *work,
                    const EigOpts &o, int *iters, int *noconv, hipStream_t s) {
    *iters = 0;
    *noconv = 0;
    const int b = eig_block_width(n, J);
    Arena ar;
    ar.base = reinterpret_cast<char *>(work);
    EigLayout L = eig_layout(ar, n, b);
    if (n <= kDirectMax) {
        TK_HIP(jacobi(M, n, n, L.theta, L.V, L.Vg, s));
        k_extract<<<J, 256, 0, s>>>(L.V, n, n, J, F);
        TK_LAUNCHED();
        TK_HIP(hipMemcpyAsync(theta_dev, L.theta, sizeof(double) * J, hipMemcpyDeviceToDevice, s));
        *iters = 1;
        return hipSuccess;
    }
    const int64_t nb = (int64_t)n * b;
    if (!o.warm) {
        k_random_cols<<<(unsigned)std::min<int64_t>(ceil_div(nb, 256), 65536), 256, 0, s>>>(X, n, b, 0, b, o.seed);
        TK_LAUNCHED();
        TK_HIP(orthonormalise(X, n, b, 0, b, L, o.seed + 1, s));
    }
    std::vector<double> h(2 * (size_t)b);
    double Eold = -1.0;
    int matvecs = 0;
    double *Xc = X;  // current block lives in X throughout
    for (int outer = 0;; ++outer) {
        // Rayleigh-Ritz
        TK_HIP(dgemm(n, b, n, M, n, false, Xc, b, L.W, b, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems, s));
        ++matvecs;
        TK_HIP(dgemm(b, b, n, Xc, b, true, L.W, b, L.S, b, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems, s));
        TK_HIP(jacobi(L.S, b, b, L.theta, L.V, L.Vg, s));
        TK_HIP(dgemm(n, b, b, Xc, b, false, L.V, b, L.Y0, b, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems,
                     s));
        TK_HIP(dgemm(n, b, b, L.W, b, false, L.V, b, L.Y1, b, 1.0, 0.0, nullptr, 0.0, nullptr, L.split, L.split_elems,
                     s));
        TK_HIP(hipMemcpyAsync(Xc, L.Y0, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
        TK_HIP(hipMemcpyAsync(L.W, L.Y1, sizeof(double) * nb, hipMemcpyDeviceToDevice, s));
        k_resid<<<b, 256, 0, s>>>(L.W, Xc, L.theta, n, b, L.res);
        TK_LAUNCHED();
        TK_HIP(hipMemcpyAsync(h.data(), L.theta, sizeof(double) * b, hipMemcpyDeviceToHost, s));
        TK_HIP(hipMemcpyAsync(h.data() + b, L.res, sizeof(double) * b, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        const double *th = h.data(), *res = h.data() + b;
        double E = 0;
        for (int j = 0; j < J; ++j) E += th[j];
        int Lk = 0;
        const double lock_tol = 1e-11 * std::max(th[0], 1e-300);
        while (Lk < J && res[Lk] <= lock_tol) ++Lk;
        bool conv = (Eold >= 0 && std::fabs(E - Eold) <= o.tol * std::fabs(E)) || Lk == J || th[0] <= 0.0;
        if (conv) break;
        if (matvecs >= o.max_iters) {
            *noconv = 1;
            break;
        }
        Eold = E;
        // Chebyshev filter on columns [Lk, b)
        const int w = b - Lk;
        double mu = th[b - 1], top = th[Lk];
        if (!(mu > 0.0) || !(top > mu * (1.0 + 1e-12))) {
            // no usable interval: a plain power step
            mu = 0.0;
        }
        double *Xa = Xc + Lk;
        double *Ya = L.Y0 + Lk, *Yb = L.Y1 + Lk, *Yc = L.Y2 + Lk;
        if (mu <= 0.0) {
            TK_HIP(dgemm(n, w, n, M, n, false, Xa, b, Ya, b, 1.0 / std::max(top, 1e-300), 0.0, nullptr, 0.0, nullptr,
                         L.split, L.split_elems, s));
            ++matvecs;
        } else {
            const double c = 0.5 * mu, e = 0.5 * mu, t = (top - c) / e;
            double sig = 1.0 / t;
            // Y1 = (M X - c X) * sig / e
            TK_HIP(dgemm(n, w, n, M, n, false, Xa, b, Ya, b, sig / e, -c * sig / e, Xa, 0.0, nullptr, L.split,
                         L.split_elems, s));
            ++matvecs;
            const double *prev = Xa;
            double *cur = Ya;
            double *bufs[3] = {Ya, Yb, Yc};
            int ci = 0;
            for (int k = 1; k < o.degree; ++k) {
                const double sig2 = 1.0 / (2.0 * t - sig);
                const double al = 2.0 * sig2 / e;
                int ni = (ci + 1) % 3;
                if (bufs[ni] == prev) ni = (ni + 1) % 3;
                double *nxt = bufs[ni];
                TK_HIP(dgemm(n, w, n, M, n, false, cur, b, nxt, b, al, -c * al, cur, -sig * sig2, prev, L.split,
                             L.split_elems, s));
                ++matvecs;
                prev = cur;
                cur = nxt;
                ci = ni;
                sig = sig2;
            }
            if (cur != Ya) TK_HIP(hipMemcpy2DAsync(Ya, sizeof(double) * b, cur, sizeof(double) * b,
                                                    sizeof(double) * w, n, hipMemcpyDeviceToDevice, s));
        }
        // Ya holds the filtered active columns; re-orthogonalise against locked
        if (Lk > 0) {
            for (int rep = 0; rep < 2; ++rep) {
                TK_HIP(dgemm(Lk, w, n, Xc, b, true, Ya, b, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                             L.split_elems, s));
                TK_HIP(dgemm(n, w, Lk, Xc, b, false, L.S, w, Ya, b, -1.0, 1.0, Ya, 0.0, nullptr, L.split,
                             L.split_elems, s));
            }
        }
        TK_HIP(hipMemcpy2DAsync(Xa, sizeof(double) * b, Ya, sizeof(double) * b, sizeof(double) * w, n,
                                hipMemcpyDeviceToDevice, s));
        TK_HIP(orthonormalise(Xc, n, b, Lk, w, L, o.seed + 17 * (outer + 2), s));
        if (Lk > 0) {
            // the CholeskyQR passes do not see the locked columns: project once more
            TK_HIP(dgemm(Lk, w, n, Xc, b, true, Xa, b, L.S, w, 1.0, 0.0, nullptr, 0.0, nullptr, L.split,
                         L.split_elems, s));
            TK_HIP(dgemm(n, w, Lk, Xc, b, false, L.S, w, Xa, b, -1.0, 1.0, Xa, 0.0, nullptr, L.split, L.split_elems,
                         s));
            TK_HIP(orthonormalise(Xc, n, b, Lk, w, L, o.seed + 31 * (outer + 2), s));
        }
    }
    *iters = matvecs;
    k_extract<<<J, 256, 0, s>>>(Xc, n, b, J, F);
    TK_LAUNCHED();
    TK_HIP(hipMemcpyAsync(theta_dev, L.theta, sizeof(double) * J, hipMemcpyDeviceToDevice, s));
    return hipSuccess;
}

}  // namespace tk
