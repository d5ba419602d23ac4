// Learned warm start: a start for the factors of HOOI and Multislice
// Projection (which the paper starts from HO-SVD, Sections 4.2 and 4.4)
// computed from a Gaussian sketch of each unfolding by a small row-wise
// perceptron.
//
//   sketch     S = X_(n) Omega (I_n x 64, FP32). Omega is never stored: its row
//              for the two other coordinates (i_a, i_b), a = n+1, b = n+2 mod 3,
//              lin = i_a I_b + i_b, comes from SplitMix64 outputs
//              k = (n 2^40 + lin) 64 + 2q + h (h = 0, 1) through the Box-Muller
//              transform: u1 = 1 - unit(k0), u2 = unit(k1), entries 2q, 2q+1 =
//              sqrt(-2 ln u1) (cos, sin)(2 pi u2).
//   features   F_i = S_i / rho_i, rho_i = ||S_i|| (zero rows stay zero).
//   network    R_i = rho_i (W2^T relu(W1^T F_i + b1) + b2), 64 -> 128 -> 128,
//              weights rounded to BF16, FP32 accumulation.
//   start      Rayleigh-Ritz of H_n = X_(n) X_(n)^T on the span of the first
//              K = min(128, 2J) outputs: Q from CholeskyQR of Rk (two passes),
//              then the J leading eigenpairs of Q^T H_n Q (FP64).
//   training   subspace-alignment loss that asks span(Rk) to contain
//              converged factors A* (n x J), L = 1 - tr(B^T C^-1 B) / J,
//              C = Rk^T Rk + lam I, B = Rk^T A*, its gradient (lam held
//              fixed) and the backward pass, in the same precisions; Adam on
//              FP32 master weights.
//
// The sketch reads the ordering whose slots are the mode-n slices, so each
// workgroup owns one row i_n and sums it in a fixed order (no atomics).
#include "common.h"

#include <algorithm>
#include <cmath>

namespace tk {

constexpr int kIn = 64, kHid = 128, kOut = 128;
constexpr int kParams = kIn * kHid + kHid + kHid * kOut + kOut;
constexpr int kMlpRows = 16;    // rows per workgroup in the forward pass
constexpr int kBwdRows = 32;    // rows per workgroup in the backward pass

int learn_param_count() { return kParams; }

__device__ inline uint64_t sm64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ inline double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// One workgroup per row i_n of the mode-n sketch; the slots of the ordering
// (hi = n, lo = n+2) for this row are i_n * I_lo .. (i_n + 1) * I_lo - 1 and
// the leaf coordinate is mode n+1. The 64 columns are formed in four passes
// of 16 (8 Box-Muller pairs), which keeps the accumulators in few registers.
constexpr int kSkPass = 16;

template <class TV>
__global__ void __launch_bounds__(256) k_sketch(const int32_t *__restrict__ ptr, const int32_t *__restrict__ lidx,
                                                const TV *__restrict__ lval, int64_t Ilo, int64_t Ib, int n,
                                                uint64_t seed, float *__restrict__ F, float *__restrict__ rho) {
    const int64_t row = blockIdx.x;
    const uint64_t mode_base = (uint64_t)n << 40;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ float part[4][kSkPass];
    __shared__ float srow[kIn];
    __shared__ float snorm;
    for (int pass = 0; pass < kIn / kSkPass; ++pass) {
        float acc[kSkPass];
#pragma unroll
        for (int c = 0; c < kSkPass; ++c) acc[c] = 0.f;
        for (int64_t sl = threadIdx.x; sl < Ilo; sl += blockDim.x) {
            const int64_t slot = row * Ilo + sl;
            const int32_t q0 = ptr[slot], q1 = ptr[slot + 1];
            for (int32_t q = q0; q < q1; ++q) {
                // a = n+1 is the leaf, b = n+2 is the slot's low coordinate
                const uint64_t lin = (uint64_t)lidx[q] * (uint64_t)Ib + (uint64_t)sl;
                const uint64_t base = (mode_base + lin) * 64 + (uint64_t)pass * kSkPass;
                const float v = (float)lval[q];
#pragma unroll
                for (int p = 0; p < kSkPass / 2; ++p) {
                    const float u1 = (float)(1.0 - unit53(sm64_at(seed, base + 2 * p)));
                    const float u2 = (float)unit53(sm64_at(seed, base + 2 * p + 1));
                    const float r = sqrtf(-2.0f * logf(u1));
                    float sn, cs;
                    sincosf(6.283185307179586f * u2, &sn, &cs);
                    acc[2 * p] += v * r * cs;
                    acc[2 * p + 1] += v * r * sn;
                }
            }
        }
        // fixed-order reduction: waves by shuffles, then the four waves in LDS
#pragma unroll
        for (int c = 0; c < kSkPass; ++c) {
            float x = acc[c];
            for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
            acc[c] = x;
        }
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < kSkPass; ++c) part[wave][c] = acc[c];
        __syncthreads();
        if (threadIdx.x < kSkPass) {
            const int c = threadIdx.x;
            srow[pass * kSkPass + c] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double t = 0;
        for (int c = 0; c < kIn; ++c) t += (double)srow[c] * srow[c];
        snorm = (float)sqrt(t);
        rho[row] = snorm;
    }
    __syncthreads();
    if (threadIdx.x < kIn) F[row * kIn + threadIdx.x] = snorm > 0.f ? srow[threadIdx.x] / snorm : 0.f;
}

__device__ inline float bf16_round(float w) { return (float)(bf16)w; }

// R (rows x 128) and, when Z1 is given, the pre-activations (rows x 128).
__global__ void __launch_bounds__(128) k_mlp_fwd(const float *__restrict__ F, const float *__restrict__ rho,
                                                 int64_t rows, const float *__restrict__ P, float *__restrict__ R,
                                                 float *__restrict__ Z1) {
    const float *W1 = P, *b1 = P + kIn * kHid, *W2 = b1 + kHid, *b2 = W2 + kHid * kOut;
    __shared__ float Fs[kMlpRows][kIn];
    __shared__ float Hs[kMlpRows][kHid];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kMlpRows;
    const int nr = (int)std::min<int64_t>(kMlpRows, rows - r0);
    for (int e = t; e < kMlpRows * kIn; e += 128) {
        const int r = e / kIn, k = e - r * kIn;
        Fs[r][k] = r < nr ? F[(r0 + r) * kIn + k] : 0.f;
    }
    __syncthreads();
    float z[kMlpRows];
#pragma unroll
    for (int r = 0; r < kMlpRows; ++r) z[r] = b1[t];
    for (int k = 0; k < kIn; ++k) {
        const float w = bf16_round(W1[k * kHid + t]);
#pragma unroll
        for (int r = 0; r < kMlpRows; ++r) z[r] += Fs[r][k] * w;
    }
#pragma unroll
    for (int r = 0; r < kMlpRows; ++r) {
        Hs[r][t] = z[r] > 0.f ? z[r] : 0.f;
        if (Z1 && r < nr) Z1[(r0 + r) * kHid + t] = z[r];
    }
    __syncthreads();
    float o[kMlpRows];
#pragma unroll
    for (int r = 0; r < kMlpRows; ++r) o[r] = b2[t];
    for (int h = 0; h < kHid; ++h) {
        const float w = bf16_round(W2[h * kOut + t]);
#pragma unroll
        for (int r = 0; r < kMlpRows; ++r) o[r] += Hs[r][h] * w;
    }
#pragma unroll
    for (int r = 0; r < kMlpRows; ++r)
        if (r < nr) R[(r0 + r) * kOut + t] = rho[r0 + r] * o[r];
}

// Per-tile parameter gradients: part[tile][param] (FP32), summed over tiles in
// a fixed order by k_grad_sum.
__global__ void __launch_bounds__(128) k_mlp_bwd(const float *__restrict__ F, const float *__restrict__ rho,
                                                 int64_t rows, const float *__restrict__ P,
                                                 const float *__restrict__ Z1, const float *__restrict__ dR,
                                                 float *__restrict__ part) {
    const float *W2 = P + kIn * kHid + kHid;
    __shared__ float Fs[kBwdRows][kIn];
    __shared__ float Hs[kBwdRows][kHid];
    __shared__ float G2[kBwdRows][kOut];   // dZ2
    __shared__ float G1[kBwdRows][kHid];   // dZ1
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kBwdRows;
    const int nr = (int)std::min<int64_t>(kBwdRows, rows - r0);
    for (int e = t; e < kBwdRows * kIn; e += 128) {
        const int r = e / kIn, k = e - r * kIn;
        Fs[r][k] = r < nr ? F[(r0 + r) * kIn + k] : 0.f;
    }
    for (int r = 0; r < kBwdRows; ++r) {
        const bool in = r < nr;
        const float z = in ? Z1[(r0 + r) * kHid + t] : 0.f;
        Hs[r][t] = z > 0.f ? z : 0.f;
        G2[r][t] = in ? rho[r0 + r] * dR[(r0 + r) * kOut + t] : 0.f;
        G1[r][t] = z;  // pre-activation for the mask, replaced below
    }
    __syncthreads();
    // dH[r][h = t] = sum_o dZ2[r][o] W2[h][o]; dZ1 = dH * (Z1 > 0)
    float dh[kBwdRows];
#pragma unroll
    for (int r = 0; r < kBwdRows; ++r) dh[r] = 0.f;
    for (int o = 0; o < kOut; ++o) {
        const float w = bf16_round(W2[t * kOut + o]);
#pragma unroll
        for (int r = 0; r < kBwdRows; ++r) dh[r] += G2[r][o] * w;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kBwdRows; ++r) G1[r][t] = G1[r][t] > 0.f ? dh[r] : 0.f;
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * kParams;
    // dW1[k][h = t] and db1[t]
    for (int k = 0; k < kIn; ++k) {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < kBwdRows; ++r) a += Fs[r][k] * G1[r][t];
        out[k * kHid + t] = a;
    }
    {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < kBwdRows; ++r) a += G1[r][t];
        out[kIn * kHid + t] = a;
    }
    // dW2[h][o = t] and db2[t]
    float *gW2 = out + kIn * kHid + kHid;
    for (int h = 0; h < kHid; ++h) {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < kBwdRows; ++r) a += Hs[r][h] * G2[r][t];
        gW2[h * kOut + t] = a;
    }
    {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < kBwdRows; ++r) a += G2[r][t];
        gW2[kHid * kOut + t] = a;
    }
}

__global__ void k_grad_sum(const float *__restrict__ part, int tiles, float *__restrict__ grad) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kParams; p += gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int tl = 0; tl < tiles; ++tl) a += part[(int64_t)tl * kParams + p];
        grad[p] = (float)a;
    }
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Rk (rows x K, FP64) = R[:, :K]
__global__ void k_take_cols(const float *__restrict__ R, int64_t rows, int K, double *__restrict__ Rk) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * K; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / K;
        const int c = (int)(e - i * K);
        Rk[e] = (double)R[i * kOut + c];
    }
}

// dR (rows x 128, FP32) = [scale * G, 0], G rows x K
__global__ void k_put_cols(const double *__restrict__ G, int64_t rows, int K, double scale, float *__restrict__ dR) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * kOut; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kOut;
        const int c = (int)(e - i * kOut);
        dR[e] = c < K ? (float)(scale * G[i * K + c]) : 0.f;
    }
}

// out (c x r) = M^T for M r x c
__global__ void k_transpose(const double *__restrict__ M, int r, int c, double *__restrict__ out) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r * c; e += gridDim.x * blockDim.x) {
        const int i = e / c, j = e - i * c;
        out[j * r + i] = M[e];
    }
}

// loss[0] = 1 - sum(B .* CB) / J over K x J entries (one workgroup)
__global__ void k_align_value(const double *__restrict__ B, const double *__restrict__ CB, int K, int J,
                              double *__restrict__ loss) {
    __shared__ double red[256];
    double a = 0.0;
    for (int e = threadIdx.x; e < K * J; e += blockDim.x) a += B[e] * CB[e];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = 1.0 - red[0] / J;
}

// ------------------------------------------------------------------ host side
template <class TV>
hipError_t learn_sketch(const int32_t *ptr, const int32_t *lidx, const TV *lval, int64_t In, int64_t Ilo, int n,
                        uint64_t seed, float *F, float *rho, hipStream_t s) {
    if (In <= 0) return hipSuccess;
    k_sketch<TV><<<(unsigned)In, 256, 0, s>>>(ptr, lidx, lval, Ilo, Ilo, n, seed, F, rho);
    TK_LAUNCHED();
    return hipSuccess;
}
template hipError_t learn_sketch<float>(const int32_t *, const int32_t *, const float *, int64_t, int64_t, int,
                                        uint64_t, float *, float *, hipStream_t);
template hipError_t learn_sketch<double>(const int32_t *, const int32_t *, const double *, int64_t, int64_t, int,
                                         uint64_t, float *, float *, hipStream_t);

hipError_t learn_forward(const float *F, const float *rho, int64_t rows, const float *P, float *R, float *Z1,
                         hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_mlp_fwd<<<(unsigned)ceil_div(rows, kMlpRows), 128, 0, s>>>(F, rho, rows, P, R, Z1);
    TK_LAUNCHED();
    return hipSuccess;
}

size_t learn_backward_scratch(int64_t rows) { return sizeof(float) * (size_t)ceil_div(std::max<int64_t>(rows, 1), kBwdRows) * kParams; }

hipError_t learn_backward(const float *F, const float *rho, int64_t rows, const float *P, const float *Z1,
                          const float *dR, float *grad, float *part, hipStream_t s) {
    const int tiles = (int)ceil_div(std::max<int64_t>(rows, 1), kBwdRows);
    if (rows > 0) {
        k_mlp_bwd<<<(unsigned)tiles, 128, 0, s>>>(F, rho, rows, P, Z1, dR, part);
        TK_LAUNCHED();
    }
    k_grad_sum<<<(unsigned)ceil_div(kParams, 256), 256, 0, s>>>(part, rows > 0 ? tiles : 0, grad);
    TK_LAUNCHED();
    return hipSuccess;
}

hipError_t learn_adam(float *P, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                      float eps, int step, hipStream_t s) {
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    k_adam<<<(unsigned)std::min<int64_t>(ceil_div(n, 256), 1024), 256, 0, s>>>(P, g, m, v, n, lr, b1, b2, eps, c1,
                                                                              c2);
    TK_LAUNCHED();
    return hipSuccess;
}

// Scratch (doubles) of the alignment loss: Rk (rows x K), E (rows x J), C,
// Ui (K x K), B, T1, CB (K x J), CBt (J x K), and the skinny partial strips.
int64_t learn_align_scratch_doubles(int64_t rows, int K, int J) {
    return 8 + rows * (K + J) + 2 * (int64_t)K * K + 4 * (int64_t)K * J + 8 + skinny_part_bound(std::max(K, J));
}

hipError_t learn_align(const float *R, int64_t rows, int K, const double *A, int J, double shift, double *loss_dev,
                       float *dR, double *scratch, hipStream_t s) {
    double *Rk = scratch, *E = Rk + rows * K, *C = E + rows * J, *Ui = C + K * K, *B = Ui + K * K;
    double *T1 = B + K * J, *CB = T1 + K * J, *CBt = CB + K * J, *part = CBt + K * J + 8;
    const int64_t pe = skinny_part_bound(std::max(K, J));
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(rows * kOut, 256), 4096);
    k_take_cols<<<g, 256, 0, s>>>(R, rows, K, Rk);
    TK_LAUNCHED();
    TK_HIP(skinny_gemm(K, K, (int)rows, Rk, K, true, Rk, K, C, K, 1.0, 0.0, nullptr, part, pe, s));
    TK_HIP(skinny_gemm(K, J, (int)rows, Rk, K, true, A, J, B, J, 1.0, 0.0, nullptr, part, pe, s));
    // C + shift tr(C) I = U^T U; C^-1 B = Ui (Ui^T B)
    TK_HIP(chol_inv_upper(C, K, shift, Ui, s));
    TK_HIP(skinny_gemm(K, J, K, Ui, K, true, B, J, T1, J, 1.0, 0.0, nullptr, part, pe, s));
    TK_HIP(skinny_gemm(K, J, K, Ui, K, false, T1, J, CB, J, 1.0, 0.0, nullptr, part, pe, s));
    k_align_value<<<1, 256, 0, s>>>(B, CB, K, J, loss_dev);
    TK_LAUNCHED();
    if (dR) {
        // E = A - Rk CB (rows x J); dRk = -(2/J) E CB^T (rows x K)
        TK_HIP(skinny_gemm((int)rows, J, K, Rk, K, false, CB, J, E, J, -1.0, 1.0, A, part, pe, s));
        k_transpose<<<(unsigned)ceil_div(K * J, 256), 256, 0, s>>>(CB, K, J, CBt);
        TK_LAUNCHED();
        TK_HIP(skinny_gemm((int)rows, K, J, E, J, false, CBt, K, Rk, K, 1.0, 0.0, nullptr, part, pe, s));
        k_put_cols<<<g, 256, 0, s>>>(Rk, rows, K, -2.0 / J, dR);
        TK_LAUNCHED();
    }
    return hipSuccess;
}

int learn_test_width(int J) { return std::min(kOut, 2 * J); }

// Start factor F (rows x J): Rayleigh-Ritz of H (rows x rows) on the span of
// the first K = learn_test_width(J) network outputs. The basis Q of that span
// comes from two CholeskyQR passes (Rk^T Rk = U^T U, Q = Rk U^-1, then once
// more on Q); gC (K) receives the diagonal of the first Cholesky factor
// squared, whose spread is the rank test, theta (J) the Ritz values.
// Scratch: Q and HQ (rows x K each), C and V (K x K), the eigensolver
// workspace `eigw` (eig_work_bytes(K, K)) and skinny partial strips.
__global__ void k_diag_sq(const double *__restrict__ U, int K, double *__restrict__ d) {
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
        const double u = U[i * K + i];  // inverse factor: diagonal is 1 / r_ii
        d[i] = u != 0.0 ? 1.0 / (u * u) : 0.0;
    }
}

hipError_t learn_start(const float *R, int64_t rows, int J, const double *H, double *F, double *theta, double *gC,
                       double *Q, double *HQ, double *C, double *V, void *eigw, double *part, int64_t part_elems,
                       hipStream_t s) {
    const int K = learn_test_width(J);
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(rows * K, 256), 4096);
    k_take_cols<<<g, 256, 0, s>>>(R, rows, K, HQ);
    TK_LAUNCHED();
    double *src = HQ, *dst = Q;
    for (int pass = 0; pass < 2; ++pass) {
        TK_HIP(skinny_gemm(K, K, (int)rows, src, K, true, src, K, C, K, 1.0, 0.0, nullptr, part, part_elems, s));
        TK_HIP(chol_inv_upper(C, K, pass == 0 ? 1e-14 : 0.0, V, s));
        if (pass == 0) {
            k_diag_sq<<<1, 128, 0, s>>>(V, K, gC);
            TK_LAUNCHED();
        }
        TK_HIP(skinny_gemm((int)rows, K, K, src, K, false, V, K, dst, K, 1.0, 0.0, nullptr, part, part_elems, s));
        std::swap(src, dst);
    }
    // src == HQ holds Q now: move it to Q, then H Q, Q^T H Q and its leading pairs
    TK_HIP(hipMemcpyAsync(Q, HQ, sizeof(double) * rows * K, hipMemcpyDeviceToDevice, s));
    TK_HIP(skinny_gemm((int)rows, K, (int)rows, H, rows, false, Q, K, HQ, K, 1.0, 0.0, nullptr, part, part_elems, s));
    TK_HIP(skinny_gemm(K, K, (int)rows, Q, K, true, HQ, K, C, K, 1.0, 0.0, nullptr, part, part_elems, s));
    EigOpts eo;
    // a start needs the leading subspace only roughly (the first sweep's
    // eigensolve refines it): three Jacobi sweeps of the K x K problem
    eo.direct_sweeps = 3;
    int it = 0, nc = 0;
    // K <= 128 is within the direct (Jacobi) size
    TK_HIP(lead_eig(C, K, J, V, V, theta, eigw, eo, &it, &nc, s));
    TK_HIP(skinny_gemm((int)rows, J, K, Q, K, false, V, J, HQ, J, 1.0, 0.0, nullptr, part, part_elems, s));
    TK_HIP(canonical_cols(HQ, rows, J, J, F, s));
    return hipSuccess;
}

}  // namespace tk
