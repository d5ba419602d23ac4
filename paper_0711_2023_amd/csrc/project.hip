// Fibre projection: the n-mode product T = X x_m F^T of a sparse tensor with
// a factor matrix (Section 3, n-mode product equation), evaluated on one of
// the fibre orderings. It is the projection that Multislice Projection
// applies to every slice (Figure 7: the products X_::k B, X_:j: C, ...) and
// the first stage of the HOOI tensor-times-matrix chain (Figure 3: U, V, W).
//
// Output layout: T[slot][r] with slot = i_hi * I_lo + i_lo (the two other
// modes) and r < J contiguous; every element is written once, empty fibres
// as zeros. The kernel is bound by HBM writes of T: each thread produces one
// output element; lanes that share a slot read the same slot pointer and
// nonzeros (broadcast) and consecutive factor entries (coalesced), and the
// factor matrix itself stays in L2.
#include "common.h"

namespace tk {

template <class TA>
struct AccOf { typedef float type; };
template <>
struct AccOf<double> { typedef double type; };

template <class TO, class TA>
__device__ inline TO to_out(TA v) { return (TO)v; }

template <class TV, class TF, class TO, int EPT>
__global__ void __launch_bounds__(256) k_project(const int32_t *__restrict__ ptr, const int32_t *__restrict__ lidx,
                                                 const TV *__restrict__ lval, const TF *__restrict__ F, int32_t J,
                                                 int64_t total, double rJ, TO *__restrict__ T) {
    typedef typename AccOf<TV>::type Acc;
    const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int64_t e = e0 + (int64_t)u * stride;
        if (e >= total) return;
        int64_t s = (int64_t)((double)e * rJ);
        if (s * J > e) --s;
        if ((s + 1) * J <= e) ++s;
        const int32_t r = (int32_t)(e - s * J);
        const int32_t p0 = ptr[s], p1 = ptr[s + 1];
        Acc acc = 0;
        for (int32_t p = p0; p < p1; ++p) acc += (Acc)lval[p] * (Acc)F[(int64_t)lidx[p] * J + r];
        T[e] = to_out<TO, Acc>(acc);
    }
}

template <class TV, class TF, class TO>
hipError_t project(const int32_t *ptr, const int32_t *lidx, const TV *lval, const TF *F, int J, int64_t nslots, TO *T,
                   hipStream_t s) {
    const int64_t total = nslots * (int64_t)J;
    if (total <= 0) return hipSuccess;
    constexpr int EPT = 4;
    int64_t blocks = ceil_div(total, 256 * EPT);
    k_project<TV, TF, TO, EPT><<<(unsigned)blocks, 256, 0, s>>>(ptr, lidx, lval, F, J, total, 1.0 / (double)J, T);
    TK_LAUNCHED();
    return hipSuccess;
}

template hipError_t project<double, double, double>(const int32_t *, const int32_t *, const double *, const double *,
                                                    int, int64_t, double *, hipStream_t);
template hipError_t project<float, float, float>(const int32_t *, const int32_t *, const float *, const float *, int,
                                                 int64_t, float *, hipStream_t);
template hipError_t project<float, float, bf16>(const int32_t *, const int32_t *, const float *, const float *, int,
                                                int64_t, bf16 *, hipStream_t);

}  // namespace tk
