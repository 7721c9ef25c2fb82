// V-cycle kernels for the smoothed prolongator (arXiv 2210.16660, Sec. 3.1:
// P = (I - omega D^-1 A) P^): with P no longer piecewise constant, the
// restriction and the prolongation are sparse products with P^T and P
// (hierarchical CSR), one thread per row with the row's entries loaded in
// batches of kSaBatch; the passes over A (residuals of the l1-Jacobi pre-
// and post-smoothing) run through the row-tile SpMV.
#pragma once

#include "kernels.hpp"

namespace pamg {

constexpr int kSaBatch = 8;

// s = sum_k val[k] * x[col[k]] over [k0, k1), in order; batched loads.
template <typename T, typename XT>
__device__ __forceinline__ T sa_row_dot(int k0, int k1, const int* __restrict__ col, const T* __restrict__ val,
                                        const XT* __restrict__ x) {
    T s = 0;
    for (int kb = k0; kb < k1; kb += kSaBatch) {
        int c[kSaBatch];
        T a[kSaBatch], xv[kSaBatch];
#pragma unroll
        for (int u = 0; u < kSaBatch; ++u) {
            const int k = min(kb + u, k1 - 1);
            c[u] = col[k];
            a[u] = val[k];
        }
#pragma unroll
        for (int u = 0; u < kSaBatch; ++u) xv[u] = (T)x[c[u]];
#pragma unroll
        for (int u = 0; u < kSaBatch; ++u)
            if (kb + u < k1) s += a[u] * xv[u];
    }
    return s;
}

// Restriction rc = P^T t (rows of P^T: coarse unknowns).
template <typename T>
static __global__ __launch_bounds__(kBlock) void k_sa_restrict(int nc, const int* __restrict__ trp,
                                                        const int* __restrict__ tci, const T* __restrict__ tv,
                                                        const T* __restrict__ t, T* __restrict__ rc,
                                                        const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int I = blockIdx.x * kBlock + threadIdx.x; I < nc; I += stride)
        rc[I] = sa_row_dot<T, T>(trp[I], trp[I + 1], tci, tv, t);
}

// Prolongation onto the pre-smoothed iterate: zp = D^-1 r + P e.
template <typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void k_sa_prolong(int n, const int* __restrict__ prp,
                                                       const int* __restrict__ pci, const T* __restrict__ pv,
                                                       const T* __restrict__ e, const RT* __restrict__ r,
                                                       const T* __restrict__ dinv, T* __restrict__ zp,
                                                       const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        zp[i] = dinv[i] * (T)r[i] + sa_row_dot<T, T>(prp[i], prp[i + 1], pci, pv, e);
}

// Post-smoothing update from the residual t = r - A zp: z = zp + D^-1 t
// (in place when z aliases t).
template <typename T>
static __global__ __launch_bounds__(kBlock) void k_sa_update(int n, const T* __restrict__ zp, const T* __restrict__ dinv,
                                                      const T* t, T* z, const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) z[i] = zp[i] + dinv[i] * t[i];
}

}  // namespace pamg
