// V-cycle kernels for the smoothed prolongator (arXiv 2210.16660, Sec. 3.1:
// P = (I - omega D^-1 A) P^): with P no longer piecewise constant, the
// restriction and the prolongation are sparse products with P^T and P
// (hierarchical CSR), next to the l1-Jacobi pre- and post-smoothing.  One
// thread per row, the row's entries loaded in batches of kSaBatch.
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

// Pre-smoothing from zero and the residual: t = r - A D^-1 r (vd = a_ij / d_j).
template <typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void k_sa_resid(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const T* __restrict__ vd,
                                                     const RT* __restrict__ r, T* __restrict__ t,
                                                     const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        t[i] = (T)r[i] - sa_row_dot<T, RT>(rp[i], rp[i + 1], ci, vd, r);
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

// Post-smoothing: z = zp + D^-1 (r - A zp).
template <typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void k_sa_post(int n, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const T* __restrict__ av,
                                                    const RT* __restrict__ r, const T* __restrict__ dinv,
                                                    const T* __restrict__ zp, T* __restrict__ z,
                                                    const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        z[i] = zp[i] + dinv[i] * ((T)r[i] - sa_row_dot<T, T>(rp[i], rp[i + 1], ci, av, zp));
}

}  // namespace pamg
