// V-cycle kernels for the smoothed prolongator (arXiv 2210.16660, Sec. 3.1:
// P = (I - omega D^-1 A) P^): with P no longer piecewise constant, the
// restriction and the prolongation are sparse products with P^T and P
// (hierarchical CSR), a group of lanes per row; the passes over A
// (residuals of the l1-Jacobi pre- and post-smoothing) run through the
// row-tile SpMV.
#pragma once

#include "kernels.hpp"

namespace pamg {

// Sum over one CSR row by a group of LPR lanes (entries strided over the
// group, four of a lane's entries loaded at once, each lane accumulating its
// entries in order; then a butterfly in fixed order): every lane gets the sum.
template <int LPR, typename T, typename XT>
__device__ __forceinline__ T sa_group_dot(int k0, int k1, int lane, const int* __restrict__ col,
                                          const T* __restrict__ val, const XT* __restrict__ x) {
    T s = 0;
    int k = k0 + lane;
    for (; k + 3 * LPR < k1; k += 4 * LPR) {
        int c[4];
        T a[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = col[k + u * LPR];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = val[k + u * LPR];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (T)x[c[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += a[u] * v[u];
    }
    for (; k < k1; k += LPR) s += val[k] * (T)x[col[k]];
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
    return s;
}

// Lanes per row for rows of `nnz / rows` entries on average: the smallest of
// 8, 16, 32, 64 that leaves each lane at most about four entries (the rows
// of P^T on the coarse levels run to hundreds of entries).
inline int sa_lanes(long long nnz, long long rows) {
    const long long avg = rows > 0 ? nnz / rows : 0;
    int g = 8;
    while (g < 64 && 4LL * g < avg) g *= 2;
    return g;
}

// Restriction rc = P^T t (rows of P^T: coarse unknowns), a group of G lanes
// per row.
template <int G, typename T>
static __global__ __launch_bounds__(kBlock) void k_sa_restrict(int nc, const int* __restrict__ trp,
                                                        const int* __restrict__ tci, const T* __restrict__ tv,
                                                        const T* __restrict__ t, T* __restrict__ rc,
                                                        const int* __restrict__ done) {
    if (*done) return;
    const int lane = threadIdx.x % G;
    const int stride = gridDim.x * (kBlock / G);
    for (int I = blockIdx.x * (kBlock / G) + threadIdx.x / G; I < nc; I += stride) {
        const T v = sa_group_dot<G, T, T>(trp[I], trp[I + 1], lane, tci, tv, t);
        if (lane == 0) rc[I] = v;
    }
}

// Prolongation onto the pre-smoothed iterate: zp = D^-1 r + P e (a group of
// G lanes per row).
template <int G, typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void k_sa_prolong(int n, const int* __restrict__ prp,
                                                       const int* __restrict__ pci, const T* __restrict__ pv,
                                                       const T* __restrict__ e, const RT* __restrict__ r,
                                                       const T* __restrict__ dinv, T* __restrict__ zp,
                                                       const int* __restrict__ done) {
    if (*done) return;
    const int lane = threadIdx.x % G;
    const int stride = gridDim.x * (kBlock / G);
    for (int i = blockIdx.x * (kBlock / G) + threadIdx.x / G; i < n; i += stride) {
        const T v = sa_group_dot<G, T, T>(prp[i], prp[i + 1], lane, pci, pv, e);
        if (lane == 0) zp[i] = dinv[i] * (T)r[i] + v;
    }
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
