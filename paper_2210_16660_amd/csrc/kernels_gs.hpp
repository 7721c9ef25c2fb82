// Hybrid forward/backward Gauss-Seidel smoother (arXiv 2210.16660, Sec. 3.1)
// and the V-cycle kernels that go with it.
//
// The smoother is x <- x + M^-1 (r - A x) with M = blockdiag(omega (L_pp +
// D_pp)): the level's rows (hierarchical order, which is the nested-aggregate
// order) are cut into blocks of nb <= 256 consecutive rows; within a block
// the correction d solves (L_pp + D_pp) d = (r - A x)_p by substitution
// (forward: earlier rows; backward, M^T: later rows) and x += d / omega.
// Blocks are independent (block Jacobi between them), one workgroup each.
// Inside a block the substitution runs by depth: a row's depth is one more
// than the deepest earlier (later) row of the block it couples to, so rows of
// one depth only need results of smaller depths (schedule built at setup);
// every row's sum over the old iterate is taken first, in parallel.
#pragma once

#include "kernels.hpp"

namespace pamg {

constexpr int kGsMaxBlock = kBlock;   // largest block (one workgroup of kBlock threads)
constexpr int kGsSmallBlock = 64;     // blocks of <= 64 rows run one wave per workgroup
constexpr int kGsFresh = 16;     // in-block entries of a row kept in LDS for the substitution
constexpr int kGsBatch = 8;      // row entries loaded together in the first pass

// One sweep.  ZERO: x_old = 0 (the first pre-smoothing sweep).  Row i of the
// block: d_i = ((r_i - sum_j a_ij x_old_j) - sum_{fresh j} a_ij d_j) / a_ii,
// fresh = in the block and earlier (forward) / later (backward).  The first
// pass reads each row once: the sum over x_old, and up to kGsFresh fresh
// entries (value, position in the block) into LDS; the substitution then
// runs depth by depth from LDS (a row with more fresh entries reads its row
// again).
template <int MAXB, typename T, typename RT, bool BACKWARD, bool ZERO>
static __global__ __launch_bounds__(MAXB) void k_hgs(
    int n, int nb, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ ainv, const uint8_t* __restrict__ depth, const int* __restrict__ maxd,
    const RT* __restrict__ r, const T* __restrict__ x_old, T* __restrict__ x_new, T omega_inv,
    const int* __restrict__ done) {
    if (*done) return;
    __shared__ T s_d[MAXB];
    __shared__ T s_fa[kGsFresh * MAXB];
    __shared__ uint8_t s_fq[kGsFresh * MAXB];
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = p * nb, b1 = min(n, b0 + nb);
    const int i = b0 + t;
    const bool own = t < nb && i < b1;
    int rb = 0, re = 0, dep = -1, nf = 0;
    T old = 0, ri = 0, xi = 0, ai = 0;
    if (own) {
        rb = rp[i];
        re = rp[i + 1];
        ri = (T)r[i];
        ai = ainv[i];
        dep = depth[i];
        if constexpr (!ZERO) xi = x_old[i];
        // the row in batches of kGsBatch entries: all loads of a batch in
        // flight together (addresses clamped into the row), then in order
        for (int k0 = rb; k0 < re; k0 += kGsBatch) {
            int jj[kGsBatch];
            T aa[kGsBatch], xx[kGsBatch];
#pragma unroll
            for (int u = 0; u < kGsBatch; ++u) {
                const int k = min(k0 + u, re - 1);
                jj[u] = ci[k];
                aa[u] = av[k];
            }
#pragma unroll
            for (int u = 0; u < kGsBatch; ++u) xx[u] = ZERO ? T(0) : x_old[jj[u]];
#pragma unroll
            for (int u = 0; u < kGsBatch; ++u) {
                if (k0 + u >= re) break;
                const int j = jj[u];
                if constexpr (!ZERO) old += aa[u] * xx[u];
                const bool f = BACKWARD ? (j > i && j < b1) : (j >= b0 && j < i);
                if (f) {
                    if (nf < kGsFresh) {
                        s_fa[nf * MAXB + t] = aa[u];
                        s_fq[nf * MAXB + t] = (uint8_t)(j - b0);
                    }
                    ++nf;
                }
            }
        }
    }
    // a thread's own fresh entries into registers (its own LDS slots: no barrier)
    T fa[kGsFresh];
    int fq[kGsFresh];
#pragma unroll
    for (int u = 0; u < kGsFresh; ++u) {
        fa[u] = u < nf ? s_fa[u * MAXB + t] : T(0);
        fq[u] = u < nf ? (int)s_fq[u * MAXB + t] : 0;
    }
    const int md = maxd[2 * p + (BACKWARD ? 1 : 0)];
    for (int d = 0; d <= md; ++d) {
        if (dep == d) {
            T fresh = 0;
            if (nf <= kGsFresh) {
#pragma unroll
                for (int u = 0; u < kGsFresh; ++u)
                    if (u < nf) fresh += fa[u] * s_d[fq[u]];
            } else {
                for (int k = rb; k < re; ++k) {
                    const int j = ci[k];
                    const bool f = BACKWARD ? (j > i && j < b1) : (j >= b0 && j < i);
                    if (f) fresh += av[k] * s_d[j - b0];
                }
            }
            s_d[t] = ((ri - old) - fresh) * ai;
        }
        __syncthreads();
    }
    if (own) x_new[i] = xi + s_d[t] * omega_inv;
}

// Dense coarsest solve e = A_L^-1 r: one wave per row of the symmetric
// inverse (row I read along its length, 64 consecutive columns per load),
// the lanes' partial sums met in a wave butterfly (fixed order); grid
// ceil(nL / 4) workgroups of four waves.
template <typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void k_gs_coarse(int nL, const T* __restrict__ ainv,
                                                      const RT* __restrict__ r, T* __restrict__ e,
                                                      const int* __restrict__ done) {
    if (*done) return;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int I = blockIdx.x * (kBlock / 64) + wave;
    T s = 0;
    if (I < nL) {
        const T* __restrict__ row = ainv + (size_t)I * nL;
#pragma unroll 4
        for (int j = lane; j < nL; j += 64) s += row[j] * (T)r[j];
    }
    s = wave_sum(s);
    if (I < nL && lane == 0) e[I] = s;
}

// z_m += p_m e_I for the members m of every coarse row I.
template <typename T>
static __global__ __launch_bounds__(kBlock) void k_gs_prolong(int nc, const int* __restrict__ aggptr,
                                                       const T* __restrict__ p, const T* __restrict__ e,
                                                       T* __restrict__ z, const int* __restrict__ done) {
    if (*done) return;
    const int stride = gridDim.x * kBlock;
    for (int I = blockIdx.x * kBlock + threadIdx.x; I < nc; I += stride) {
        const T eI = e[I];
        for (int m = aggptr[I]; m < aggptr[I + 1]; ++m) z[m] = z[m] + p[m] * eI;
    }
}

// Level-0 output: z_out = z (FP64) and per-workgroup partials of z . dv.
template <typename T>
static __global__ __launch_bounds__(kBlock) void k_gs_out(int n, const T* __restrict__ z, double* __restrict__ z_out,
                                                   const double* __restrict__ dv, double* __restrict__ partial,
                                                   const int* __restrict__ done) {
    if (*done) return;
    __shared__ double s_red[kBlock / 64];
    const int stride = gridDim.x * kBlock;
    double dot = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double zi = (double)z[i];
        z_out[i] = zi;
        dot += zi * dv[i];
    }
    dot = block_sum(dot, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = dot;
}

}  // namespace pamg
