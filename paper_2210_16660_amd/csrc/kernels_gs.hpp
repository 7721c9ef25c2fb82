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
// one depth only need results of smaller depths (schedule built at setup).
// The residual of the old iterate, r - A x_old, comes from the row-tile SpMV
// (coalesced, like every other pass over A); the sweep kernel then reads
// only each row's in-block entries, which are consecutive in the sorted row
// (their range is part of the schedule).
#pragma once

#include "kernels.hpp"

namespace pamg {

constexpr int kGsMaxBlock = kBlock;   // largest block (one workgroup of kBlock threads)
constexpr int kGsSmallBlock = 64;     // blocks of <= 64 rows run one wave per workgroup
constexpr int kGsFresh = 16;          // in-block entries of a row held in registers
static_assert(kGsFresh % 4 == 0, "the substitution reads its slots in groups of four");
constexpr int kGsBatch = 8;           // entries past those loaded together in a depth step
constexpr int kGsWideBatch = 32;      // the same on levels with long rows (few blocks, registers to spare)
constexpr int kGsWideRow = 64;        // mean row length from which a level takes the wide batch

// One sweep from t = r - A x_old (ZERO: x_old = 0 and t = r, the first
// pre-smoothing sweep).  Row i of the block: d_i = (t_i - sum_{fresh j}
// a_ij d_j) / a_ii with fresh = in the block and earlier (forward) / later
// (backward), in column order; x_new = x_old + d / omega.
template <int MAXB, typename T, typename TT, bool BACKWARD, bool ZERO, int RB = kGsBatch>
static __global__ __launch_bounds__(MAXB) void k_hgs(
    int n, int nb, const int* __restrict__ ci, const T* __restrict__ av, const int2* __restrict__ fr,
    const T* __restrict__ ainv, const uint8_t* __restrict__ depth, const int* __restrict__ maxd,
    const TT* __restrict__ tin, const T* __restrict__ x_old, T* __restrict__ x_new, T omega_inv,
    const int* __restrict__ done) {
    if (*done) return;
    __shared__ T s_d[MAXB];
    const int p = blockIdx.x, t = threadIdx.x;
    const int b0 = p * nb, b1 = min(n, b0 + nb);
    const int i = b0 + t;
    const bool own = t < nb && i < b1;
    int dep = -1, nf = 0, kf = 0;
    T ti = 0, xi = 0, ai = 0;
    if (own) {
        const int2 f = fr[i];
        const int before = f.y & 0xff, after = (f.y >> 8) & 0xff, diag = (f.y >> 16) & 1;
        nf = BACKWARD ? after : before;
        kf = BACKWARD ? f.x + before + diag : f.x;
        ti = (T)tin[i];
        ai = ainv[i];
        dep = depth[i];
        if constexpr (!ZERO) xi = x_old[i];
    }
    // the row's first kGsFresh in-block entries: every load issued at once
    // (indices clamped into the row's range; entry 0 for a row with none),
    // the conditions applied afterwards, so no load waits for another
    T fa[kGsFresh];
    int fq[kGsFresh];
    const int kb = nf > 0 ? kf : 0, kl = nf > 0 ? nf - 1 : 0;
#pragma unroll
    for (int u = 0; u < kGsFresh; ++u) {
        const int k = kb + min(u, kl);
        fa[u] = av[k];
        fq[u] = ci[k];
    }
#pragma unroll
    for (int u = 0; u < kGsFresh; ++u) {
        fa[u] = u < nf ? fa[u] : T(0);
        fq[u] = u < nf ? fq[u] - b0 : 0;
    }
    // every value a slot can read is finite from the start, so a slot past
    // the row's count (coefficient 0 at column 0) adds exactly +0
    s_d[t] = T(0);
    __syncthreads();
    const int md = maxd[2 * p + (BACKWARD ? 1 : 0)];
    for (int d = 0; d <= md; ++d) {
        if (dep == d) {
            // slots in groups of four: a group's LDS reads are issued
            // together, and a group no row at this depth reaches is skipped
            T fresh = 0;
#pragma unroll
            for (int g = 0; g < kGsFresh; g += 4) {
                if (g == 0 || nf > g) {
                    T dj[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) dj[u] = s_d[fq[g + u]];
#pragma unroll
                    for (int u = 0; u < 4; ++u) fresh += fa[g + u] * dj[u];
                }
            }
            // entries past the registers: RB at a time, loaded together at
            // clamped indices, added in order.  The wide form (long coarse
            // rows, registers to spare) also issues the batch's LDS reads
            // together (a slot past the row adds exactly +0); the narrow one
            // keeps a branch per entry, which holds the level-0 kernels'
            // registers down
            for (int k0 = kf + kGsFresh; k0 < kf + nf; k0 += RB) {
                T ab[RB];
                int cb[RB];
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int k = min(k0 + u, kf + nf - 1);
                    ab[u] = av[k];
                    cb[u] = ci[k] - b0;
                }
                if constexpr (RB > kGsBatch) {
#pragma unroll
                    for (int u = 0; u < RB; ++u) {
                        ab[u] = k0 + u < kf + nf ? ab[u] : T(0);
                        cb[u] = k0 + u < kf + nf ? cb[u] : 0;
                    }
                    T db[RB];
#pragma unroll
                    for (int u = 0; u < RB; ++u) db[u] = s_d[cb[u]];
#pragma unroll
                    for (int u = 0; u < RB; ++u) fresh += ab[u] * db[u];
                } else {
#pragma unroll
                    for (int u = 0; u < RB; ++u)
                        if (k0 + u < kf + nf) fresh += ab[u] * s_d[cb[u]];
                }
            }
            s_d[t] = (ti - fresh) * ai;
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
