// Device kernels of the solve phase (gfx950, wave64).
//
// Storage: every level is CSR in hierarchical order, in which the members of
// each aggregate are adjacent rows (the tentative prolongator of
// eq. (prolongator) then maps the contiguous rows aggptr[I]..aggptr[I+1]-1
// to coarse row I).  Tiles are row ranges (or aggregate ranges) whose
// entries fit kTileNnz; one workgroup streams a tile's col/val arrays once,
// fully coalesced, into LDS as products a_ij * x_j, then finishes each row
// from LDS.  A fixed grid walks the tiles: the tiles are split into eight
// contiguous chunks, one per XCD (workgroups are dispatched round-robin over
// the XCDs), so neighbouring tiles share an L2 for their vector gathers.
// Every reduction is deterministic: per-workgroup partials in a fixed order,
// then a single-workgroup finalize kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pamg {

constexpr int kXcds = 8;
constexpr int kMaxGrid = 2048;      // workgroups of a tile or vector kernel (also max partials)

struct SolveState {
    double beta, alpha, rho, rho_old, delta, delta_old, gamma;
    double rr, bb, tol, rnorm, bnorm;
    int iter, done, status, first, maxit, fixed_iters, krylov, pad;
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup; result valid in thread 0.  Fixed order.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* s_red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) t += s_red[i];
    }
    return t;
}

// Tiles handled by this workgroup: first, first+stride, ... < end.
struct TileWalk {
    int first, stride, end;
};
__device__ __forceinline__ TileWalk tile_walk(int ntiles) {
    const int G = gridDim.x, b = blockIdx.x;
    TileWalk w;
    if (G < kXcds) {
        w.first = b; w.stride = G; w.end = ntiles;
        return w;
    }
    const int x = b % kXcds, j = b / kXcds;
    const int gx = G / kXcds + (x < G % kXcds ? 1 : 0);
    w.first = (int)((long long)ntiles * x / kXcds) + j;
    w.end = (int)((long long)ntiles * (x + 1) / kXcds);
    w.stride = gx;
    return w;
}

inline int tile_grid(int ntiles) { return ntiles < kMaxGrid ? (ntiles > 0 ? ntiles : 1) : kMaxGrid; }

// ----------------------------------------------------------------------------
// Down-sweep at level l (pre-smooth from zero, residual, restriction):
//   z = D^-1 r;  t = r - A z;  rc[I] = sum_{i in G_I} p_i t_i
// Tiles are ranges of coarse rows.  z is never stored: z_j = dinv_j r_j is
// formed at the gather.
template <typename T, typename RT>
__global__ __launch_bounds__(kBlock) void k_down(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const RT* __restrict__ r, const T* __restrict__ dinv, const T* __restrict__ p,
    const int* __restrict__ aggptr, const int* __restrict__ tiles, int ntiles,
    T* __restrict__ rc, const int* __restrict__ done) {
    if (*done) return;
    __shared__ T s_prod[kTileNnz];
    __shared__ T s_red[kBlock / 64];
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    for (int t = w.first; t < w.end; t += w.stride) {
        const int c0 = tiles[t], c1 = tiles[t + 1];
        const int f0 = aggptr[c0], f1 = aggptr[c1];
        const int k0 = rp[f0], k1 = rp[f1];
        if (k1 - k0 <= kTileNnz) {
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const int k = k0 + it * kBlock + tid;
                if (k < k1) {
                    const int c = ci[k];
                    s_prod[k - k0] = av[k] * (dinv[c] * (T)r[c]);
                }
            }
            __syncthreads();
            const int I = c0 + tid;
            if (I < c1) {
                T acc = 0;
                const int m1 = aggptr[I + 1];
                for (int m = aggptr[I]; m < m1; ++m) {
                    T s = 0;
                    const int e = rp[m + 1] - k0;
                    for (int k = rp[m] - k0; k < e; ++k) s += s_prod[k];
                    acc += p[m] * ((T)r[m] - s);
                }
                rc[I] = acc;
            }
            __syncthreads();
        } else {
            // one aggregate whose rows exceed a tile
            T acc = 0;
            for (int m = f0; m < f1; ++m) {
                T s = 0;
                for (int k = rp[m] + tid; k < rp[m + 1]; k += kBlock) {
                    const int c = ci[k];
                    s += av[k] * (dinv[c] * (T)r[c]);
                }
                s = block_sum(s, s_red);
                if (tid == 0) acc += p[m] * ((T)r[m] - s);
            }
            if (tid == 0) rc[c0] = acc;
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------
// Up-sweep at level l: post-smooth z = zp + D^-1 (r - A zp), then
//   l > 0: prolongate into level l-1:  zp_f[m] = dinv_f[m] r_f[m] + p_f[m] z_I
//          for the members m of coarse row I (= this level's row);
//   l = 0: write z (FP64) and accumulate the partial of z . dv.
template <typename T, typename RT, typename RTF, bool TO_OUT>
__global__ __launch_bounds__(kBlock) void k_up(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ zp, const RT* __restrict__ r, const T* __restrict__ dinv,
    const int* __restrict__ tiles, int ntiles,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f,
    double* __restrict__ z_out, const double* __restrict__ dv, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (*done) return;
    __shared__ T s_prod[kTileNnz];
    __shared__ T s_red[kBlock / 64];
    __shared__ double s_redd[kBlock / 64];
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    double dot = 0.0;
    for (int t = w.first; t < w.end; t += w.stride) {
        const int i0 = tiles[t], i1 = tiles[t + 1];
        const int k0 = rp[i0], k1 = rp[i1];
        if (k1 - k0 <= kTileNnz) {
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const int k = k0 + it * kBlock + tid;
                if (k < k1) s_prod[k - k0] = av[k] * zp[ci[k]];
            }
            __syncthreads();
            const int i = i0 + tid;
            if (i < i1) {
                T s = 0;
                const int e = rp[i + 1] - k0;
                for (int k = rp[i] - k0; k < e; ++k) s += s_prod[k];
                const T z = zp[i] + dinv[i] * ((T)r[i] - s);
                if constexpr (TO_OUT) {
                    z_out[i] = (double)z;
                    dot += (double)z * dv[i];
                } else {
                    const int m1 = aggptr_f[i + 1];
                    for (int m = aggptr_f[i]; m < m1; ++m) zp_f[m] = dinv_f[m] * (T)r_f[m] + p_f[m] * z;
                }
            }
            __syncthreads();
        } else {
            T s = 0;
            for (int k = k0 + tid; k < k1; k += kBlock) s += av[k] * zp[ci[k]];
            s = block_sum(s, s_red);
            if (tid == 0) {
                const T z = zp[i0] + dinv[i0] * ((T)r[i0] - s);
                if constexpr (TO_OUT) {
                    z_out[i0] = (double)z;
                    dot += (double)z * dv[i0];
                } else {
                    for (int m = aggptr_f[i0]; m < aggptr_f[i0 + 1]; ++m) zp_f[m] = dinv_f[m] * (T)r_f[m] + p_f[m] * z;
                }
            }
            __syncthreads();
        }
    }
    if constexpr (TO_OUT) {
        dot = block_sum(dot, s_redd);
        if (tid == 0) partial[blockIdx.x] = dot;
    }
}

// ----------------------------------------------------------------------------
// Coarsest level: z = A_L^-1 r (dense symmetric inverse, one workgroup; r is
// staged in LDS, nL <= 4096), then prolongate into level L-1 as in k_up, or
// (single-level hierarchy) write z.
template <typename T, typename RT, typename RTF, bool TO_OUT>
__global__ __launch_bounds__(kBlock) void k_coarse(
    int nL, const T* __restrict__ ainv, const RT* __restrict__ r,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f,
    double* __restrict__ z_out, const double* __restrict__ dv, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (*done) return;
    extern __shared__ __align__(16) unsigned char s_raw[];
    T* s_r = reinterpret_cast<T*>(s_raw);
    __shared__ double s_redd[kBlock / 64];
    const int tid = threadIdx.x;
    for (int i = tid; i < nL; i += kBlock) s_r[i] = (T)r[i];
    __syncthreads();
    double dot = 0.0;
    for (int I = tid; I < nL; I += kBlock) {
        T z = 0;
        for (int j = 0; j < nL; ++j) z += ainv[(size_t)j * nL + I] * s_r[j];
        if constexpr (TO_OUT) {
            z_out[I] = (double)z;
            dot += (double)z * dv[I];
        } else {
            for (int m = aggptr_f[I]; m < aggptr_f[I + 1]; ++m) zp_f[m] = dinv_f[m] * (T)r_f[m] + p_f[m] * z;
        }
    }
    if constexpr (TO_OUT) {
        dot = block_sum(dot, s_redd);
        if (tid == 0) partial[0] = dot;
    }
}

// ----------------------------------------------------------------------------
// Prolongation alone (parity checks): zp_f[m] = dinv_f[m] r_f[m] + p_f[m] e[I]
// for the members m of every coarse row I.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(int nc, const T* __restrict__ e, const int* __restrict__ aggptr,
                                                    const double* __restrict__ r_f, const T* __restrict__ dinv_f,
                                                    const T* __restrict__ p_f, T* __restrict__ zp_f) {
    const int stride = gridDim.x * kBlock;
    for (int I = blockIdx.x * kBlock + threadIdx.x; I < nc; I += stride) {
        const T z = e[I];
        for (int m = aggptr[I]; m < aggptr[I + 1]; ++m) zp_f[m] = dinv_f[m] * (T)r_f[m] + p_f[m] * z;
    }
}

// ----------------------------------------------------------------------------
// y = A x  (or y = b - A x when b != nullptr), row tiles; optional partial of
// y . y.
template <typename T, typename XT, typename YT>
__global__ __launch_bounds__(kBlock) void k_spmv(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const XT* __restrict__ x, const double* __restrict__ b, YT* __restrict__ y,
    const int* __restrict__ tiles, int ntiles, double* __restrict__ partial) {
    __shared__ T s_prod[kTileNnz];
    __shared__ T s_red[kBlock / 64];
    __shared__ double s_redd[kBlock / 64];
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    double nrm = 0.0;
    for (int t = w.first; t < w.end; t += w.stride) {
        const int i0 = tiles[t], i1 = tiles[t + 1];
        const int k0 = rp[i0], k1 = rp[i1];
        if (k1 - k0 <= kTileNnz) {
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const int k = k0 + it * kBlock + tid;
                if (k < k1) s_prod[k - k0] = av[k] * (T)x[ci[k]];
            }
            __syncthreads();
            const int i = i0 + tid;
            if (i < i1) {
                T s = 0;
                const int e = rp[i + 1] - k0;
                for (int k = rp[i] - k0; k < e; ++k) s += s_prod[k];
                double v = b ? b[i] - (double)s : (double)s;
                y[i] = (YT)v;
                nrm += v * v;
            }
            __syncthreads();
        } else {
            T s = 0;
            for (int k = k0 + tid; k < k1; k += kBlock) s += av[k] * (T)x[ci[k]];
            s = block_sum(s, s_red);
            if (tid == 0) {
                double v = b ? b[i0] - (double)s : (double)s;
                y[i0] = (YT)v;
                nrm += v * v;
            }
            __syncthreads();
        }
    }
    if (partial) {
        nrm = block_sum(nrm, s_redd);
        if (tid == 0) partial[blockIdx.x] = nrm;
    }
}

// ----------------------------------------------------------------------------
// Krylov step, part 1: p = z + beta p_old (p = z on the first iteration),
// q = A p, partials of p.q and p.r.  p_j is formed at the gather from z and
// p_old (ping-pong buffers), with the same expression as for the owned rows.
__global__ __launch_bounds__(kBlock) void k_krylov_pq(
    const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ av,
    const double* __restrict__ z, const double* __restrict__ p_old, double* __restrict__ p_new,
    double* __restrict__ q, const double* __restrict__ r,
    const int* __restrict__ tiles, int ntiles, const SolveState* __restrict__ st,
    double* __restrict__ partial, const int* __restrict__ done) {
    if (*done) return;
    __shared__ double s_prod[kTileNnz];
    __shared__ double s_red[kBlock / 64];
    const int tid = threadIdx.x;
    const bool first = st->first != 0;
    const double beta = st->beta;
    const TileWalk w = tile_walk(ntiles);
    double pq = 0.0, pr = 0.0;
    for (int t = w.first; t < w.end; t += w.stride) {
        const int i0 = tiles[t], i1 = tiles[t + 1];
        const int k0 = rp[i0], k1 = rp[i1];
        if (k1 - k0 <= kTileNnz) {
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const int k = k0 + it * kBlock + tid;
                if (k < k1) {
                    const int c = ci[k];
                    const double pj = first ? z[c] : z[c] + beta * p_old[c];
                    s_prod[k - k0] = av[k] * pj;
                }
            }
            __syncthreads();
            const int i = i0 + tid;
            if (i < i1) {
                double s = 0.0;
                const int e = rp[i + 1] - k0;
                for (int k = rp[i] - k0; k < e; ++k) s += s_prod[k];
                const double pi = first ? z[i] : z[i] + beta * p_old[i];
                p_new[i] = pi;
                q[i] = s;
                pq += pi * s;
                pr += pi * r[i];
            }
            __syncthreads();
        } else {
            double s = 0.0;
            for (int k = k0 + tid; k < k1; k += kBlock) {
                const int c = ci[k];
                const double pj = first ? z[c] : z[c] + beta * p_old[c];
                s += av[k] * pj;
            }
            s = block_sum(s, s_red);
            if (tid == 0) {
                const double pi = first ? z[i0] : z[i0] + beta * p_old[i0];
                p_new[i0] = pi;
                q[i0] = s;
                pq += pi * s;
                pr += pi * r[i0];
            }
            __syncthreads();
        }
    }
    pq = block_sum(pq, s_red);
    __syncthreads();
    pr = block_sum(pr, s_red);
    if (tid == 0) {
        partial[2 * blockIdx.x] = pq;
        partial[2 * blockIdx.x + 1] = pr;
    }
}

// Krylov step, part 2: x += alpha p, r -= alpha q, partial of r.r.
__global__ __launch_bounds__(kBlock) void k_krylov_update(
    int n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, const SolveState* __restrict__ st, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (*done) return;
    __shared__ double s_red[kBlock / 64];
    const double alpha = st->alpha;
    double rr = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rr += ri * ri;
    }
    rr = block_sum(rr, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = rr;
}

// Fixed-order sum of `count` partials spaced `stride` apart (one workgroup).
__device__ __forceinline__ double reduce_partials(const double* __restrict__ partial, int count, int stride,
                                                  double* s_red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) s += partial[(size_t)i * stride];
    return block_sum(s, s_red);
}

// beta (and rho for PCG) from the partials of z.dv written by the level-0 up-sweep.
__global__ __launch_bounds__(kBlock) void k_fin_beta(SolveState* __restrict__ st, const double* __restrict__ partial,
                                                     int count) {
    if (st->done) return;
    __shared__ double s_red[kBlock / 64];
    const double d = reduce_partials(partial, count, 1, s_red);
    if (threadIdx.x == 0) {
        if (st->krylov == PAMG_KRYLOV_CG) {        // d = r.z
            st->rho = d;
            st->beta = st->first ? 0.0 : d / st->rho_old;
        } else {                                    // d = z.q_old
            st->beta = st->first ? 0.0 : -d / st->delta_old;
        }
    }
}

// delta = p.q, gamma = p.r, alpha.
__global__ __launch_bounds__(kBlock) void k_fin_alpha(SolveState* __restrict__ st, const double* __restrict__ partial,
                                                      int count) {
    if (st->done) return;
    __shared__ double s_red[kBlock / 64];
    const double pq = reduce_partials(partial, count, 2, s_red);
    __syncthreads();
    const double pr = reduce_partials(partial + 1, count, 2, s_red);
    if (threadIdx.x == 0) {
        st->delta = pq;
        st->gamma = pr;
        if (!(pq > 0.0)) {
            st->status = (pq != pq) ? PAMG_E_NUMERIC : PAMG_E_NOT_SPD;
            st->done = 1;
            return;
        }
        const double num = (st->krylov == PAMG_KRYLOV_CG) ? st->rho : pr;
        st->alpha = num / pq;
        if (st->krylov == PAMG_KRYLOV_CG) st->rho_old = st->rho;
        st->delta_old = pq;
        st->first = 0;
    }
}

// ||r||, iteration count and the stopping test ||r|| <= tol ||b||.
__global__ __launch_bounds__(kBlock) void k_fin_norm(SolveState* __restrict__ st, const double* __restrict__ partial,
                                                     int count) {
    if (st->done) return;
    __shared__ double s_red[kBlock / 64];
    const double rr = reduce_partials(partial, count, 1, s_red);
    if (threadIdx.x == 0) {
        st->rr = rr;
        const double rn = sqrt(rr);
        st->rnorm = rn;
        const int it = st->iter + 1;
        st->iter = it;
        if (rn != rn) {
            st->status = PAMG_E_NUMERIC;
            st->done = 1;
        } else if (st->fixed_iters > 0) {
            if (it >= st->fixed_iters) { st->status = PAMG_OK; st->done = 1; }
        } else if (rn <= st->tol * st->bnorm) {
            st->status = PAMG_OK;
            st->done = 1;
        } else if (it >= st->maxit) {
            st->status = PAMG_NOT_CONVERGED;
            st->done = 1;
        }
    }
}

// Start of a solve (or restart): ||b||, ||r|| from partials (b.b in bb_part,
// r.r in rr_part); sets the stopping state.  bb_count == 0: keep st->bnorm.
__global__ __launch_bounds__(kBlock) void k_fin_init(SolveState* __restrict__ st, const double* __restrict__ bb_part,
                                                     int bb_count, const double* __restrict__ rr_part, int rr_count) {
    __shared__ double s_red[kBlock / 64];
    double bb = 0.0;
    if (bb_count > 0) bb = reduce_partials(bb_part, bb_count, 1, s_red);
    __syncthreads();
    const double rr = reduce_partials(rr_part, rr_count, 1, s_red);
    if (threadIdx.x == 0) {
        if (bb_count > 0) {
            st->bb = bb;
            st->bnorm = sqrt(bb);
        }
        st->rr = rr;
        st->rnorm = sqrt(rr);
        st->first = 1;
        st->done = 0;
        st->status = PAMG_NOT_CONVERGED;
        if (st->bnorm == 0.0) {
            st->status = PAMG_OK;
            st->done = 2;            // zero right-hand side: x = 0
        } else if (st->fixed_iters <= 0 && st->rnorm <= st->tol * st->bnorm) {
            st->status = PAMG_OK;
            st->done = 1;
        } else if (st->rnorm != st->rnorm) {
            st->status = PAMG_E_NUMERIC;
            st->done = 1;
        }
    }
}

// ----------------------------------------------------------------------------
// vector helpers
template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_gather(int n, const int* __restrict__ idx, const S* __restrict__ src,
                                                   D* __restrict__ dst) {
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = (D)src[idx[i]];
}

template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(long long n, const S* __restrict__ src, D* __restrict__ dst) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = (D)src[i];
}

// b.b partials, and optionally r = b (x0 = 0) with r.r partials equal to b.b
__global__ __launch_bounds__(kBlock) void k_norm2(int n, const double* __restrict__ b, double* __restrict__ copy_to,
                                                  double* __restrict__ partial) {
    __shared__ double s_red[kBlock / 64];
    double s = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double v = b[i];
        if (copy_to) copy_to[i] = v;
        s += v * v;
    }
    s = block_sum(s, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_fill(long long n, double* __restrict__ x, double v) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = v;
}

}  // namespace pamg
