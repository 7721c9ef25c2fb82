// Multi-right-hand-side kernels: the same V-cycle and Krylov steps applied to
// kW = 16 independent right-hand sides at once.
//
// Vectors are n x 16, row-major, in hierarchical order: the 16 values of a
// row are one 128-byte (FP64) or 64-byte (FP32) line, so every gathered
// neighbour is one line and every matrix entry is read once per 16 columns.
// A row is handled by a group of kW/CPL lanes, each lane owning CPL adjacent
// columns.  Per column the arithmetic is a fixed sequence (entries in CSR
// order, members in order), independent of the unroll depth U, of CPL and
// of the other columns: a column's result does not depend on what else is
// in the batch.  Reductions are per-workgroup partials combined in a fixed
// order by single-workgroup finalize kernels, one recurrence per column.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace pamg {

constexpr int kW = 16;   // right-hand sides per batch

struct BatchCol {
    double beta, alpha, rho, rho_old, delta_old, rnorm, bnorm, tol;
    int iter, done, status, first, maxit, fixed_iters, active, pad;
};

struct BatchState {
    BatchCol col[kW];
    int all_done, krylov, pad0, pad1;
};

// ---------------------------------------------------------------- helpers

template <typename T, int C>
struct Vec {
    T v[C];
};

template <typename T, int C>
__device__ __forceinline__ Vec<T, C> vload(const T* p) {
    Vec<T, C> r;
    if constexpr (C == 1) {
        r.v[0] = p[0];
    } else if constexpr (C == 2) {
        using V2 = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
        const V2 t = *reinterpret_cast<const V2*>(p);
        r.v[0] = t.x;
        r.v[1] = t.y;
    } else if constexpr (std::is_same<T, float>::value) {
        static_assert(C == 4, "1, 2 or 4 columns per lane");
        const float4 t = *reinterpret_cast<const float4*>(p);
        r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    } else {
        static_assert(C == 4, "1, 2 or 4 columns per lane");
        const double2 t0 = *reinterpret_cast<const double2*>(p);
        const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
        r.v[0] = t0.x; r.v[1] = t0.y; r.v[2] = t1.x; r.v[3] = t1.y;
    }
    return r;
}

template <typename T, int C>
__device__ __forceinline__ void vstore(T* p, const Vec<T, C>& a) {
    if constexpr (C == 1) {
        p[0] = a.v[0];
    } else if constexpr (C == 2) {
        using V2 = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
        V2 t;
        t.x = a.v[0];
        t.y = a.v[1];
        *reinterpret_cast<V2*>(p) = t;
    } else if constexpr (std::is_same<T, float>::value) {
        float4 t;
        t.x = a.v[0]; t.y = a.v[1]; t.z = a.v[2]; t.w = a.v[3];
        *reinterpret_cast<float4*>(p) = t;
    } else {
        double2 t0, t1;
        t0.x = a.v[0]; t0.y = a.v[1];
        t1.x = a.v[2]; t1.y = a.v[3];
        *reinterpret_cast<double2*>(p) = t0;
        *reinterpret_cast<double2*>(p + 2) = t1;
    }
}

// Units (rows or coarse rows) handled by one row group: first, +stride, < end;
// units are split into contiguous per-XCD chunks as in tile_walk.
__device__ __forceinline__ TileWalk unit_walk(int nunits, int gpb, int g) {
    const int G = gridDim.x, b = blockIdx.x;
    TileWalk w;
    if (G < kXcds) {
        w.first = b * gpb + g;
        w.stride = G * gpb;
        w.end = nunits;
        return w;
    }
    const int x = b % kXcds, j = b / kXcds;
    const int gx = G / kXcds + (x < G % kXcds ? 1 : 0);
    w.first = (int)((long long)nunits * x / kXcds) + j * gpb + g;
    w.end = (int)((long long)nunits * (x + 1) / kXcds);
    w.stride = gx * gpb;
    return w;
}

inline int unit_grid(long long nunits, int gpb) {
    long long g = (nunits + gpb - 1) / gpb;
    if (g > kMaxGrid) g = kMaxGrid;
    return g < 1 ? 1 : (int)g;
}

// s[q] += sum over row entries [kb, ke) of a_k x[c_k][col0 + q], in entry order.
// (The lanes of a group load the same index and value; plain loads keep the
// line in L2 for the group's next entries: non-temporal loads made the
// 16-column engine 1.6x slower.)
template <int U, int CPL, typename T, typename XT>
__device__ __forceinline__ void row_accumulate(int kb, int ke, const int* __restrict__ ci, const T* __restrict__ av,
                                               const XT* __restrict__ x, int col0, T (&s)[CPL]) {
    int k = kb;
    for (; k + U <= ke; k += U) {
        int c[U];
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = ci[k + u];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = av[k + u];
        Vec<XT, CPL> xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = vload<XT, CPL>(x + (size_t)c[u] * kW + col0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < CPL; ++q) s[q] += a[u] * (T)xv[u].v[q];
    }
    for (; k < ke; ++k) {
        const Vec<XT, CPL> xv = vload<XT, CPL>(x + (size_t)ci[k] * kW + col0);
        const T a = av[k];
#pragma unroll
        for (int q = 0; q < CPL; ++q) s[q] += a * (T)xv.v[q];
    }
}

// ---------------------------------------------------------------- V-cycle

// Down-sweep: rc[I] = sum_{m in G_I} p_m (r_m - (A D^-1 r)_m), per column.
template <int U, int CPL, typename T, typename RT>
static __global__ __launch_bounds__(kBlock) void kb_down(int nc, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const T* __restrict__ vd, const RT* __restrict__ r,
                                                  const T* __restrict__ p, const int* __restrict__ aggptr,
                                                  T* __restrict__ rc, const int* __restrict__ done) {
    if (*done) return;
    constexpr int LPR = kW / CPL, GPB = kBlock / LPR;
    const int g = threadIdx.x / LPR, col0 = (threadIdx.x % LPR) * CPL;
    const TileWalk w = unit_walk(nc, GPB, g);
    for (int I = w.first; I < w.end; I += w.stride) {
        const int m0 = aggptr[I], m1 = aggptr[I + 1];
        T acc[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) acc[q] = 0;
        for (int m = m0; m < m1; ++m) {
            T s[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) s[q] = 0;
            row_accumulate<U, CPL, T, RT>(rp[m], rp[m + 1], ci, vd, r, col0, s);
            const Vec<RT, CPL> rm = vload<RT, CPL>(r + (size_t)m * kW + col0);
            const T pm = p[m];
#pragma unroll
            for (int q = 0; q < CPL; ++q) acc[q] += pm * ((T)rm.v[q] - s[q]);
        }
        Vec<T, CPL> o;
#pragma unroll
        for (int q = 0; q < CPL; ++q) o.v[q] = acc[q];
        vstore<T, CPL>(rc + (size_t)I * kW + col0, o);
    }
}

// Up-sweep at level l > 0: z = zp + D^-1 (r - A zp), prolongated into level
// l-1: zp_f[m] = dinv_f[m] r_f[m] + p_f[m] z for the members m of row i.
template <int U, int CPL, typename T, typename RT, typename RTF>
static __global__ __launch_bounds__(kBlock) void kb_up(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const T* __restrict__ av, const T* __restrict__ zp,
                                                const RT* __restrict__ r, const T* __restrict__ dinv,
                                                const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f,
                                                const T* __restrict__ dinv_f, const T* __restrict__ p_f,
                                                T* __restrict__ zp_f, const int* __restrict__ done) {
    if (*done) return;
    constexpr int LPR = kW / CPL, GPB = kBlock / LPR;
    const int g = threadIdx.x / LPR, col0 = (threadIdx.x % LPR) * CPL;
    const TileWalk w = unit_walk(n, GPB, g);
    for (int i = w.first; i < w.end; i += w.stride) {
        T s[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) s[q] = 0;
        row_accumulate<U, CPL, T, T>(rp[i], rp[i + 1], ci, av, zp, col0, s);
        const Vec<T, CPL> zpi = vload<T, CPL>(zp + (size_t)i * kW + col0);
        const Vec<RT, CPL> ri = vload<RT, CPL>(r + (size_t)i * kW + col0);
        const T di = dinv[i];
        T z[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) z[q] = zpi.v[q] + di * ((T)ri.v[q] - s[q]);
        for (int m = aggptr_f[i]; m < aggptr_f[i + 1]; ++m) {
            const Vec<RTF, CPL> rf = vload<RTF, CPL>(r_f + (size_t)m * kW + col0);
            const T df = dinv_f[m], pf = p_f[m];
            Vec<T, CPL> o;
#pragma unroll
            for (int q = 0; q < CPL; ++q) o.v[q] = prolong_value(df, (T)rf.v[q], pf, z[q]);
            vstore<T, CPL>(zp_f + (size_t)m * kW + col0, o);
        }
    }
}

// Level-0 up-sweep: z = zp + D^-1 (r - A zp) written in FP64, with per-column
// partials of z . dv.  Fixed shape, whatever the tuning (its partial sums
// must not depend on it): unroll 8 and four columns per lane (one 16-byte
// load in FP32, two in FP64).
template <typename T>
constexpr int up0_cols() { return 4; }
template <typename T>
constexpr int up0_rows_per_block() { return kBlock / (kW / up0_cols<T>()); }

// z is written in the cycle's precision T: with the FP32 cycle z is a float
// (exactly its FP64 widening), so the Krylov pass gathers 64-byte rows.
template <typename T>
static __global__ __launch_bounds__(kBlock) void kb_up0(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const T* __restrict__ av, const T* __restrict__ zp,
                                                 const T* __restrict__ r, const T* __restrict__ dinv,
                                                 T* __restrict__ z_out, const double* __restrict__ dv,
                                                 double* __restrict__ partial, const int* __restrict__ done) {
    if (*done) return;
    constexpr int CPL = up0_cols<T>(), LPR = kW / CPL, GPB = kBlock / LPR;
    __shared__ double s_dot[GPB][kW];
    const int g = threadIdx.x / LPR, col0 = (threadIdx.x % LPR) * CPL;
    const TileWalk w = unit_walk(n, GPB, g);
    double dot[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) dot[q] = 0.0;
    for (int i = w.first; i < w.end; i += w.stride) {
        T s[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) s[q] = 0;
        row_accumulate<8, CPL, T, T>(rp[i], rp[i + 1], ci, av, zp, col0, s);
        const size_t e = (size_t)i * kW + col0;
        const Vec<T, CPL> zv = vload<T, CPL>(zp + e);
        const T di = dinv[i];
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const T z = zv.v[q] + di * (r[e + q] - s[q]);
            z_out[e + q] = z;
            dot[q] += (double)z * dv[e + q];
        }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) s_dot[g][col0 + q] = dot[q];
    __syncthreads();
    if (threadIdx.x < kW) {
        double t = 0.0;
        for (int q = 0; q < GPB; ++q) t += s_dot[q][threadIdx.x];
        partial[(size_t)blockIdx.x * kW + threadIdx.x] = t;
    }
}

// Coarsest level: Z = A_L^-1 R (nL x nL times nL x 16), then prolongation
// into level L-1 or (single level) z out with per-column partials of z . dv.
// FP64 uses the matrix cores: v_mfma_f64_16x16x4_f64 on 16-row blocks, one
// wave per block.  Z goes through the scratch zc (nL x 16).
template <typename T, typename RT, typename RTF, bool OUT>
static __global__ __launch_bounds__(kCoarseThreads) void kb_coarse(
    int nL, const T* __restrict__ ainv, const RT* __restrict__ r, T* __restrict__ zc,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f, double* __restrict__ z_out, const double* __restrict__ dv,
    double* __restrict__ partial, const int* __restrict__ done) {
    if (*done) return;
    const int tid = threadIdx.x, wave = tid / 64, l = tid % 64;
    constexpr int kWaves = kCoarseThreads / 64;
    if constexpr (std::is_same<T, double>::value) {
        // A tile (16 x 4): lane l holds A[l % 16][l / 16]; B tile (4 x 16):
        // lane l holds B[l / 16][l % 16]; D (16 x 16): result register i of
        // lane l holds row 4 i + l / 16 of column l % 16 (one-row groups for
        // the FP64 instruction).
        using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
        for (int rb = wave; rb * 16 < nL; rb += kWaves) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            const int m = rb * 16 + (l % 16);
            for (int k0 = 0; k0 < nL; k0 += 4) {
                const int k = k0 + l / 16;
                const double a = (m < nL && k < nL) ? ainv[(size_t)m * nL + k] : 0.0;
                const double b = (k < nL) ? (double)r[(size_t)k * kW + (l % 16)] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = rb * 16 + 4 * i + (l / 16);
                if (row < nL) zc[(size_t)row * kW + (l % 16)] = acc[i];
            }
        }
    } else {
        for (int e = tid; e < nL * kW; e += kCoarseThreads) {
            const int I = e / kW, c = e % kW;
            T s = 0;
            for (int j = 0; j < nL; ++j) s += ainv[(size_t)I * nL + j] * (T)r[(size_t)j * kW + c];
            zc[e] = s;
        }
    }
    __threadfence_block();
    __syncthreads();
    double dot = 0.0;
    for (int e = tid; e < nL * kW; e += kCoarseThreads) {
        const int I = e / kW, c = e % kW;
        const T z = zc[e];
        if constexpr (OUT) {
            z_out[e] = (double)z;
            dot += (double)z * dv[e];
        } else {
            for (int m = aggptr_f[I]; m < aggptr_f[I + 1]; ++m)
                zp_f[(size_t)m * kW + c] = prolong_value(dinv_f[m], (T)r_f[(size_t)m * kW + c], p_f[m], z);
        }
    }
    if constexpr (OUT) {
        __shared__ double s_dot[kCoarseThreads / kW][kW];
        s_dot[tid / kW][tid % kW] = dot;
        __syncthreads();
        if (tid < kW) {
            double t = 0.0;
            for (int q = 0; q < kCoarseThreads / kW; ++q) t += s_dot[q][tid];
            partial[tid] = t;
        }
    }
}

// Large coarsest level (L >= 1): the product and the prolongation into level
// L-1 spread over many workgroups of 256 threads (OUT: the product is written
// to z_out instead, n_L x 16 in FP64, for the per-operator parity check).  FP64: one wave per 16-row
// block on the matrix cores (four waves, 64 rows per workgroup), prolongated
// straight from the result registers.  FP32: a workgroup owns 16 rows and its
// threads split the columns j in 16 fixed ranges (one row and all 16
// right-hand sides per thread), meeting in LDS in a fixed order; small row
// blocks give ceil(n_L / 16) workgroups, enough to spread a coarsest level of
// a few thousand rows over the chip.
template <typename T>
constexpr int coarse_rows_block_rows_b() { return std::is_same<T, double>::value ? 64 : 16; }
// Coarsest sizes from which the many-workgroup kernel replaces the single
// workgroup: FP64 keeps the single-workgroup matrix-core product up to the
// single-right-hand-side threshold; FP32, whose single workgroup computes
// each (row, column) entry as a serial loop over n_L, switches early.
template <typename T>
constexpr int coarse_rows_min_b() { return std::is_same<T, double>::value ? kCoarseRowsMin : 32; }
template <typename T>
inline int coarse_rows_grid_b(int nL) {
    return (nL + coarse_rows_block_rows_b<T>() - 1) / coarse_rows_block_rows_b<T>();
}

template <typename T, typename RT, typename RTF, bool OUT = false>
static __global__ __launch_bounds__(kBlock) void kb_coarse_rows(
    int nL, const T* __restrict__ ainv, const RT* __restrict__ r,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f, double* __restrict__ z_out, const int* __restrict__ done) {
    if (*done) return;
    const int tid = threadIdx.x, wave = tid / 64, l = tid % 64;
    if constexpr (std::is_same<T, double>::value) {
        using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
        const int rb = blockIdx.x * (kBlock / 64) + wave;        // 16-row block of this wave
        if (rb * 16 >= nL) return;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        const int m = rb * 16 + (l % 16);
        for (int k0 = 0; k0 < nL; k0 += 4) {
            const int k = k0 + l / 16;
            const double a = (m < nL && k < nL) ? ainv[(size_t)m * nL + k] : 0.0;
            const double b = (k < nL) ? (double)r[(size_t)k * kW + (l % 16)] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        const int c = l % 16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int I = rb * 16 + 4 * i + (l / 16);
            if (I >= nL) continue;
            const T z = acc[i];
            if constexpr (OUT) {
                z_out[(size_t)I * kW + c] = (double)z;
                continue;
            }
            for (int mm = aggptr_f[I]; mm < aggptr_f[I + 1]; ++mm)
                zp_f[(size_t)mm * kW + c] = prolong_value(dinv_f[mm], (T)r_f[(size_t)mm * kW + c], p_f[mm], z);
        }
    } else {
        constexpr int R = coarse_rows_block_rows_b<T>(), G = kBlock / R;
        __shared__ T s_part[G][R][kW + 1];
        const int g = tid / R, lt = tid % R;
        const int I = blockIdx.x * R + lt;
        const int j0 = (int)((long long)nL * g / G), j1 = (int)((long long)nL * (g + 1) / G);
        T acc[kW];
#pragma unroll
        for (int c = 0; c < kW; ++c) acc[c] = 0;
        if (I < nL) {
            for (int j = j0; j < j1; ++j) {
                const T a = ainv[(size_t)j * nL + I];
#pragma unroll
                for (int c = 0; c < kW; ++c) acc[c] += a * (T)r[(size_t)j * kW + c];
            }
        }
#pragma unroll
        for (int c = 0; c < kW; ++c) s_part[g][lt][c] = acc[c];
        __syncthreads();
        for (int e = tid; e < R * kW; e += kBlock) {
            const int row = e / kW, c = e % kW;
            const int II = blockIdx.x * R + row;
            if (II >= nL) continue;
            T z = s_part[0][row][c];
            for (int q = 1; q < G; ++q) z += s_part[q][row][c];
            if constexpr (OUT) {
                z_out[(size_t)II * kW + c] = (double)z;
                continue;
            }
            for (int mm = aggptr_f[II]; mm < aggptr_f[II + 1]; ++mm)
                zp_f[(size_t)mm * kW + c] = prolong_value(dinv_f[mm], (T)r_f[(size_t)mm * kW + c], p_f[mm], z);
        }
    }
}

// FP64 -> FP32 copy of n x 16 values (the FP32 cycle's level-0 right-hand
// side, for the debug entry point; in the iteration every writer of R also
// writes R32).
static __global__ __launch_bounds__(kBlock) void kb_narrow(long long cnt, const double* __restrict__ src,
                                                    float* __restrict__ dst, const int* __restrict__ done) {
    if (*done) return;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += stride) dst[i] = (float)src[i];
}

// ---------------------------------------------------------------- Krylov

// p = z + beta_c p_old (p = z on a column's first iteration), q = A p as
// A z + beta_c q_old (the same vector in exact arithmetic: only z is
// gathered, one line per entry instead of two), and per-column partials of
// p.q and p.r.  A column on its first iteration, or finished, takes q = A z
// (an idle column's q stays bounded).  q holds q_old on entry; each element
// is read before it is overwritten, by the same lane.  Fixed shape: unroll 8,
// four columns per lane (two 16-byte loads).
constexpr int kKrylovCols = 4;
constexpr int kKrylovRowsPerBlock = kBlock / (kW / kKrylovCols);

template <typename ZT>
static __global__ __launch_bounds__(kBlock) void kb_krylov_pq(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ av, const ZT* __restrict__ z,
                                                       const double* __restrict__ p_old, double* __restrict__ p_new,
                                                       double* __restrict__ q, const double* __restrict__ r,
                                                       const BatchState* __restrict__ st, double* __restrict__ partial,
                                                       const int* __restrict__ done) {
    if (*done) return;
    constexpr int CPL = kKrylovCols, LPR = kW / CPL, GPB = kBlock / LPR;
    __shared__ double s_pq[GPB][kW], s_pr[GPB][kW];
    const int g = threadIdx.x / LPR, col0 = (threadIdx.x % LPR) * CPL;
    bool first[CPL], fresh[CPL];
    double beta[CPL], pq[CPL], pr[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const BatchCol& C = st->col[col0 + c];
        first[c] = C.first != 0;
        fresh[c] = first[c] || C.done != 0;
        beta[c] = C.beta;
        pq[c] = 0.0;
        pr[c] = 0.0;
    }
    const TileWalk w = unit_walk(n, GPB, g);
    for (int i = w.first; i < w.end; i += w.stride) {
        double s[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) s[c] = 0.0;
        row_accumulate<8, CPL, double, ZT>(rp[i], rp[i + 1], ci, av, z, col0, s);
        const size_t e = (size_t)i * kW + col0;
        const Vec<ZT, CPL> zi = vload<ZT, CPL>(z + e);
        const Vec<double, CPL> po = vload<double, CPL>(p_old + e);
        const Vec<double, CPL> qo = vload<double, CPL>(q + e), ri = vload<double, CPL>(r + e);
        Vec<double, CPL> pn, qn;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const double zc = (double)zi.v[c];
            pn.v[c] = first[c] ? zc : zc + beta[c] * po.v[c];
            qn.v[c] = fresh[c] ? s[c] : s[c] + beta[c] * qo.v[c];
            pq[c] += pn.v[c] * qn.v[c];
            pr[c] += pn.v[c] * ri.v[c];
        }
        vstore<double, CPL>(p_new + e, pn);
        vstore<double, CPL>(q + e, qn);
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        s_pq[g][col0 + c] = pq[c];
        s_pr[g][col0 + c] = pr[c];
    }
    __syncthreads();
    if (threadIdx.x < kW) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < GPB; ++t) { a += s_pq[t][threadIdx.x]; b += s_pr[t][threadIdx.x]; }
        partial[((size_t)blockIdx.x * kW + threadIdx.x) * 2] = a;
        partial[((size_t)blockIdx.x * kW + threadIdx.x) * 2 + 1] = b;
    }
}

// x += alpha_c p, r -= alpha_c q for the active columns; partials of r.r.
// r32 (the FP32 cycle): r rounded to FP32 beside it, the cycle's level-0
// right-hand side.
static __global__ __launch_bounds__(kBlock) void kb_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                    float* __restrict__ r32, const double* __restrict__ p,
                                                    const double* __restrict__ q, const BatchState* __restrict__ st,
                                                    double* __restrict__ partial, const int* __restrict__ done) {
    if (*done) return;
    constexpr int GPB = kBlock / kW;
    __shared__ double s_rr[GPB][kW];
    const int g = threadIdx.x / kW, lane = threadIdx.x % kW;
    const bool live = st->col[lane].done == 0;
    const double alpha = st->col[lane].alpha;
    double rr = 0.0;
    const int stride = gridDim.x * GPB;
    for (int i = blockIdx.x * GPB + g; i < n; i += stride) {
        const size_t e = (size_t)i * kW + lane;
        double ri = r[e];
        if (live) {
            x[e] += alpha * p[e];
            ri -= alpha * q[e];
            r[e] = ri;
            if (r32) r32[e] = (float)ri;
        }
        rr += ri * ri;
    }
    s_rr[g][lane] = rr;
    __syncthreads();
    if (threadIdx.x < kW) {
        double t = 0.0;
        for (int q2 = 0; q2 < GPB; ++q2) t += s_rr[q2][threadIdx.x];
        partial[(size_t)blockIdx.x * kW + threadIdx.x] = t;
    }
}

// Fixed-order per-column sums of `count` partials (partial gi of column c at
// ((gi * kW + c) * stride + off)) by one workgroup of kFinThreads: thread t
// takes column t % kW and the partials gi = t / kW, + kFinParts, ...
// (neighbouring threads read neighbouring columns of one partial), four loads
// in flight; the kFinParts part sums of a column then meet in LDS in part
// order.  The result is valid in threads 0 .. kW-1 (thread c: column c).
constexpr int kFinThreads = 1024;
constexpr int kFinParts = kFinThreads / kW;

__device__ __forceinline__ double col_sum(const double* __restrict__ partial, int count, int stride, int off,
                                          double (*s_part)[kW]) {
    const int c = threadIdx.x % kW, part = threadIdx.x / kW;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int gi = part;
    for (; gi + 3 * kFinParts < count; gi += 4 * kFinParts) {
        s0 += partial[((size_t)gi * kW + c) * stride + off];
        s1 += partial[((size_t)(gi + kFinParts) * kW + c) * stride + off];
        s2 += partial[((size_t)(gi + 2 * kFinParts) * kW + c) * stride + off];
        s3 += partial[((size_t)(gi + 3 * kFinParts) * kW + c) * stride + off];
    }
    for (; gi < count; gi += kFinParts) s0 += partial[((size_t)gi * kW + c) * stride + off];
    s_part[part][c] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < kW)
        for (int q = 0; q < kFinParts; ++q) t += s_part[q][threadIdx.x];
    __syncthreads();
    return t;
}

// all_done = no active column left running (read after the barrier, which
// orders this workgroup's global writes).
__device__ __forceinline__ void update_all_done(BatchState* st) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int all = 1;
        for (int c = 0; c < kW; ++c)
            if (st->col[c].active && !st->col[c].done) all = 0;
        st->all_done = all;
    }
}

// beta (and rho for PCG) from the partials of z.dv.
static __global__ __launch_bounds__(kFinThreads) void kb_fin_beta(BatchState* __restrict__ st,
                                                                  const double* __restrict__ partial, int count) {
    if (st->all_done) return;
    __shared__ double s_part[kFinParts][kW];
    const int c = threadIdx.x;
    const double d = col_sum(partial, count, 1, 0, s_part);
    if (c < kW) {
        BatchCol& C = st->col[c];
        if (C.active && !C.done) {
            if (st->krylov == PAMG_KRYLOV_CG) {
                C.rho = d;
                C.beta = C.first ? 0.0 : d / C.rho_old;
            } else {
                C.beta = C.first ? 0.0 : -d / C.delta_old;
            }
        }
    }
}

static __global__ __launch_bounds__(kFinThreads) void kb_fin_alpha(BatchState* __restrict__ st,
                                                                   const double* __restrict__ partial, int count) {
    if (st->all_done) return;
    __shared__ double s_part[kFinParts][kW];
    const int c = threadIdx.x;
    const double pq = col_sum(partial, count, 2, 0, s_part);
    const double pr = col_sum(partial, count, 2, 1, s_part);
    if (c < kW) {
        BatchCol& C = st->col[c];
        if (C.active && !C.done) {
            if (!(pq > 0.0)) {
                C.status = (pq != pq) ? PAMG_E_NUMERIC : PAMG_E_NOT_SPD;
                C.done = 1;
                C.alpha = 0.0;
            } else {
                const double num = (st->krylov == PAMG_KRYLOV_CG) ? C.rho : pr;
                C.alpha = num / pq;
                if (st->krylov == PAMG_KRYLOV_CG) C.rho_old = C.rho;
                C.delta_old = pq;
                C.first = 0;
            }
        }
    }
    update_all_done(st);
}

static __global__ __launch_bounds__(kFinThreads) void kb_fin_norm(BatchState* __restrict__ st,
                                                                  const double* __restrict__ partial, int count) {
    if (st->all_done) return;
    __shared__ double s_part[kFinParts][kW];
    const int c = threadIdx.x;
    const double rr = col_sum(partial, count, 1, 0, s_part);
    if (c < kW) {
        BatchCol& C = st->col[c];
        if (C.active && !C.done) {
            const double rn = sqrt(rr);
            C.rnorm = rn;
            const int it = C.iter + 1;
            C.iter = it;
            if (rn != rn) {
                C.status = PAMG_E_NUMERIC;
                C.done = 1;
            } else if (C.fixed_iters > 0) {
                if (it >= C.fixed_iters) { C.status = PAMG_OK; C.done = 1; }
            } else if (rn <= C.tol * C.bnorm) {
                C.status = PAMG_OK;
                C.done = 1;
            } else if (it >= C.maxit) {
                C.status = PAMG_NOT_CONVERGED;
                C.done = 1;
            }
        }
    }
    update_all_done(st);
}

// Start (or restart) the columns in `mask`: ||b|| and ||r|| from partials
// (bb_count == 0: keep bnorm), first iteration next, stopping state.
static __global__ __launch_bounds__(kFinThreads) void kb_fin_init(BatchState* __restrict__ st,
                                                                  const double* __restrict__ bb_part, int bb_count,
                                                                  const double* __restrict__ rr_part, int rr_count,
                                                                  int mask) {
    __shared__ double s_part[kFinParts][kW];
    const int c = threadIdx.x;
    const double bb = bb_count > 0 ? col_sum(bb_part, bb_count, 1, 0, s_part) : 0.0;
    const double rr = col_sum(rr_part, rr_count, 1, 0, s_part);
    if (c < kW && ((mask >> c) & 1)) {
        BatchCol& C = st->col[c];
        if (bb_count > 0) C.bnorm = sqrt(bb);
        C.rnorm = sqrt(rr);
        C.first = 1;
        C.done = 0;
        C.active = 1;
        C.status = PAMG_NOT_CONVERGED;
        if (C.bnorm == 0.0) {
            C.status = PAMG_OK;
            C.done = 2;   // zero right-hand side: x = 0
        } else if (C.fixed_iters <= 0 && C.rnorm <= C.tol * C.bnorm) {
            C.status = PAMG_OK;
            C.done = 1;
        } else if (C.rnorm != C.rnorm) {
            C.status = PAMG_E_NUMERIC;
            C.done = 1;
        }
    }
    update_all_done(st);
}

// Load columns from caller buffers (src[c] != nullptr: column c of b in the
// caller's numbering): B[:, c] = b_c (hierarchical order), R[:, c] = B[:, c],
// X[:, c] = 0; per-column partials of b.b (also r.r).
static __global__ __launch_bounds__(kBlock) void kb_load(int n, const int* __restrict__ iperm,
                                                  const double* const* __restrict__ src, double* __restrict__ B,
                                                  double* __restrict__ R, float* __restrict__ R32,
                                                  double* __restrict__ X, double* __restrict__ partial) {
    constexpr int GPB = kBlock / kW;
    __shared__ double s_bb[GPB][kW];
    const int g = threadIdx.x / kW, lane = threadIdx.x % kW;
    const double* sc = src[lane];
    double bb = 0.0;
    const int stride = gridDim.x * GPB;
    for (int i = blockIdx.x * GPB + g; i < n; i += stride) {
        const size_t e = (size_t)i * kW + lane;
        if (sc) {
            const double v = sc[iperm[i]];
            B[e] = v;
            R[e] = v;
            if (R32) R32[e] = (float)v;
            X[e] = 0.0;
            bb += v * v;
        }
    }
    s_bb[g][lane] = bb;
    __syncthreads();
    if (threadIdx.x < kW) {
        double t = 0.0;
        for (int q = 0; q < GPB; ++q) t += s_bb[q][threadIdx.x];
        partial[(size_t)blockIdx.x * kW + threadIdx.x] = t;
    }
}

// Store columns (dst[c] != nullptr): dst_c[i] = X[perm[i], c] (caller order);
// a column whose right-hand side was zero gets x = 0.
static __global__ __launch_bounds__(kBlock) void kb_store(int n, const int* __restrict__ perm, double* const* __restrict__ dst,
                                                   const double* __restrict__ X, const BatchState* __restrict__ st) {
    constexpr int GPB = kBlock / kW;
    const int g = threadIdx.x / kW, lane = threadIdx.x % kW;
    double* dc = dst[lane];
    if (!dc) return;
    const bool zero = st->col[lane].done == 2;
    const int stride = gridDim.x * GPB;
    for (int i = blockIdx.x * GPB + g; i < n; i += stride) dc[i] = zero ? 0.0 : X[(size_t)perm[i] * kW + lane];
}

// Y = B - A X (all columns) and per-column partials of y.y; with `commit`
// set, columns in `mask` also take Y as their recurrence residual R.
static __global__ __launch_bounds__(kBlock) void kb_resid(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ av, const double* __restrict__ X,
                                                   const double* __restrict__ B, double* __restrict__ Y,
                                                   double* __restrict__ R, float* __restrict__ R32, int mask,
                                                   double* __restrict__ partial) {
    constexpr int GPB = kBlock / kW;
    __shared__ double s_yy[GPB][kW];
    const int g = threadIdx.x / kW, lane = threadIdx.x % kW;
    const TileWalk w = unit_walk(n, GPB, g);
    double yy = 0.0;
    const bool commit = R != nullptr && ((mask >> lane) & 1);
    for (int i = w.first; i < w.end; i += w.stride) {
        double s[1] = {0.0};
        row_accumulate<4, 1, double, double>(rp[i], rp[i + 1], ci, av, X, lane, s);
        const size_t e = (size_t)i * kW + lane;
        const double y = B[e] - s[0];
        Y[e] = y;
        if (commit) {
            R[e] = y;
            if (R32) R32[e] = (float)y;
        }
        yy += y * y;
    }
    s_yy[g][lane] = yy;
    __syncthreads();
    if (threadIdx.x < kW) {
        double t = 0.0;
        for (int q = 0; q < GPB; ++q) t += s_yy[q][threadIdx.x];
        partial[(size_t)blockIdx.x * kW + threadIdx.x] = t;
    }
}

// 16 caller vectors (column c at src + c*n, canonical order) into the
// hierarchical n x 16 layout, and back.
template <typename D>
static __global__ __launch_bounds__(kBlock) void kb_cols_in(int n, const int* __restrict__ iperm,
                                                            const double* __restrict__ src, D* __restrict__ dst) {
    const long long total = (long long)n * kW;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
        const int i = (int)(e / kW), c = (int)(e % kW);
        dst[e] = (D)src[(size_t)c * n + iperm[i]];
    }
}

template <typename S>
static __global__ __launch_bounds__(kBlock) void kb_cols_out(int n, const int* __restrict__ perm,
                                                             const S* __restrict__ src, double* __restrict__ dst) {
    const long long total = (long long)n * kW;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
        const int c = (int)(e / n), i = (int)(e % n);
        dst[e] = (double)src[(size_t)perm[i] * kW + c];
    }
}

// Gather a level's n x 16 block from canonical into hierarchical order (and back).
template <typename S, typename D>
static __global__ __launch_bounds__(kBlock) void kb_permute(int n, const int* __restrict__ idx, const S* __restrict__ src,
                                                     D* __restrict__ dst) {
    const long long total = (long long)n * kW;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
        const int i = (int)(e / kW), c = (int)(e % kW);
        dst[e] = (D)src[(size_t)idx[i] * kW + c];
    }
}

}  // namespace pamg
