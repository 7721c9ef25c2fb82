// Device kernels of the solve phase (gfx950, wave64).
//
// Storage: every level is CSR in hierarchical order, in which the members of
// each aggregate are adjacent rows (the tentative prolongator of
// eq. (prolongator) then maps the contiguous rows aggptr[I]..aggptr[I+1]-1
// to coarse row I).  Tiles are row ranges (or aggregate ranges) whose
// entries fit one tile; one workgroup streams a tile's col/val arrays once,
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

// zp = d r + p z (pre-smoothed value plus prolongated correction) with an
// explicit fused multiply-add: the product d r is rounded, p z is fused.
// Spelled out so that every kernel variant rounds it identically.
template <typename T>
__device__ __forceinline__ T prolong_value(T d, T r, T p, T z) {
    const T dr = d * r;
    return fma(p, z, dr);
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

// Tile descriptors (precomputed on the host, one 16-byte load per tile):
//   row tile          {k0, k1, r0, r1}: entries [k0, k1) of rows [r0, r1)
//   restriction tile  {k0, k1, c0, c1}: entries [k0, k1) of the fine rows that
//                     are the members of coarse rows [c0, c1)
// A tile holds at most ITEMS*kBlock entries (ITEMS chosen per level so that
// small levels still spread over all CUs), except a single row / aggregate
// longer than that, which takes the block-reduction path.
//
// Phase 1 of every tile kernel issues all of a thread's col/val loads at once
// (indices clamped into the tile, so there is no branch between the loads),
// then the gathers, then writes the products to LDS; the per-row data each
// thread needs in phase 2 is loaded in the same batch.

// The tile kernels keep four workgroups per CU (the LDS of the largest FP64
// tiles allows four): __launch_bounds__(kBlock, 4) holds them to 128 VGPRs,
// i.e. four waves per SIMD.

// Streamed matrix arrays are read exactly once per pass: non-temporal loads
// keep them from evicting the gathered vectors from L2.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

template <int ITEMS>
__device__ __forceinline__ void tile_slots(int k0, int k1, int (&kk)[ITEMS]) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int k = k0 + it * kBlock + (int)threadIdx.x;
        kk[it] = k < k1 ? k : k1 - 1;
    }
}

// Column dictionary of a tile (span = first entry in ucol, length): the
// distinct columns of its entries, ascending.  The vector values at those
// columns are gathered once per tile into LDS (s_x), so each distinct column
// is fetched once and neighbouring lanes read neighbouring addresses; every
// entry then reads its value from LDS through its 16-bit dictionary position.
//
// A workgroup walks its tiles one ahead: the next tile's descriptor and
// dictionary span are loaded when a tile starts, and its dictionary columns
// once the tile's own matrix loads are in flight, so that the first
// dependent step of a tile is the gather of its dictionary values (instead
// of descriptor, then columns, then values, each waiting on the one before).
constexpr int kDictSlots = 8;   // a dictionary holds at most kDictSlots * kBlock columns
static_assert(kDictMaxLarge <= kDictSlots * kBlock, "dictionary longer than the prefetch slots");
static_assert(kDictItems <= kDictSlots, "dictionary tiles of kDictItems * kBlock entries must fit the slots");

struct TileNext {
    int4 d;                  // descriptor of the next tile
    int2 sp;                 // its dictionary span
    int c[kDictSlots];       // its dictionary columns: slot s holds column s * kBlock + thread
};

__device__ __forceinline__ void next_desc(TileNext& N, int t, const int4* __restrict__ tiles,
                                          const int2* __restrict__ span, bool dict) {
    N.d = tiles[t];
    N.sp = dict ? span[t] : make_int2(0, 0);
}

__device__ __forceinline__ void next_cols(TileNext& N, const int* __restrict__ ucol) {
#pragma unroll
    for (int s = 0; s < kDictSlots; ++s) {
        const int j = s * kBlock + (int)threadIdx.x;
        if (s * kBlock < N.sp.y) N.c[s] = ucol[N.sp.x + (j < N.sp.y ? j : N.sp.y - 1)];
    }
}

// The dictionary values of a tile (span sp, columns c) gathered into s_x.
template <typename T, class G>
__device__ __forceinline__ void tile_dict_gather(int2 sp, const int (&c)[kDictSlots], T* s_x, G gather) {
    T x[kDictSlots];
#pragma unroll
    for (int s = 0; s < kDictSlots; ++s)
        if (s * kBlock < sp.y) x[s] = gather(c[s]);
#pragma unroll
    for (int s = 0; s < kDictSlots; ++s) {
        const int j = s * kBlock + (int)threadIdx.x;
        if (s * kBlock < sp.y && j < sp.y) s_x[j] = x[s];
    }
}

// Tiles of at least 2048 entries (the large levels) use the dictionary; the
// small tiles of the small levels, where one more dependent load per tile
// costs more than it saves, gather per entry.
template <int ITEMS>
constexpr bool tile_uses_dict() { return ITEMS >= kDictItems; }

template <int ITEMS, typename T, class G>
__device__ __forceinline__ void tile_direct(const int* __restrict__ ci, const int (&kk)[ITEMS], T (&x)[ITEMS],
                                            G gather) {
    int c[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) c[it] = ld_stream(&ci[kk[it]]);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) x[it] = gather(c[it]);
}

template <int ITEMS, typename T>
__device__ __forceinline__ void tile_store(int k0, int k1, const T (&a)[ITEMS], const T (&x)[ITEMS], T* s_prod) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int k = k0 + it * kBlock + (int)threadIdx.x;
        if (k < k1) s_prod[k - k0] = a[it] * x[it];
    }
}

template <int ITEMS>
__device__ __forceinline__ void tile_local(const uint16_t* __restrict__ loc, const int (&kk)[ITEMS],
                                           uint16_t (&li)[ITEMS]) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) li[it] = ld_stream(&loc[kk[it]]);
}

// Dictionary tiles: the products a_k x_c(k) are formed in registers (a is
// overwritten), then, after a barrier that ends every read of the
// dictionary values, stored over them: the products and the dictionary share
// one LDS buffer of max(ITEMS * kBlock, dictionary length) values, which
// keeps four workgroups of the largest tiles resident per CU.
template <int ITEMS, typename T>
__device__ __forceinline__ void tile_products_dict(T (&a)[ITEMS], const uint16_t (&li)[ITEMS], const T* s_x) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) a[it] = a[it] * s_x[li[it]];
}

template <int ITEMS, typename T>
__device__ __forceinline__ void tile_store_prod(int k0, int k1, const T (&prod)[ITEMS], T* s_prod) {
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int k = k0 + it * kBlock + (int)threadIdx.x;
        if (k < k1) s_prod[k - k0] = prod[it];
    }
}

// Dynamic LDS bytes of a tile kernel launch: the dictionary values (dmax of
// the level), which dictionary tiles also use for their products.
template <int ITEMS, typename T>
inline size_t tile_lds_bytes(int dmax) {
    const int n = tile_uses_dict<ITEMS>() ? (dmax > ITEMS * kBlock ? dmax : ITEMS * kBlock) : dmax;
    return (size_t)n * sizeof(T);
}

// Products array of a tile kernel: the dynamic buffer for dictionary tiles,
// a static one (sized ITEMS * kBlock) otherwise.
#define PAMG_TILE_LDS(T, ITEMS)                                                                  \
    __shared__ T s_prod_static[tile_uses_dict<ITEMS>() ? 1 : ITEMS * kBlock];                   \
    extern __shared__ __align__(16) unsigned char s_dyn[];                                       \
    T* s_x = reinterpret_cast<T*>(s_dyn);                                                        \
    T* s_prod = tile_uses_dict<ITEMS>() ? s_x : s_prod_static;

// ----------------------------------------------------------------------------
// Down-sweep at level l (pre-smooth from zero, residual, restriction):
//   z = D^-1 r;  t = r - A z = r - (A D^-1) r;  rc[I] = sum_{i in G_I} p_i t_i
// `ad` holds the column-scaled values a_ij / d_j, so one gather of r suffices
// (g = r).  With another smoother the same pass takes the smoothed z as g and
// the plain values as `ad`: rc[I] = sum_{i in G_I} p_i (r_i - (A z)_i).
template <int ITEMS, typename T, typename RT, typename GT>
static __global__ __launch_bounds__(kBlock, 4) void k_down(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ ad,
    const RT* __restrict__ r, const GT* __restrict__ g, const T* __restrict__ p, const int* __restrict__ aggptr,
    const int4* __restrict__ tiles, int ntiles,
    const int2* __restrict__ span, const int* __restrict__ ucol, const uint16_t* __restrict__ loc, T* __restrict__ rc, const int* __restrict__ done) {
    if (*done) return;
    PAMG_TILE_LDS(T, ITEMS)
    __shared__ T s_u[kBlock];
    __shared__ T s_red[kBlock / 64];
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    constexpr bool DICT = tile_uses_dict<ITEMS>();
    TileNext nx;
    if (w.first < w.end) {
        next_desc(nx, w.first, tiles, span, DICT);
        if constexpr (DICT) next_cols(nx, ucol);
    }
    for (int t = w.first; t < w.end; t += w.stride) {
        const int4 d = nx.d;
        const int2 sp = nx.sp;
        int cc[kDictSlots];
#pragma unroll
        for (int q = 0; q < kDictSlots; ++q) cc[q] = nx.c[q];
        const bool more = t + w.stride < w.end;
        if (more) next_desc(nx, t + w.stride, tiles, span, DICT);
        const int k0 = d.x, k1 = d.y, c0 = d.z, c1 = d.w;
        if (k1 - k0 <= ITEMS * kBlock) {
            int kk[ITEMS];
            T a[ITEMS];
            uint16_t li[ITEMS];
            tile_slots<ITEMS>(k0, k1, kk);
            const auto gather = [&](int c) { return (T)g[c]; };
            T x[ITEMS];
            if constexpr (tile_uses_dict<ITEMS>()) {
                tile_dict_gather<T>(sp, cc, s_x, gather);
                tile_local<ITEMS>(loc, kk, li);
            } else {
                tile_direct<ITEMS, T>(ci, kk, x, gather);
            }
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) a[it] = ld_stream(&ad[kk[it]]);
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);      // the next tile's columns, behind this tile's loads
            }
            // phase 2: thread j finishes fine row f0 + j (the tile holds at
            // most kBlock fine rows), u_m = p_m (r_m - s_m) into LDS; then
            // thread j sums the members of coarse row c0 + j in order.
            const int f0 = aggptr[c0], f1 = aggptr[c1];
            const int m = f0 + tid;
            const bool fown = m < f1;
            const int mc = fown ? m : f1 - 1;
            const int e0 = rp[mc], e1 = rp[mc + 1];
            const T rm = (T)r[mc], pm = p[mc];
            const int I = c0 + tid;
            const bool own = I < c1;
            const int Ic = own ? I : c1 - 1;
            const int a0 = aggptr[Ic] - f0, a1 = aggptr[Ic + 1] - f0;
            if constexpr (tile_uses_dict<ITEMS>()) {
                __syncthreads();                // dictionary values in LDS
                tile_products_dict<ITEMS>(a, li, s_x);
                __syncthreads();                // dictionary reads done: products take its place
                tile_store_prod<ITEMS>(k0, k1, a, s_prod);
            } else {
                tile_store<ITEMS>(k0, k1, a, x, s_prod);
            }
            __syncthreads();
            if (fown) {
                T s = 0;
                for (int k = e0 - k0; k < e1 - k0; ++k) s += s_prod[k];
                s_u[tid] = pm * (rm - s);
            }
            __syncthreads();
            if (own) {
                T acc = s_u[a0];
                for (int j = a0 + 1; j < a1; ++j) acc += s_u[j];
                rc[I] = acc;
            }
            // no barrier here: the next tile writes s_x and s_prod (last read
            // before the barrier above) and s_u only after two barriers
        } else {
            // one aggregate whose rows exceed a tile
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);
            }
            const int f0 = aggptr[c0], f1 = aggptr[c1];
            T acc = 0;
            for (int m = f0; m < f1; ++m) {
                T s = 0;
                for (int k = rp[m] + tid; k < rp[m + 1]; k += kBlock) s += ad[k] * (T)g[ci[k]];
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
//   l = 0: write z (as ZO: FP64, or FP32 from the FP32 cycle, which is exact)
//   and accumulate the partial of z . dv.
// MODE: kUpOut (l = 0), kUpPair (aggregates of at most two rows: the row's
// thread writes its members), kUpWide (larger aggregates: z is staged in LDS
// and the tile's fine rows are written one per thread, coalesced).
constexpr int kUpOut = 0, kUpPair = 1, kUpWide = 2;

template <int ITEMS, typename T, typename RT, typename RTF, int MODE, typename ZO = double>
static __global__ __launch_bounds__(kBlock, 4) void k_up(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ zp, const RT* __restrict__ r, const T* __restrict__ dinv,
    const int4* __restrict__ tiles, int ntiles,
    const int2* __restrict__ span, const int* __restrict__ ucol, const uint16_t* __restrict__ loc,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f,
    ZO* __restrict__ z_out, const double* __restrict__ dv, double* __restrict__ partial,
    const int* __restrict__ done) {
    constexpr bool TO_OUT = MODE == kUpOut;
    if (*done) return;
    PAMG_TILE_LDS(T, ITEMS)
    __shared__ T s_red[kBlock / 64];
    __shared__ double s_redd[kBlock / 64];
    __shared__ T s_z[kBlock];                          // kUpWide: z of the tile's rows
    __shared__ uint8_t s_own[kBlock << kMaxAggSteps];  // kUpWide: owning row of each fine row
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    double dot = 0.0;
    constexpr bool DICT = tile_uses_dict<ITEMS>();
    TileNext nx;
    if (w.first < w.end) {
        next_desc(nx, w.first, tiles, span, DICT);
        if constexpr (DICT) next_cols(nx, ucol);
    }
    for (int t = w.first; t < w.end; t += w.stride) {
        const int4 d = nx.d;
        const int2 sp = nx.sp;
        int cc[kDictSlots];
#pragma unroll
        for (int q = 0; q < kDictSlots; ++q) cc[q] = nx.c[q];
        const bool more = t + w.stride < w.end;
        if (more) next_desc(nx, t + w.stride, tiles, span, DICT);
        const int k0 = d.x, k1 = d.y, i0 = d.z, i1 = d.w;
        if (k1 - k0 <= ITEMS * kBlock) {
            int kk[ITEMS];
            T a[ITEMS];
            uint16_t li[ITEMS];
            tile_slots<ITEMS>(k0, k1, kk);
            const auto gather = [&](int c) { return zp[c]; };
            T x[ITEMS];
            if constexpr (tile_uses_dict<ITEMS>()) {
                tile_dict_gather<T>(sp, cc, s_x, gather);
                tile_local<ITEMS>(loc, kk, li);
            } else {
                tile_direct<ITEMS, T>(ci, kk, x, gather);
            }
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) a[it] = ld_stream(&av[kk[it]]);
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);      // the next tile's columns, behind this tile's loads
            }
            const int i = i0 + tid;
            const bool own = i < i1;
            const int ic = own ? i : i1 - 1;
            const int rb = rp[ic], re = rp[ic + 1];
            const T zpi = zp[ic], di = dinv[ic];
            const T ri = (T)r[ic];
            // operands of the prolongation, loaded before the barriers
            int a0 = 0, a1 = 0, F0 = 0, F1 = 0;
            double dvi = 0.0;
            T rf0 = 0, df0 = 0, pf0 = 0, rf1 = 0, df1 = 0, pf1 = 0;
            if constexpr (MODE == kUpOut) {
                dvi = dv[ic];
            } else if constexpr (MODE == kUpPair) {
                a0 = aggptr_f[ic]; a1 = aggptr_f[ic + 1];
                rf0 = (T)r_f[a0]; df0 = dinv_f[a0]; pf0 = p_f[a0];
                if (a1 - a0 >= 2) { rf1 = (T)r_f[a0 + 1]; df1 = dinv_f[a0 + 1]; pf1 = p_f[a0 + 1]; }
            } else {
                // the fine rows F0..F1 of the tile's rows, one per thread
                a0 = aggptr_f[ic]; a1 = aggptr_f[ic + 1];
                F0 = aggptr_f[i0]; F1 = aggptr_f[i1];
                const int m = F0 + tid < F1 ? F0 + tid : F1 - 1;
                rf0 = (T)r_f[m]; df0 = dinv_f[m]; pf0 = p_f[m];
            }
            if constexpr (tile_uses_dict<ITEMS>()) {
                __syncthreads();                // dictionary values in LDS
                tile_products_dict<ITEMS>(a, li, s_x);
                __syncthreads();                // dictionary reads done: products take its place
                tile_store_prod<ITEMS>(k0, k1, a, s_prod);
            } else {
                tile_store<ITEMS>(k0, k1, a, x, s_prod);
            }
            __syncthreads();
            T z = 0;
            if (own) {
                T s = 0;
                for (int k = rb - k0; k < re - k0; ++k) s += s_prod[k];
                z = zpi + di * (ri - s);
            }
            if constexpr (MODE == kUpOut) {
                if (own) {
                    z_out[i] = (ZO)z;
                    dot += (double)z * dvi;
                }
                __syncthreads();
            } else if constexpr (MODE == kUpPair) {
                if (own) {
                    zp_f[a0] = prolong_value(df0, rf0, pf0, z);
                    if (a1 - a0 >= 2) zp_f[a0 + 1] = prolong_value(df1, rf1, pf1, z);
                    for (int m = a0 + 2; m < a1; ++m) zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], z);
                }
                __syncthreads();
            } else {
                if (own) {
                    s_z[tid] = z;
                    for (int m = a0; m < a1; ++m) s_own[m - F0] = (uint8_t)tid;
                }
                __syncthreads();
                if (F0 + tid < F1) zp_f[F0 + tid] = prolong_value(df0, rf0, pf0, s_z[s_own[tid]]);
                for (int j = tid + kBlock; j < F1 - F0; j += kBlock) {
                    const int m = F0 + j;
                    zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], s_z[s_own[j]]);
                }
                // no barrier here: the next tile writes s_x and s_prod (last
                // read before the barrier above), s_z and s_own only after
                // its own first barrier
            }
        } else {
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);
            }
            T s = 0;
            for (int k = k0 + tid; k < k1; k += kBlock) s += av[k] * zp[ci[k]];
            s = block_sum(s, s_red);
            if (tid == 0) {
                const T z = zp[i0] + dinv[i0] * ((T)r[i0] - s);
                if constexpr (TO_OUT) {
                    z_out[i0] = (ZO)z;
                    dot += (double)z * dv[i0];
                } else {
                    for (int m = aggptr_f[i0]; m < aggptr_f[i0 + 1]; ++m) zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], z);
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
// Coarsest level: z = A_L^-1 r with the dense symmetric inverse, one
// workgroup of 1024 threads: the columns j are split into G groups whose
// partial sums meet in LDS (fixed order), then each row I prolongates into
// level L-1 as in k_up, or (single-level hierarchy) writes z.
// Dynamic LDS: (1 + G) * nL values, G = 16 (nL <= 256), 4 (nL <= 1024), else 1.
constexpr int kCoarseThreads = 1024;
inline int coarse_groups(int nL) { return nL <= 256 ? 16 : (nL <= 1024 ? 4 : 1); }

template <typename T, typename RT, typename RTF, bool TO_OUT>
static __global__ __launch_bounds__(kCoarseThreads) void k_coarse(
    int nL, int G, const T* __restrict__ ainv, const RT* __restrict__ r,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f,
    double* __restrict__ z_out, const double* __restrict__ dv, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (*done) return;
    extern __shared__ __align__(16) unsigned char s_raw[];
    T* s_r = reinterpret_cast<T*>(s_raw);
    T* s_part = s_r + nL;
    __shared__ double s_redd[kCoarseThreads / 64];
    const int tid = threadIdx.x;
    for (int i = tid; i < nL; i += kCoarseThreads) s_r[i] = (T)r[i];
    __syncthreads();
    const int per = kCoarseThreads / G;          // threads per column group
    const int g = tid / per, lt = tid % per;
    const int j0 = (int)((long long)nL * g / G), j1 = (int)((long long)nL * (g + 1) / G);
    for (int I = lt; I < nL; I += per) {
        T s = 0;
        for (int j = j0; j < j1; ++j) s += ainv[(size_t)j * nL + I] * s_r[j];
        s_part[(size_t)g * nL + I] = s;
    }
    __syncthreads();
    double dot = 0.0;
    for (int I = tid; I < nL; I += kCoarseThreads) {
        T z = 0;
        for (int q = 0; q < G; ++q) z += s_part[(size_t)q * nL + I];
        if constexpr (TO_OUT) {
            z_out[I] = (double)z;
            dot += (double)z * dv[I];
        } else {
            for (int m = aggptr_f[I]; m < aggptr_f[I + 1]; ++m) zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], z);
        }
    }
    if constexpr (TO_OUT) {
        dot = wave_sum(dot);
        if ((tid & 63) == 0) s_redd[tid >> 6] = dot;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int q = 0; q < kCoarseThreads / 64; ++q) t += s_redd[q];
            partial[0] = t;
        }
    }
}

// ----------------------------------------------------------------------------
// Coarsest level when it is large (a stalled coarsening can leave thousands of
// rows): the same product and prolongation as k_coarse, one wave per row.  The
// inverse is symmetric, so row I is read along its length (coalesced, 64
// consecutive columns per load) and the lanes' partial sums meet in a wave
// butterfly (fixed order); ceil(nL / 4) workgroups of four waves, so even a
// coarsest level of a few thousand rows spreads over the whole chip.
constexpr int kCoarseRowsMin = 512;          // above this size the coarsest runs on many workgroups
constexpr int kCoarseRowsPerBlock = kBlock / 64;
inline int coarse_rows_grid(int nL) { return (nL + kCoarseRowsPerBlock - 1) / kCoarseRowsPerBlock; }

template <typename T, typename RT, typename RTF, bool TO_OUT>
static __global__ __launch_bounds__(kBlock) void k_coarse_rows(
    int nL, const T* __restrict__ ainv, const RT* __restrict__ r,
    const int* __restrict__ aggptr_f, const RTF* __restrict__ r_f, const T* __restrict__ dinv_f,
    const T* __restrict__ p_f, T* __restrict__ zp_f,
    double* __restrict__ z_out, const double* __restrict__ dv, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (*done) return;
    __shared__ double s_dot[kCoarseRowsPerBlock];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int I = blockIdx.x * kCoarseRowsPerBlock + wave;
    T s = 0;
    if (I < nL) {
        const T* __restrict__ row = ainv + (size_t)I * nL;
#pragma unroll 4
        for (int j = lane; j < nL; j += 64) s += row[j] * (T)r[j];
    }
    const T z = wave_sum(s);
    double dot = 0.0;
    if (I < nL) {
        if constexpr (TO_OUT) {
            if (lane == 0) {
                z_out[I] = (double)z;
                dot = (double)z * dv[I];
            }
        } else {
            for (int m = aggptr_f[I] + lane; m < aggptr_f[I + 1]; m += 64)
                zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], z);
        }
    }
    if constexpr (TO_OUT) {
        if (lane == 0) s_dot[wave] = dot;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int q = 0; q < kCoarseRowsPerBlock; ++q) t += s_dot[q];
            partial[blockIdx.x] = t;
        }
    }
}

// ----------------------------------------------------------------------------
// Prolongation alone (parity checks): zp_f[m] = dinv_f[m] r_f[m] + p_f[m] e[I]
// for the members m of every coarse row I.
template <typename T>
static __global__ __launch_bounds__(kBlock) void k_prolong(int nc, const T* __restrict__ e, const int* __restrict__ aggptr,
                                                    const double* __restrict__ r_f, const T* __restrict__ dinv_f,
                                                    const T* __restrict__ p_f, T* __restrict__ zp_f) {
    const int stride = gridDim.x * kBlock;
    for (int I = blockIdx.x * kBlock + threadIdx.x; I < nc; I += stride) {
        const T z = e[I];
        for (int m = aggptr[I]; m < aggptr[I + 1]; ++m) zp_f[m] = prolong_value(dinv_f[m], (T)r_f[m], p_f[m], z);
    }
}

// ----------------------------------------------------------------------------
// y = A x  (or y = b - A x when b != nullptr), row tiles; optional partial of
// y . y.  Other epilogues (no partial), d = dscale: kSpmvProlong
// y_i = d_i b_i + (A x)_i (the smoothed prolongation D^-1 r + P e);
// kSpmvSmooth y_i = x_i + d_i t_i with t = b - A x rounded to T (an
// l1-Jacobi step from x); kSpmvAdd y_i = b_i + (A x)_i (a correction
// z + P e added to the smoothed iterate).  done
// (optional): the solve's converged flag.
constexpr int kSpmvPlain = 0, kSpmvProlong = 1, kSpmvSmooth = 2, kSpmvAdd = 3;

template <int ITEMS, typename T, typename XT, typename YT, typename BT = double, int EPI = kSpmvPlain>
static __global__ __launch_bounds__(kBlock, 4) void k_spmv(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const XT* __restrict__ xv, const BT* __restrict__ b, const T* __restrict__ dscale, YT* __restrict__ y,
    const int4* __restrict__ tiles, int ntiles,
    const int2* __restrict__ span, const int* __restrict__ ucol, const uint16_t* __restrict__ loc, double* __restrict__ partial,
    const int* __restrict__ done) {
    if (done && *done) return;
    PAMG_TILE_LDS(T, ITEMS)
    __shared__ T s_red[kBlock / 64];
    __shared__ double s_redd[kBlock / 64];
    const int tid = threadIdx.x;
    const TileWalk w = tile_walk(ntiles);
    double nrm = 0.0;
    constexpr bool DICT = tile_uses_dict<ITEMS>();
    TileNext nx;
    if (w.first < w.end) {
        next_desc(nx, w.first, tiles, span, DICT);
        if constexpr (DICT) next_cols(nx, ucol);
    }
    for (int t = w.first; t < w.end; t += w.stride) {
        const int4 d = nx.d;
        const int2 sp = nx.sp;
        int cc[kDictSlots];
#pragma unroll
        for (int q = 0; q < kDictSlots; ++q) cc[q] = nx.c[q];
        const bool more = t + w.stride < w.end;
        if (more) next_desc(nx, t + w.stride, tiles, span, DICT);
        const int k0 = d.x, k1 = d.y, i0 = d.z, i1 = d.w;
        if (k1 - k0 <= ITEMS * kBlock) {
            int kk[ITEMS];
            T a[ITEMS];
            uint16_t li[ITEMS];
            tile_slots<ITEMS>(k0, k1, kk);
            const auto gather = [&](int c) { return (T)xv[c]; };
            T x[ITEMS];
            if constexpr (tile_uses_dict<ITEMS>()) {
                tile_dict_gather<T>(sp, cc, s_x, gather);
                tile_local<ITEMS>(loc, kk, li);
            } else {
                tile_direct<ITEMS, T>(ci, kk, x, gather);
            }
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) a[it] = ld_stream(&av[kk[it]]);
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);      // the next tile's columns, behind this tile's loads
            }
            // phase 2: G lanes per row (G = 1 unless the tile has few, long
            // rows), each summing a strided part, then a fixed-order butterfly
            int G = 1;
            while (G < 64 && 2 * G * (i1 - i0) <= kBlock) G *= 2;
            const int lane = tid & (G - 1);
            const int i = i0 + tid / G;
            const bool own = i < i1;
            const int ic = own ? i : i1 - 1;
            const int rb = rp[ic], re = rp[ic + 1];
            const double bi = b ? (double)b[ic] : 0.0;
            const T di = (EPI == kSpmvProlong || EPI == kSpmvSmooth) ? dscale[ic] : T(0);
            const T xi = EPI == kSpmvSmooth ? (T)xv[ic] : T(0);
            if constexpr (tile_uses_dict<ITEMS>()) {
                __syncthreads();                // dictionary values in LDS
                tile_products_dict<ITEMS>(a, li, s_x);
                __syncthreads();                // dictionary reads done: products take its place
                tile_store_prod<ITEMS>(k0, k1, a, s_prod);
            } else {
                tile_store<ITEMS>(k0, k1, a, x, s_prod);
            }
            __syncthreads();
            T s = 0;
            if (own)
                for (int k = rb - k0 + lane; k < re - k0; k += G) s += s_prod[k];
            for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
            if (own && lane == 0) {
                if constexpr (EPI == kSpmvProlong) {
                    y[i] = (YT)(di * (T)bi + s);
                } else if constexpr (EPI == kSpmvAdd) {
                    y[i] = (YT)((T)bi + s);
                } else if constexpr (EPI == kSpmvSmooth) {
                    const T t = (T)(bi - (double)s);
                    y[i] = (YT)(xi + di * t);
                } else {
                    const double v = b ? bi - (double)s : (double)s;
                    y[i] = (YT)v;
                    nrm += v * v;
                }
            }
            __syncthreads();
        } else {
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);
            }
            T s = 0;
            for (int k = k0 + tid; k < k1; k += kBlock) s += av[k] * (T)xv[ci[k]];
            s = block_sum(s, s_red);
            if (tid == 0) {
                if constexpr (EPI == kSpmvProlong) {
                    y[i0] = (YT)(dscale[i0] * (T)b[i0] + s);
                } else if constexpr (EPI == kSpmvAdd) {
                    y[i0] = (YT)((T)b[i0] + s);
                } else if constexpr (EPI == kSpmvSmooth) {
                    const T t = (T)((double)b[i0] - (double)s);
                    y[i0] = (YT)((T)xv[i0] + dscale[i0] * t);
                } else {
                    const double v = b ? (double)b[i0] - (double)s : (double)s;
                    y[i0] = (YT)v;
                    nrm += v * v;
                }
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
// q = A p computed as A z + beta q_old (the same vector in exact arithmetic,
// so that only z is gathered: one dictionary gather per tile instead of two;
// q holds q_old on entry and each row's element is read before its owner
// overwrites it), partials of p.q and p.r.  On the first iteration (and after
// a restart) q = A z.  z is FP64, or FP32 when it comes from the FP32 cycle
// (whose z values are FP32 numbers: the same sums, half the gathered bytes).
template <int ITEMS, typename ZT = double>
static __global__ __launch_bounds__(kBlock, 4) void k_krylov_pq(
    const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ av,
    const ZT* __restrict__ z, const double* __restrict__ p_old, double* __restrict__ p_new,
    double* __restrict__ q, const double* __restrict__ r,
    const int4* __restrict__ tiles, int ntiles,
    const int2* __restrict__ span, const int* __restrict__ ucol, const uint16_t* __restrict__ loc,
    const SolveState* __restrict__ st, double* __restrict__ partial, const int* __restrict__ done) {
    if (*done) return;
    PAMG_TILE_LDS(double, ITEMS)
    __shared__ double s_red[kBlock / 64];
    const int tid = threadIdx.x;
    const bool first = st->first != 0;
    const double beta = st->beta;
    const TileWalk w = tile_walk(ntiles);
    double pq = 0.0, pr = 0.0;
    constexpr bool DICT = tile_uses_dict<ITEMS>();
    TileNext nx;
    if (w.first < w.end) {
        next_desc(nx, w.first, tiles, span, DICT);
        if constexpr (DICT) next_cols(nx, ucol);
    }
    for (int t = w.first; t < w.end; t += w.stride) {
        const int4 d = nx.d;
        const int2 sp = nx.sp;
        int cc[kDictSlots];
#pragma unroll
        for (int q = 0; q < kDictSlots; ++q) cc[q] = nx.c[q];
        const bool more = t + w.stride < w.end;
        if (more) next_desc(nx, t + w.stride, tiles, span, DICT);
        const int k0 = d.x, k1 = d.y, i0 = d.z, i1 = d.w;
        if (k1 - k0 <= ITEMS * kBlock) {
            int kk[ITEMS];
            double a[ITEMS];
            uint16_t li[ITEMS];
            tile_slots<ITEMS>(k0, k1, kk);
            const auto gather = [&](int c) { return (double)z[c]; };
            double x[ITEMS];
            if constexpr (tile_uses_dict<ITEMS>()) {
                tile_dict_gather<double>(sp, cc, s_x, gather);
                tile_local<ITEMS>(loc, kk, li);
            } else {
                tile_direct<ITEMS, double>(ci, kk, x, gather);
            }
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) a[it] = ld_stream(&av[kk[it]]);
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);      // the next tile's columns, behind this tile's loads
            }
            const int i = i0 + tid;
            const bool own = i < i1;
            const int ic = own ? i : i1 - 1;
            const int rb = rp[ic], re = rp[ic + 1];
            const double zi = (double)z[ic], poi = p_old[ic], ri = r[ic], qoi = q[ic];
            if constexpr (tile_uses_dict<ITEMS>()) {
                __syncthreads();                // dictionary values in LDS
                tile_products_dict<ITEMS>(a, li, s_x);
                __syncthreads();                // dictionary reads done: products take its place
                tile_store_prod<ITEMS>(k0, k1, a, s_prod);
            } else {
                tile_store<ITEMS>(k0, k1, a, x, s_prod);
            }
            __syncthreads();
            if (own) {
                double s = 0.0;
                for (int k = rb - k0; k < re - k0; ++k) s += s_prod[k];
                const double pi = first ? zi : zi + beta * poi;
                const double qi = first ? s : s + beta * qoi;
                p_new[i] = pi;
                q[i] = qi;
                pq += pi * qi;
                pr += pi * ri;
            }
            __syncthreads();
        } else {
            if constexpr (DICT) {
                if (more) next_cols(nx, ucol);
            }
            double s = 0.0;
            for (int k = k0 + tid; k < k1; k += kBlock) s += av[k] * (double)z[ci[k]];
            s = block_sum(s, s_red);
            if (tid == 0) {
                const double pi = first ? (double)z[i0] : (double)z[i0] + beta * p_old[i0];
                s = first ? s : s + beta * q[i0];
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
static __global__ __launch_bounds__(kBlock) void k_krylov_update(
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
static __global__ __launch_bounds__(kBlock) void k_fin_beta(SolveState* __restrict__ st, const double* __restrict__ partial,
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
static __global__ __launch_bounds__(kBlock) void k_fin_alpha(SolveState* __restrict__ st, const double* __restrict__ partial,
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
static __global__ __launch_bounds__(kBlock) void k_fin_norm(SolveState* __restrict__ st, const double* __restrict__ partial,
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
static __global__ __launch_bounds__(kBlock) void k_fin_init(SolveState* __restrict__ st, const double* __restrict__ bb_part,
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
static __global__ __launch_bounds__(kBlock) void k_gather(int n, const int* __restrict__ idx, const S* __restrict__ src,
                                                   D* __restrict__ dst) {
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = (D)src[idx[i]];
}

template <typename S, typename D>
static __global__ __launch_bounds__(kBlock) void k_convert(long long n, const S* __restrict__ src, D* __restrict__ dst) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = (D)src[i];
}

// b.b partials, and optionally r = b (x0 = 0) with r.r partials equal to b.b
static __global__ __launch_bounds__(kBlock) void k_norm2(int n, const double* __restrict__ b, double* __restrict__ copy_to,
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

static __global__ __launch_bounds__(kBlock) void k_fill(long long n, double* __restrict__ x, double v) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = v;
}

}  // namespace pamg
