// Device construction of the large levels of the AMG hierarchy (arXiv
// 2210.16660, Sec. 3.1), bitwise the host construction (setup.cpp):
//   * l1 diagonal, edge weights of eq. (weights) and the eligibility c > 1;
//   * the matching: locally dominant edges in parallel rounds (every alive
//     vertex points at its heaviest eligible unmatched neighbour under the
//     strict order (c desc, lo asc, hi asc); mutual pointers are matched; a
//     vertex without such a neighbour stays single).  For a strict total order
//     on the edges this is the greedy matching, the one the host's Suitor
//     algorithm computes and eq. (approximatematch) approximates;
//   * aggregates numbered by smallest member and the tentative prolongator of
//     eq. (prolongator);
//   * the Galerkin product with every coarse entry summed in the canonical
//     order (ascending (min(i,j), max(i,j), i)), one wavefront per coarse row;
//   * with aggregate-size composition (agg_steps = s > 1), every s-th
//     pairwise level kept, its aggregates and prolongator entries composed
//     over the s pairwise steps (p multiplied finest first);
//   * the hierarchical numbering, the permuted rows (columns ascending), the
//     column-scaled values and the tiles' column dictionaries.
// A level is built here while it is large (more rows than the dense limit,
// the coarsening limit and a size floor) and its rows are short (at most
// kRowCap entries); the first level that is not, and every coarser one, is
// built on the host from that level's matrix and near-null vector.
//
// Compiled with -ffp-contract=off: each written floating-point operation is
// one IEEE binary64 operation (division and square root correctly rounded),
// as on the host.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <numeric>

#include "dsetup.hpp"

namespace pamg {
namespace {

constexpr int kSB = 256;                 // threads of the elementwise and scan kernels
constexpr int kScanItems = 8;
constexpr int kScanTile = kSB * kScanItems;
constexpr int kRowCap = 256;             // longest row of a level built on the device
constexpr int kTermCap = 2 * kRowCap;    // Galerkin terms of one coarse row (two members)
constexpr int kRunCap = 4;               // terms of one coarse entry (2 x 2 members)
constexpr int kDictCap = kMaxItems * kBlock;   // entries of the largest tile
constexpr int kGridCap = 1 << 20;        // workgroups of the grid-stride kernels

inline int grid_for(long long n, int per) {
    long long g = (n + per - 1) / per;
    return (int)std::max<long long>(1, std::min<long long>(g, kGridCap));
}

// Device temporaries of one build (freed when it ends).
struct Temps {
    pamg_context* ctx;
    hipStream_t s;
    std::vector<DevAlloc> list;
    template <typename T>
    T* get(size_t count) {
        const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
        void* p = ctx_alloc(ctx, bytes, s);
        list.push_back({p, bytes});
        return static_cast<T*>(p);
    }
    void release(void* p) {
        for (size_t i = 0; i < list.size(); ++i)
            if (list[i].p == p) {
                HIP_CHECK(hipStreamSynchronize(s));
                ctx_free(ctx, p, list[i].bytes, s);
                list.erase(list.begin() + i);
                return;
            }
    }
    ~Temps() {
        (void)hipStreamSynchronize(s);
        ctx_free_all(ctx, list);
    }
};

template <typename T>
T read1(const T* d, hipStream_t s) {
    T x;
    HIP_CHECK(hipMemcpyAsync(&x, d, sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return x;
}

template <typename T>
void to_host(std::vector<T>& out, const T* d, size_t count, hipStream_t s) {
    out.resize(count);
    if (count) HIP_CHECK(hipMemcpyAsync(out.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

template <typename T>
void to_device(T* d, const T* src, size_t count, hipStream_t s) {
    if (count) HIP_CHECK(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

#define GRID_STRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
                               i += (long long)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ scans

// Exclusive prefix sums of in[0..n) into out[0..n] (out[n] = total); each
// workgroup scans kScanTile elements and leaves its total in blk.
template <typename TIn>
__global__ __launch_bounds__(kSB) void k_scan_local(long long n, const TIn* in, long long* out, long long* blk) {
    __shared__ long long s[kSB];
    const long long i0 = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    long long loc[kScanItems];
    long long sum = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const long long i = i0 + u;
        loc[u] = sum;
        sum += (i < n) ? (long long)in[i] : 0;
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kSB; off <<= 1) {
        const long long t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    const long long excl = s[threadIdx.x] - sum;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const long long i = i0 + u;
        if (i <= n) out[i] = excl + loc[u];
    }
    if (threadIdx.x == kSB - 1) blk[blockIdx.x] = s[kSB - 1];
}

__global__ void k_scan_add(long long n, long long* out, const long long* off) {
    GRID_STRIDE(i, n + 1) out[i] += off[i / kScanTile];
}

// out[0..n]: exclusive sums of in[0..n), out[n] the total (returned).
template <typename TIn>
long long scan(Temps& T, long long n, const TIn* in, long long* out, hipStream_t s) {
    const long long nb = (n + 1 + kScanTile - 1) / kScanTile;
    long long* blk = T.get<long long>(nb + 1);
    hipLaunchKernelGGL(k_scan_local<TIn>, dim3((unsigned)nb), dim3(kSB), 0, s, n, in, out, blk);
    if (nb > 1) {
        long long* off = T.get<long long>(nb + 1);
        scan<long long>(T, nb, blk, off, s);
        hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n + 1, kSB)), dim3(kSB), 0, s, n, out, (const long long*)off);
        T.release(off);
    }
    T.release(blk);
    return read1(out + n, s);
}

__global__ void k_to_int(long long n, const long long* in, int* out) { GRID_STRIDE(i, n) out[i] = (int)in[i]; }

__global__ void k_fill_d(long long n, double* x, double v) { GRID_STRIDE(i, n) x[i] = v; }

// ---------------------------------------------------------- level kernels

// d_i = sum_j |a_ij| (ascending columns), a_ii, dinv = 1/d; the longest row.
__global__ void k_l1diag(int n, const int* rp, const int* ci, const double* v, double* dinv, double* diag,
                         int* maxrow) {
    int mx = 0;
    GRID_STRIDE(i, n) {
        double d = 0.0, dg = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            d += fabs(v[k]);
            if (ci[k] == i) dg = v[k];
        }
        dinv[i] = 1.0 / d;
        diag[i] = dg;
        mx = max(mx, rp[i + 1] - rp[i]);
    }
    atomicMax(maxrow, mx);
}

// validate_csr's row checks, one thread per row, in the same order (no
// entry of a row whose bounds are out of order is read): the smallest
// failing row and its check, as (row << 8) | check.
__global__ void k_validate(int n, long long nnz, const int* rp, const int* ci, const double* v,
                           unsigned long long* first) {
    GRID_STRIDE(i, n) {
        const int b = rp[i], e = rp[i + 1];
        int err = 0;
        if (e < b || b < 0 || (long long)e > nnz) err = 1;
        bool diag = false;
        for (int k = b; k < e && !err; ++k) {
            const int c = ci[k];
            if (c < 0 || c >= n) {
                err = 2;
            } else if (k > b && c <= ci[k - 1]) {
                err = 3;
            } else if (c == (int)i) {
                diag = true;
                if (!(v[k] > 0.0)) err = 4;
            }
            if (!isfinite(v[k])) err = 6;
        }
        if (!err && !diag) err = 5;
        if (err) atomicMin(first, ((unsigned long long)i << 8) | (unsigned long long)err);
    }
}

// check_symmetry: every entry has a mirror with the same bits.
__global__ void k_check_symmetry(int n, const int* rp, const int* ci, const double* v, int* asym) {
    GRID_STRIDE(i, n) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            int b = rp[j], e = rp[j + 1];
            while (b < e) {
                const int m = (b + e) >> 1;
                if (ci[m] < (int)i) b = m + 1; else e = m;
            }
            if (b >= rp[j + 1] || ci[b] != (int)i || __double_as_longlong(v[b]) != __double_as_longlong(v[k]))
                atomicOr(asym, 1);
        }
    }
}

__device__ inline double edge_weight(double a_lohi, double a_lolo, double a_hihi, double w_lo, double w_hi) {
    double num = ((2.0 * a_lohi) * w_lo) * w_hi;
    double den = (a_lolo * w_lo) * w_lo + (a_hihi * w_hi) * w_hi;
    return 1.0 - num / den;
}

__device__ inline bool heavier(double c1, int lo1, int hi1, double c2, int lo2, int hi2) {
    if (c1 != c2) return c1 > c2;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

__device__ inline int find_col(const int* ci, int b, int e, int col) {
    while (b < e) {
        const int m = (b + e) >> 1;
        if (ci[m] < col) b = m + 1; else e = m;
    }
    return b;
}

// Weight of every off-diagonal entry from the upper entry (lo, hi) of its
// edge (both directions carry the same value); 0 on the diagonal.  Flags an
// entry whose transposed entry is not stored (the device matching scans rows,
// so the pattern must be symmetric).
__global__ void k_weights(int n, const int* rp, const int* ci, const double* v, const double* diag, const double* w,
                          double* c, int* asym) {
    GRID_STRIDE(i, n) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            if (j == (int)i) {
                c[k] = 0.0;
                continue;
            }
            const int t = find_col(ci, rp[j], rp[j + 1], (int)i);
            if (t >= rp[j + 1] || ci[t] != (int)i) {
                atomicOr(asym, 1);
                c[k] = 0.0;
                continue;
            }
            const int lo = min((int)i, j), hi = max((int)i, j);
            const double a = j > (int)i ? v[k] : v[t];
            c[k] = edge_weight(a, diag[lo], diag[hi], w[lo], w[hi]);
        }
    }
}

// Bitonic sort (ascending) of P (a power of two) keys in LDS by one workgroup.
template <typename K>
__device__ inline void lds_bitonic(K* key, int P) {
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
                const int a = 2 * t - (t & (stride - 1));
                const int b = a + stride;
                const K x = key[a], y = key[b];
                const bool up = (a & size) == 0;
                if ((x > y) == up) {
                    key[a] = y;
                    key[b] = x;
                }
            }
            __syncthreads();
        }
}

constexpr unsigned char kAlive = 0, kMatched = 1, kSingle = 2;

// A neighbour of vertex i in the matching order: heavier first; for equal
// weights the edge with the smaller (lo, hi) first, which for a fixed i is
// the smaller neighbour index.  x > y: x comes after y.
struct Nbr {
    double c;
    int j;
    __device__ bool operator>(const Nbr& y) const { return c < y.c || (c == y.c && j > y.j); }
};

// Every vertex's eligible neighbours (c > 1) in the matching order, at its
// row's positions in adj; their number in ecnt.  One wavefront per row.
__global__ __launch_bounds__(64) void k_sort_adj(int n, const int* rp, const int* ci, const double* c, int* adj,
                                                 int* ecnt) {
    __shared__ Nbr key[kRowCap];
    const int lane = threadIdx.x;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int b = rp[i], len = rp[i + 1] - b;
        int P = 1;
        while (P < len) P <<= 1;
        int cnt = 0;
        for (int t = lane; t < P; t += 64) {
            Nbr x{-1.0, INT_MAX};
            if (t < len) {
                const int j = ci[b + t];
                const double cc = c[b + t];
                if (j != i && cc > 1.0) {
                    x = Nbr{cc, j};
                    ++cnt;
                }
            }
            key[t] = x;
        }
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        __syncthreads();
        lds_bitonic(key, P);
        for (int t = lane; t < cnt; t += 64) adj[b + t] = key[t].j;
        if (lane == 0) ecnt[i] = cnt;
        __syncthreads();
    }
}

// One round, first half: every alive vertex picks its heaviest eligible
// neighbour that is not matched (the first unmatched one in its sorted list;
// matched vertices stay matched, so the cursor only moves forward); none
// left: it stays single.
__global__ void k_pick(int n, const int* rp, const int* ecnt, const int* adj, const int* mate, unsigned char* state,
                       int* cur, int* cand) {
    GRID_STRIDE(i, n) {
        if (state[i] != kAlive) continue;
        int q = cur[i];
        const int e = rp[i] + ecnt[i];
        while (q < e && mate[adj[q]] >= 0) ++q;
        cur[i] = q;
        if (q < e) {
            cand[i] = adj[q];
        } else {
            cand[i] = -1;
            state[i] = kSingle;
        }
    }
}

__global__ void k_cursor(int n, const int* rp, int* cur) { GRID_STRIDE(i, n) cur[i] = rp[i]; }

// Second half: mutual picks are matched.  flag[0] = 1 if a vertex is still
// alive after the round, flag[1] = 1 if a vertex was matched (plain stores of
// 1, one per workgroup that has one; the caller clears them).
constexpr int kCommitGrid = 2048;
__global__ __launch_bounds__(kSB) void k_commit(int n, const int* cand, int* mate, unsigned char* state, int* flag) {
    __shared__ int any[2];
    if (threadIdx.x < 2) any[threadIdx.x] = 0;
    __syncthreads();
    bool alive = false, matched = false;
    GRID_STRIDE(i, n) {
        if (state[i] != kAlive) continue;
        const int j = cand[i];
        if (cand[j] == (int)i) {
            mate[i] = j;
            state[i] = kMatched;
            matched = true;
        } else {
            alive = true;
        }
    }
    if (alive) any[0] = 1;
    if (matched) any[1] = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (any[0]) flag[0] = 1;
        if (any[1]) flag[1] = 1;
    }
}

// Aggregate leaders (smallest member) and aggregate sizes.
__global__ void k_leaders(int n, const int* mate, int* lead, int* size) {
    GRID_STRIDE(i, n) {
        const int m = mate[i];
        const bool l = m < 0 || m > (int)i;
        lead[i] = l ? 1 : 0;
        size[i] = l ? (m < 0 ? 1 : 2) : 0;
    }
}

// agg, p, the coarse near-null vector, the members of each aggregate.
__global__ void k_aggregate(int n, const int* mate, const double* w, const long long* aid, const long long* msz,
                            int* agg, double* p, double* wc, int* mem_ptr, int* mem) {
    GRID_STRIDE(i, n) {
        const int m = mate[i];
        if (m < 0) {
            const int I = (int)aid[i];
            agg[i] = I;
            p[i] = w[i] / fabs(w[i]);
            wc[I] = fabs(w[i]);
            mem_ptr[I] = (int)msz[i];
            mem[msz[i]] = (int)i;
        } else {
            const int lo = min((int)i, m), hi = max((int)i, m);
            const double nu = sqrt(w[lo] * w[lo] + w[hi] * w[hi]);
            const int I = (int)aid[lo];
            agg[i] = I;
            p[i] = w[i] / nu;
            if ((int)i == lo) {
                wc[I] = nu;
                mem_ptr[I] = (int)msz[i];
                mem[msz[i]] = lo;
                mem[msz[i] + 1] = hi;
            }
        }
    }
}

struct GTerm {
    int k1, k2, k3;
    double t;
};

// Galerkin A_c = P^T A P, one wavefront per coarse row.  The row's terms
// (entries of its members' rows) are sorted by coarse column J; every coarse
// entry then sums its terms in ascending (min(i,j), max(i,j), i).  Count pass
// (FILL false): distinct columns per row, the longest coarse row; fill pass:
// columns and values at crp.
template <bool FILL>
__global__ __launch_bounds__(64) void k_galerkin(int nc, const int* mem_ptr, const int* mem, const int* rp,
                                                 const int* ci, const double* v, const int* agg, const double* p,
                                                 int* cnt, const long long* crp, int* cci, double* cv, int* bad) {
    __shared__ unsigned long long key[kTermCap];
    const int lane = threadIdx.x;
    int longest = 0;
    for (int I = blockIdx.x; I < nc; I += gridDim.x) {
        const int q0 = mem_ptr[I], q1 = mem_ptr[I + 1];
        const int i0 = mem[q0], i1 = q1 - q0 > 1 ? mem[q0 + 1] : -1;
        const int b0 = rp[i0], len0 = rp[i0 + 1] - b0;
        const int b1 = i1 >= 0 ? rp[i1] : 0, len1 = i1 >= 0 ? rp[i1 + 1] - b1 : 0;
        const int T = len0 + len1;
        if (T > kTermCap) {
            if (lane == 0) atomicOr(bad, 1);
            continue;
        }
        int P = 1;
        while (P < T) P <<= 1;
        for (int t = lane; t < P; t += 64) {
            unsigned long long kk = ~0ull;
            if (t < T) {
                const int k = t < len0 ? b0 + t : b1 + (t - len0);
                kk = ((unsigned long long)(unsigned)agg[ci[k]] << 32) | (unsigned)t;
            }
            key[t] = kk;
        }
        __syncthreads();
        lds_bitonic(key, P);
        const long long base = FILL ? crp[I] : 0;
        int runs = 0;
        for (int c0 = 0; c0 < T; c0 += 64) {
            const int s = c0 + lane;
            const bool start = s < T && (s == 0 || (key[s] >> 32) != (key[s - 1] >> 32));
            const unsigned long long mask = __ballot(start);
            if (FILL && start) {
                const int r = runs + __popcll(mask & ((1ull << lane) - 1));
                const unsigned J = (unsigned)(key[s] >> 32);
                GTerm g[kRunCap];
                int m = 0;
                for (int e = s; e < T && (unsigned)(key[e] >> 32) == J; ++e) {
                    if (m == kRunCap) {
                        atomicOr(bad, 2);
                        break;
                    }
                    const int t = (int)(key[e] & 0xffffffffu);
                    const int k = t < len0 ? b0 + t : b1 + (t - len0);
                    const int i = t < len0 ? i0 : i1;
                    const int j = ci[k];
                    GTerm x{min(i, j), max(i, j), i, v[k] * (p[i] * p[j])};
                    int u = m++;
                    while (u > 0 && (g[u - 1].k1 > x.k1 || (g[u - 1].k1 == x.k1 && (g[u - 1].k2 > x.k2 ||
                                     (g[u - 1].k2 == x.k2 && g[u - 1].k3 > x.k3))))) {
                        g[u] = g[u - 1];
                        --u;
                    }
                    g[u] = x;
                }
                double sum = g[0].t;
                for (int u = 1; u < m; ++u) sum = sum + g[u].t;
                cci[base + r] = (int)J;
                cv[base + r] = sum;
            }
            runs += __popcll(mask);
        }
        if (!FILL && lane == 0) cnt[I] = runs;
        longest = max(longest, runs);
        __syncthreads();
    }
    if (!FILL && lane == 0) atomicMax(bad + 1, longest);
}

// ------------------------------------------------------------ layout kernels

__global__ void k_agg_sizes(int nc, const int* cip, const int* mem_ptr, int* sz) {
    GRID_STRIDE(Ip, nc) {
        const int I = cip[Ip];
        sz[Ip] = mem_ptr[I + 1] - mem_ptr[I];
    }
}

// Members of the aggregate at hierarchical coarse index Ip take the fine
// positions aggptr[Ip].., ascending.
__global__ void k_place(int nc, int n, const int* cip, const int* mem_ptr, const int* mem, const long long* ap,
                        int* aggptr, int* iperm, int* perm) {
    GRID_STRIDE(Ip, nc) {
        const int I = cip[Ip];
        const int q = (int)ap[Ip];
        aggptr[Ip] = q;
        for (int r = 0; r < mem_ptr[I + 1] - mem_ptr[I]; ++r) {
            const int i = mem[mem_ptr[I] + r];
            iperm[q + r] = i;
            perm[i] = q + r;
        }
        if (Ip == nc - 1) aggptr[nc] = n;
    }
}

__global__ void k_row_len(int n, const int* iperm, const int* rp, int* len) {
    GRID_STRIDE(ip, n) {
        const int i = iperm[ip];
        len[ip] = rp[i + 1] - rp[i];
    }
}

// Row ip of the permuted matrix: row iperm[ip] with columns renumbered by
// perm and sorted ascending (one wavefront per row); dinv and p follow.
__global__ __launch_bounds__(64) void k_reorder(int n, const int* iperm, const int* perm, const int* rp,
                                                const int* ci, const double* v, const double* dinv, const double* p,
                                                const long long* rp2, int* ci2, double* v2, double* dinv2,
                                                double* p2) {
    __shared__ unsigned long long key[kRowCap];
    const int lane = threadIdx.x;
    for (int ip = blockIdx.x; ip < n; ip += gridDim.x) {
        const int i = iperm[ip];
        const int b = rp[i], len = rp[i + 1] - b;
        int P = 1;
        while (P < len) P <<= 1;
        for (int t = lane; t < P; t += 64)
            key[t] = t < len ? (((unsigned long long)(unsigned)perm[ci[b + t]] << 32) | (unsigned)t) : ~0ull;
        __syncthreads();
        lds_bitonic(key, P);
        const long long o = rp2[ip];
        for (int t = lane; t < len; t += 64) {
            ci2[o + t] = (int)(key[t] >> 32);
            v2[o + t] = v[b + (int)(key[t] & 0xffffffffu)];
        }
        if (lane == 0) {
            dinv2[ip] = dinv[i];
            if (p2) p2[ip] = p[i];
        }
        __syncthreads();
    }
}

__global__ void k_vd(long long nnz, const int* ci, const double* v, const double* dinv, double* vd) {
    GRID_STRIDE(k, nnz) vd[k] = v[k] * dinv[ci[k]];
}

// Column dictionary of each tile: its distinct columns, ascending (count
// pass: their number and the longest; fill pass: the columns at the tile's
// offset and every entry's 16-bit position).  A tile longer than cap (one
// long row) has none.
template <bool FILL>
__global__ __launch_bounds__(kSB) void k_dict(int ntiles, const int4* tiles, const int* ci, int cap, int* dlen,
                                              const long long* doff, int* dcol, uint16_t* loc, int* maxlen) {
    __shared__ int key[kDictCap];
    __shared__ int uq[kDictCap];
    __shared__ int wsum[kSB / 64 + 1];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 d = tiles[t];
        const int k0 = d.x, m = d.y - d.x;
        if (m > cap) {
            if (!FILL && threadIdx.x == 0) dlen[t] = 0;
            continue;
        }
        int P = 1;
        while (P < m) P <<= 1;
        for (int u = threadIdx.x; u < P; u += kSB) key[u] = u < m ? ci[k0 + u] : INT_MAX;
        __syncthreads();
        lds_bitonic(key, P);
        // distinct columns: a scan of the run-start flags, kSB-element chunks
        int total = 0;
        for (int c0 = 0; c0 < m; c0 += kSB) {
            const int u = c0 + threadIdx.x;
            const bool st = u < m && (u == 0 || key[u] != key[u - 1]);
            const unsigned long long mask = __ballot(st);
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            if (lane == 0) wsum[wv] = __popcll(mask);
            __syncthreads();
            int before = 0, all = 0;
            for (int q = 0; q < kSB / 64; ++q) {
                if (q < wv) before += wsum[q];
                all += wsum[q];
            }
            if (FILL && st) {
                const int pos = total + before + __popcll(mask & ((1ull << lane) - 1));
                uq[pos] = key[u];
                dcol[doff[t] + pos] = key[u];
            }
            total += all;
            __syncthreads();
        }
        if (!FILL) {
            if (threadIdx.x == 0) {
                dlen[t] = total;
                atomicMax(maxlen, total);
            }
        } else {
            for (int u = threadIdx.x; u < m; u += kSB) {
                const int col = ci[k0 + u];
                int b = 0, e = total;
                while (b < e) {
                    const int h = (b + e) >> 1;
                    if (uq[h] < col) b = h + 1; else e = h;
                }
                loc[k0 + u] = (uint16_t)b;
            }
        }
        __syncthreads();
    }
}

__global__ void k_spans(int ntiles, const long long* doff, const int* dlen, int* span) {
    GRID_STRIDE(t, ntiles) {
        span[2 * t] = (int)doff[t];
        span[2 * t + 1] = dlen[t];
    }
}

// ------------------------------------------------------ aggregate composition

// The pairwise levels composed into one kept level (at most kMaxAggSteps).
struct Chain {
    const int* agg[kMaxAggSteps];
    const double* p[kMaxAggSteps];
    int steps;
};

// Composed aggregate and prolongator entry of every row of a kept level: the
// row's aggregate followed through the chain, p multiplied finest first.
__global__ void k_compose(int n, Chain c, int* cagg, double* cp) {
    GRID_STRIDE(i, n) {
        int I = c.agg[0][i];
        double pc = c.p[0][i];
        for (int m = 1; m < c.steps; ++m) {
            pc = pc * c.p[m][I];
            I = c.agg[m][I];
        }
        cagg[i] = I;
        cp[i] = pc;
    }
}

__global__ void k_count_members(int n, const int* cagg, int* cnt) { GRID_STRIDE(i, n) atomicAdd(&cnt[cagg[i]], 1); }

__global__ void k_fill_members(int n, const int* cagg, const long long* mptr, int* fill, int* mem) {
    GRID_STRIDE(i, n) {
        const int I = cagg[i];
        mem[mptr[I] + atomicAdd(&fill[I], 1)] = (int)i;
    }
}

// Members of each composed aggregate ascending (at most 2^kMaxAggSteps).
__global__ void k_sort_members(int nc, const long long* mptr, int* mem, int* mem_ptr, int* longest) {
    int mx = 0;
    GRID_STRIDE(I, nc) {
        const int b = (int)mptr[I], e = (int)mptr[I + 1];
        for (int q = b + 1; q < e; ++q) {
            const int x = mem[q];
            int u = q;
            while (u > b && mem[u - 1] > x) {
                mem[u] = mem[u - 1];
                --u;
            }
            mem[u] = x;
        }
        mem_ptr[I] = b;
        if (I == nc - 1) mem_ptr[nc] = e;
        mx = max(mx, e - b);
    }
    atomicMax(longest, mx);
}

// ------------------------------------------------------------------ driver

// A level in canonical numbering, as the device loop leaves it.
struct CanLevel {
    int n = 0, nc = 0, pairs = 0, maxrow = 0;
    long long nnz = 0;
    int *rp = nullptr, *ci = nullptr;
    double *v = nullptr, *w = nullptr, *dinv = nullptr, *p = nullptr;
    int *agg = nullptr, *mem_ptr = nullptr, *mem = nullptr;
};

int grid_rows(long long n) { return (int)std::min<long long>(std::max<long long>(n, 1), kGridCap); }

enum Coarsened { kCoarsened, kNoPairs, kAsymmetric };

// Matching, aggregates and Galerkin product of level L (canonical); fills the
// next level's matrix and near-null vector.  kNoPairs: the level is left to
// the host; kAsymmetric: the pattern is not symmetric (only the input level
// can be), the whole build is left to the host.
Coarsened coarsen(Temps& T, CanLevel& L, CanLevel& C, hipStream_t s) {
    const int n = L.n;
    double* diag = T.get<double>(n);
    double* c = T.get<double>(L.nnz);
    int* flag = T.get<int>(4);
    HIP_CHECK(hipMemsetAsync(flag, 0, 4 * sizeof(int), s));
    hipLaunchKernelGGL(k_l1diag, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)L.rp, (const int*)L.ci,
                       (const double*)L.v, L.dinv, diag, flag + 2);
    hipLaunchKernelGGL(k_weights, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)L.rp, (const int*)L.ci,
                       (const double*)L.v, (const double*)diag, (const double*)L.w, c, flag);
    int head[3];
    HIP_CHECK(hipMemcpyAsync(head, flag, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (head[0]) return kAsymmetric;
    T.release(diag);
    // eligible neighbours in the matching order
    int* adj = T.get<int>(L.nnz);
    int* ecnt = T.get<int>(n);
    hipLaunchKernelGGL(k_sort_adj, dim3(grid_rows(n)), dim3(64), 0, s, n, (const int*)L.rp, (const int*)L.ci,
                       (const double*)c, adj, ecnt);
    T.release(c);
    // matching rounds, kRoundsPerCheck between looks at the counters (a
    // round with nothing alive changes nothing); every round with an alive
    // vertex matches at least the heaviest picked edge
    constexpr int kRoundsPerCheck = 8;
    int* mate = T.get<int>(n);
    int* cand = T.get<int>(n);
    int* cur = T.get<int>(n);
    unsigned char* state = T.get<unsigned char>(n);
    HIP_CHECK(hipMemsetAsync(mate, 0xff, sizeof(int) * n, s));
    HIP_CHECK(hipMemsetAsync(state, 0, n, s));
    hipLaunchKernelGGL(k_cursor, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)L.rp, cur);
    int* cnt = flag + 2;
    const int gc = std::min(grid_for(n, kSB), kCommitGrid);
    for (long long round = 0;; round += kRoundsPerCheck) {
        HIP_CHECK(hipMemsetAsync(cnt, 0, 2 * sizeof(int), s));
        for (int r = 0; r < kRoundsPerCheck; ++r) {
            HIP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int), s));
            hipLaunchKernelGGL(k_pick, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)L.rp,
                               (const int*)ecnt, (const int*)adj, (const int*)mate, state, cur, cand);
            hipLaunchKernelGGL(k_commit, dim3(gc), dim3(kSB), 0, s, n, (const int*)cand, mate, state, cnt);
        }
        int rc[2];
        HIP_CHECK(hipMemcpyAsync(rc, cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (rc[0] == 0) break;
        if (rc[1] == 0 || round > n) throw Error(PAMG_E_DEVICE, "device matching made no progress");
    }
    T.release(adj);
    T.release(ecnt);
    T.release(cur);
    T.release(cand);
    T.release(state);
    // aggregates
    int* lead = T.get<int>(n);
    int* size = T.get<int>(n);
    hipLaunchKernelGGL(k_leaders, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)mate, lead, size);
    long long* aid = T.get<long long>((size_t)n + 1);
    long long* msz = T.get<long long>((size_t)n + 1);
    const long long nc = scan<int>(T, n, lead, aid, s);
    scan<int>(T, n, size, msz, s);
    T.release(lead);
    T.release(size);
    L.nc = (int)nc;
    L.pairs = (int)(n - nc);
    if (L.pairs == 0) {
        T.release(mate);
        T.release(aid);
        T.release(msz);
        return kNoPairs;
    }
    int* agg = T.get<int>(n);
    L.agg = agg;
    L.p = T.get<double>(n);
    C.w = T.get<double>(nc);
    L.mem_ptr = T.get<int>(nc + 1);
    L.mem = T.get<int>(n);
    hipLaunchKernelGGL(k_aggregate, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)mate, (const double*)L.w,
                       (const long long*)aid, (const long long*)msz, agg, L.p, C.w, L.mem_ptr, L.mem);
    to_device(L.mem_ptr + nc, &n, 1, s);
    T.release(mate);
    T.release(aid);
    T.release(msz);
    // Galerkin product
    int* ccnt = T.get<int>(nc);
    long long* crp = T.get<long long>((size_t)nc + 1);
    HIP_CHECK(hipMemsetAsync(flag, 0, 4 * sizeof(int), s));
    const int gg = grid_rows(nc);
    hipLaunchKernelGGL(k_galerkin<false>, dim3(gg), dim3(64), 0, s, (int)nc, (const int*)L.mem_ptr,
                       (const int*)L.mem, (const int*)L.rp, (const int*)L.ci, (const double*)L.v, (const int*)agg,
                       (const double*)L.p, ccnt, (const long long*)nullptr, (int*)nullptr, (double*)nullptr, flag);
    const long long cnnz = scan<int>(T, nc, ccnt, crp, s);
    if (cnnz >= (1ll << 31)) throw Error(PAMG_E_OOM, "coarse matrix exceeds 2^31 entries");
    C.n = (int)nc;
    C.nnz = cnnz;
    C.rp = T.get<int>(nc + 1);
    C.ci = T.get<int>(cnnz);
    C.v = T.get<double>(cnnz);
    C.dinv = T.get<double>(nc);
    hipLaunchKernelGGL(k_galerkin<true>, dim3(gg), dim3(64), 0, s, (int)nc, (const int*)L.mem_ptr,
                       (const int*)L.mem, (const int*)L.rp, (const int*)L.ci, (const double*)L.v, (const int*)agg,
                       (const double*)L.p, ccnt, (const long long*)crp, C.ci, C.v, flag);
    hipLaunchKernelGGL(k_to_int, dim3(grid_for(nc + 1, kSB)), dim3(kSB), 0, s, nc + 1, (const long long*)crp, C.rp);
    HIP_CHECK(hipMemcpyAsync(head, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (head[0]) throw Error(PAMG_E_DEVICE, "device Galerkin product: a coarse row exceeds its term capacity");
    C.maxrow = head[1];
    T.release(ccnt);
    T.release(crp);
    return kCoarsened;
}

// Host copy of a canonical level (matrix and near-null vector).
void download_level(const CanLevel& L, HostLevel& out, hipStream_t s) {
    out.A.n = L.n;
    to_host(out.A.rp, L.rp, (size_t)L.n + 1, s);
    to_host(out.A.ci, L.ci, (size_t)L.nnz, s);
    to_host(out.A.v, L.v, (size_t)L.nnz, s);
    to_host(out.w, L.w, (size_t)L.n, s);
}

}  // namespace

bool device_setup_applies(const pamg_params& prm) {
    return prm.device_setup != 0 && prm.host_only == 0 && prm.agg_steps >= 1 && prm.smooth_prolongator == 0 &&
           (prm.smoother == PAMG_SMOOTHER_L1_JACOBI || prm.smoother == PAMG_SMOOTHER_HYBRID_GS) &&
           prm.match_all_edges == 0;
}

namespace {

// Per row of a level with blocks of nb rows: 1 / a_ii and the range of the
// row's entries whose columns lie in its block (first such entry; the counts
// before and after the row; whether a_ii is stored), as the host schedule.
__global__ void k_gs_rows(int n, int nb, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, double* __restrict__ ainv, int* __restrict__ fresh,
                          int* __restrict__ bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int b0 = i / nb * nb, b1 = min(n, b0 + nb);
        int first = -1, before = 0, after = 0, diag = 0;
        double a = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            if (j >= b0 && j < b1 && first < 0) first = k;
            if (j >= b0 && j < i) ++before;
            if (j > i && j < b1) ++after;
            if (j == i) {
                if (!(v[k] > 0.0)) *bad = 1;
                a = 1.0 / v[k];
                diag = 1;
            }
        }
        ainv[i] = a;
        fresh[2 * (size_t)i] = first < 0 ? rp[i] : first;
        fresh[2 * (size_t)i + 1] = before | after << 8 | diag << 16;
    }
}

// Per block: each row's depth in the block's forward (earlier rows) and
// backward (later rows) dependency graph, and the block's largest depths; one
// thread walks its block's rows in order, as the host schedule.
__global__ void k_gs_depths(int n, int nb, int nblk, const int* __restrict__ rp, const int* __restrict__ ci,
                            uint8_t* __restrict__ df, uint8_t* __restrict__ db, int* __restrict__ maxd) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nblk; p += gridDim.x * blockDim.x) {
        const int b0 = p * nb, b1 = min(n, b0 + nb);
        int mf = 0, mb = 0;
        for (int i = b0; i < b1; ++i) {
            int d = 0;
            for (int k = rp[i]; k < rp[i + 1]; ++k) {
                const int j = ci[k];
                if (j >= b0 && j < i) d = max(d, (int)df[j] + 1);
            }
            df[i] = (uint8_t)d;
            mf = max(mf, d);
        }
        for (int i = b1 - 1; i >= b0; --i) {
            int d = 0;
            for (int k = rp[i]; k < rp[i + 1]; ++k) {
                const int j = ci[k];
                if (j > i && j < b1) d = max(d, (int)db[j] + 1);
            }
            db[i] = (uint8_t)d;
            mb = max(mb, d);
        }
        maxd[2 * p] = mf;
        maxd[2 * p + 1] = mb;
    }
}

}  // namespace

void device_gs_schedule(pamg_hierarchy* h, DevLevelOut& D, int nb, hipStream_t s) {
    const int n = D.n, nblk = (n + nb - 1) / nb;
    D.gs_nblk = nblk;
    D.gs_ainv = dalloc<double>(h, n, s);
    D.gs_fresh = dalloc<int>(h, 2 * (size_t)n, s);
    D.gs_df = dalloc<uint8_t>(h, n, s);
    D.gs_db = dalloc<uint8_t>(h, n, s);
    D.gs_maxd = dalloc<int>(h, 2 * (size_t)nblk, s);
    Temps T{h->ctx, s, {}};
    int* bad = T.get<int>(1);
    HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_gs_rows, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, nb, (const int*)D.rp, (const int*)D.ci,
                       (const double*)D.v, D.gs_ainv, D.gs_fresh, bad);
    hipLaunchKernelGGL(k_gs_depths, dim3(grid_for(nblk, 64)), dim3(64), 0, s, n, nb, nblk, (const int*)D.rp,
                       (const int*)D.ci, D.gs_df, D.gs_db, D.gs_maxd);
    HIP_CHECK(hipGetLastError());
    if (read1(bad, s)) throw Error(PAMG_E_NOT_SPD, "non-positive diagonal on a coarse level (Gauss-Seidel smoother)");
}

std::unique_ptr<DeviceBuild> device_build(pamg_hierarchy* h, const pamg_csr& A, const pamg_params& prm,
                                          hipStream_t s) {
    std::unique_ptr<DeviceBuild> out(new DeviceBuild());
    Temps T{h->ctx, s, {}};
    const int floor_rows = prm.device_min_rows > 0 ? prm.device_min_rows : kDeviceMinRows;
    const int limit = std::max({floor_rows, prm.max_dense, prm.max_coarse});
    auto dev_level = [&](const CanLevel& L, int l) {
        return L.n > limit && l + 1 < prm.max_levels && L.maxrow <= kRowCap;
    };
    // level 0: the input matrix (its header checked by the caller), w = 1
    std::vector<CanLevel> lev(1);
    {
        CanLevel& L0 = lev[0];
        L0.n = A.n;
        L0.nnz = A.nnz;
        int mx = 0;
        for (int i = 0; i < A.n; ++i) mx = std::max(mx, A.row_ptr[i + 1] - A.row_ptr[i]);
        L0.maxrow = mx;
        if (!dev_level(L0, 0)) return nullptr;   // the host build validates it
        L0.rp = T.get<int>((size_t)A.n + 1);
        L0.ci = T.get<int>(A.nnz);
        L0.v = T.get<double>(A.nnz);
        L0.w = T.get<double>(A.n);
        to_device(L0.rp, A.row_ptr, (size_t)A.n + 1, s);
        to_device(L0.ci, A.col_idx, (size_t)A.nnz, s);
        to_device(L0.v, A.val, (size_t)A.nnz, s);
        // validate_csr's row checks before any kernel follows the columns
        unsigned long long* first = T.get<unsigned long long>(1);
        HIP_CHECK(hipMemsetAsync(first, 0xff, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_validate, dim3(grid_for(A.n, kSB)), dim3(kSB), 0, s, A.n, (long long)A.nnz,
                           (const int*)L0.rp, (const int*)L0.ci, (const double*)L0.v, first);
        const unsigned long long f = read1(first, s);
        if (f != ~0ull) throw Error(PAMG_E_INVALID, csr_error((int)(f & 0xff), (int64_t)(f >> 8)));
        if (prm.check_symmetry) {
            int* asym = T.get<int>(1);
            HIP_CHECK(hipMemsetAsync(asym, 0, sizeof(int), s));
            hipLaunchKernelGGL(k_check_symmetry, dim3(grid_for(A.n, kSB)), dim3(kSB), 0, s, A.n,
                               (const int*)L0.rp, (const int*)L0.ci, (const double*)L0.v, asym);
            if (read1(asym, s)) throw Error(PAMG_E_INVALID, "matrix is not bitwise symmetric");
        }
        hipLaunchKernelGGL(k_fill_d, dim3(grid_for(A.n, kSB)), dim3(kSB), 0, s, (long long)A.n, L0.w, 1.0);
    }
    // device (pairwise) levels
    const int steps = std::max(1, prm.agg_steps);
    int built = 0;
    for (;;) {
        CanLevel& L = lev[built];
        L.dinv = T.get<double>(L.n);
        CanLevel C;
        const Coarsened r = coarsen(T, L, C, s);
        if (r == kAsymmetric) return nullptr;
        if (r == kNoPairs) break;          // the host takes this level
        lev.push_back(C);
        ++built;
        if (!dev_level(lev[built], built)) break;
    }
    // the host continues from a kept level (a multiple of the composition
    // step), so that every composed prolongator lies on one side
    const int m = built / steps * steps;
    if (m == 0) return nullptr;
    // host levels from level m
    {
        HostHierarchy& Hs = out->host;
        Hs.lev.emplace_back();
        download_level(lev[m], Hs.lev[0], s);
        pamg_params p2 = prm;
        p2.max_levels = prm.max_levels - m;
        extend_hierarchy(Hs, p2);
        const HostCSR& AL = Hs.lev.back().A;
        if (AL.n > prm.max_dense)
            throw Error(PAMG_E_STALLED, "coarsening stalled at " + std::to_string(AL.n) +
                                            " unknowns, above the dense-solve limit");
        if (steps > 1) compose_levels(Hs, steps);
        out->host_lay = build_layout(Hs);
    }
    // kept device levels: every steps-th pairwise level below m, with its
    // aggregates and prolongator composed over the steps in between
    const int K = m / steps;
    out->m = K;
    std::vector<int> kp(K), knc(K);
    std::vector<double*> kcp(K);
    std::vector<int*> kmptr(K), kmem(K);
    for (int j = 0; j < K; ++j) {
        const int a = j * steps;
        const CanLevel& L = lev[a];
        kp[j] = a;
        knc[j] = lev[a + steps].n;
        if (steps == 1) {
            kcp[j] = L.p;
            kmptr[j] = L.mem_ptr;
            kmem[j] = L.mem;
            continue;
        }
        Chain ch{};
        ch.steps = steps;
        for (int q = 0; q < steps; ++q) {
            ch.agg[q] = lev[a + q].agg;
            ch.p[q] = lev[a + q].p;
        }
        const int n = L.n, nc = knc[j];
        int* cagg = T.get<int>(n);
        kcp[j] = T.get<double>(n);
        hipLaunchKernelGGL(k_compose, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, ch, cagg, kcp[j]);
        int* cnt = T.get<int>(nc);
        HIP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int) * nc, s));
        hipLaunchKernelGGL(k_count_members, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)cagg, cnt);
        long long* mptr = T.get<long long>((size_t)nc + 1);
        scan<int>(T, nc, cnt, mptr, s);
        HIP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int) * nc, s));
        kmem[j] = T.get<int>(n);
        kmptr[j] = T.get<int>((size_t)nc + 1);
        hipLaunchKernelGGL(k_fill_members, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)cagg,
                           (const long long*)mptr, cnt, kmem[j]);
        int* longest = T.get<int>(1);
        HIP_CHECK(hipMemsetAsync(longest, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_sort_members, dim3(grid_for(nc, kSB)), dim3(kSB), 0, s, nc, (const long long*)mptr,
                           kmem[j], kmptr[j], longest);
        if (read1(longest, s) > (1 << kMaxAggSteps)) throw Error(PAMG_E_DEVICE, "composed aggregate too large");
        T.release(cnt);
        T.release(mptr);
        T.release(cagg);
    }
    // device layouts of the kept levels K-1 .. 0 (their arrays belong to the hierarchy)
    out->dev.resize(K);
    const int* cip = nullptr;   // hierarchical -> canonical of the coarser level
    std::vector<int> cip_host;
    int* cip_dev = nullptr;
    cip_host = out->host_lay[0].iperm;
    cip_dev = T.get<int>(cip_host.size());
    to_device(cip_dev, cip_host.data(), cip_host.size(), s);
    cip = cip_dev;
    for (int j = K - 1; j >= 0; --j) {
        const CanLevel& L = lev[kp[j]];
        DevLevelOut& D = out->dev[j];
        const int n = L.n, nc = knc[j];
        const int* mem_ptr = kmptr[j];
        const int* mem = kmem[j];
        D.n = n;
        D.nc = nc;
        D.nnz = L.nnz;
        D.pairs = L.pairs;
        int* sz = T.get<int>(nc);
        long long* ap = T.get<long long>((size_t)nc + 1);
        hipLaunchKernelGGL(k_agg_sizes, dim3(grid_for(nc, kSB)), dim3(kSB), 0, s, nc, cip, mem_ptr, sz);
        scan<int>(T, nc, sz, ap, s);
        D.aggptr = dalloc<int>(h, (size_t)nc + 1, s);
        D.iperm = dalloc<int>(h, n, s);
        D.perm = dalloc<int>(h, n, s);
        hipLaunchKernelGGL(k_place, dim3(grid_for(nc, kSB)), dim3(kSB), 0, s, nc, n, cip, mem_ptr, mem,
                           (const long long*)ap, D.aggptr, D.iperm, D.perm);
        T.release(sz);
        T.release(ap);
        int* len = T.get<int>(n);
        long long* rp2 = T.get<long long>((size_t)n + 1);
        hipLaunchKernelGGL(k_row_len, dim3(grid_for(n, kSB)), dim3(kSB), 0, s, n, (const int*)D.iperm,
                           (const int*)L.rp, len);
        scan<int>(T, n, len, rp2, s);
        T.release(len);
        D.rp = dalloc<int>(h, (size_t)n + 1, s);
        D.ci = dalloc<int>(h, L.nnz, s);
        D.v = dalloc<double>(h, L.nnz, s);
        D.dinv = dalloc<double>(h, n, s);
        D.p = dalloc<double>(h, n, s);
        hipLaunchKernelGGL(k_reorder, dim3(grid_rows(n)), dim3(64), 0, s, n, (const int*)D.iperm,
                           (const int*)D.perm, (const int*)L.rp, (const int*)L.ci, (const double*)L.v,
                           (const double*)L.dinv, (const double*)kcp[j], (const long long*)rp2, D.ci, D.v, D.dinv,
                           D.p);
        hipLaunchKernelGGL(k_to_int, dim3(grid_for(n + 1, kSB)), dim3(kSB), 0, s, (long long)n + 1,
                           (const long long*)rp2, D.rp);
        T.release(rp2);
        D.vd = dalloc<double>(h, L.nnz, s);
        hipLaunchKernelGGL(k_vd, dim3(grid_for(L.nnz, kSB)), dim3(kSB), 0, s, L.nnz, (const int*)D.ci,
                           (const double*)D.v, (const double*)D.dinv, D.vd);
        // tiles (host partition of the row pointer) and dictionaries
        std::vector<int32_t> rp_h, ap_h;
        to_host(rp_h, D.rp, (size_t)n + 1, s);
        to_host(ap_h, D.aggptr, (size_t)nc + 1, s);
        for (int32_t c = 0; c < nc; ++c) D.max_agg = std::max(D.max_agg, ap_h[c + 1] - ap_h[c]);
        int items = first_tile_items(L.nnz);
        std::vector<int32_t> up, down;
        int* dl_up = nullptr;
        int* dl_down = nullptr;
        int* flag = T.get<int>(2);
        int max_up = 0, max_down = 0;
        for (;;) {
            const int cap = items * kBlock;
            make_tiles(rp_h, ap_h, n, nc, cap, up, down);
            D.items = items;
            if (items < kDictItems) break;
            int4* tu = T.get<int4>(up.size() / 4);
            int4* td = T.get<int4>(down.size() / 4);
            to_device(reinterpret_cast<int*>(tu), up.data(), up.size(), s);
            to_device(reinterpret_cast<int*>(td), down.data(), down.size(), s);
            dl_up = T.get<int>(up.size() / 4);
            dl_down = T.get<int>(down.size() / 4);
            HIP_CHECK(hipMemsetAsync(flag, 0, 2 * sizeof(int), s));
            const int nu = (int)(up.size() / 4), nd = (int)(down.size() / 4);
            // the dictionaries hold permuted columns
            hipLaunchKernelGGL(k_dict<false>, dim3(grid_rows(nu)), dim3(kSB), 0, s, nu, (const int4*)tu,
                               (const int*)D.ci, cap, dl_up, (const long long*)nullptr, (int*)nullptr,
                               (uint16_t*)nullptr, flag);
            hipLaunchKernelGGL(k_dict<false>, dim3(grid_rows(nd)), dim3(kSB), 0, s, nd, (const int4*)td,
                               (const int*)D.ci, cap, dl_down, (const long long*)nullptr, (int*)nullptr,
                               (uint16_t*)nullptr, flag + 1);
            int mx[2];
            HIP_CHECK(hipMemcpyAsync(mx, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            max_up = mx[0];
            max_down = mx[1];
            if (items == kDictItems || std::max(max_up, max_down) <= kDictMaxLarge) {
                // fill the dictionaries
                auto fill = [&](int nt, const int4* tt, int* dl, int maxl, DevDict& dd) {
                    long long* off = T.get<long long>((size_t)nt + 1);
                    const long long tot = scan<int>(T, nt, dl, off, s);
                    if (tot >= (1ll << 31)) throw Error(PAMG_E_OOM, "tile dictionaries exceed 2^31 entries");
                    dd.col = dalloc<int>(h, tot, s);
                    dd.loc = dalloc<uint16_t>(h, L.nnz, s);
                    dd.span = dalloc<int>(h, 2 * (size_t)nt, s);
                    HIP_CHECK(hipMemsetAsync(dd.loc, 0, sizeof(uint16_t) * L.nnz, s));
                    hipLaunchKernelGGL(k_dict<true>, dim3(grid_rows(nt)), dim3(kSB), 0, s, nt, tt,
                                       (const int*)D.ci, cap, dl, (const long long*)off, dd.col, dd.loc, flag);
                    hipLaunchKernelGGL(k_spans, dim3(grid_for(nt, kSB)), dim3(kSB), 0, s, nt, (const long long*)off,
                                       (const int*)dl, dd.span);
                    dd.len = tot;
                    dd.max_len = maxl;
                    T.release(off);
                };
                fill(nu, tu, dl_up, max_up, D.up_dict);
                fill(nd, td, dl_down, max_down, D.down_dict);
                HIP_CHECK(hipStreamSynchronize(s));
                break;
            }
            items /= 2;
        }
        D.up_tiles = dalloc<int>(h, up.size(), s);
        to_device(D.up_tiles, up.data(), up.size(), s);
        D.n_up = (int)(up.size() / 4);
        D.down_tiles = dalloc<int>(h, down.size(), s);
        to_device(D.down_tiles, down.data(), down.size(), s);
        D.n_down = (int)(down.size() / 4);
        cip = D.iperm;
    }
    HIP_CHECK(hipStreamSynchronize(s));
    return out;
}

}  // namespace pamg
