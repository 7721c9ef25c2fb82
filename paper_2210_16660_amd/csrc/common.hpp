// Internal declarations shared by the host setup and the device driver.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "pamg.h"

namespace pamg {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

// Host CSR in canonical numbering.
struct HostCSR {
    int32_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// One level of the canonical hierarchy built on the host.
struct HostLevel {
    HostCSR A;
    std::vector<double> w;      // near-null vector
    std::vector<double> dinv;   // 1 / sum_j |a_ij|
    std::vector<int32_t> agg;   // aggregate of each unknown (levels < L)
    std::vector<double> p;      // prolongator entry of each unknown (levels < L)
    int32_t pairs = 0;
    HostCSR P;                  // smoothed prolongator n_l x n_{l+1} (smooth_prolongator only)
    double omega_p = 0.0;
};

// One level of the pairwise chain that aggregate-size composition condenses:
// its pairwise aggregates and prolongator (levels < last) and, for a level
// that composition dropped, its pattern.  Kept for coefficient-only reuse.
struct PairLevel {
    int32_t kept = -1;                  // its index among the kept levels, or -1 (dropped)
    HostCSR S;                          // pattern (rp, ci) of a dropped level; values unused
    std::vector<int32_t> agg;
    std::vector<double> p;
};

struct HostHierarchy {
    std::vector<HostLevel> lev;         // 0..L
    std::vector<PairLevel> chain;       // the pairwise levels behind lev (empty: lev itself)
};

// Device-ready layout of one level in hierarchical (aggregate-contiguous) order.
struct TileDict {
    std::vector<int32_t> span;      // 2 ints per tile: first dictionary entry, dictionary length
    std::vector<int32_t> col;       // the dictionaries, tile after tile
    std::vector<uint16_t> local;    // per matrix entry: position of its column in the tile's dictionary
    int32_t max_len = 0;            // longest dictionary of the level
};

// A CSR matrix's row tiles (<= kTileRows rows and <= items * kBlock entries,
// or one longer row; 4 ints per tile: k0, k1, r0, r1) with their column
// dictionaries (tiles of >= kDictItems items per thread): the layout of the
// tile kernels, used for the smoothed prolongator's P and P^T.
struct TiledRows {
    int items = 1;
    std::vector<int32_t> tiles;
    TileDict dict;
};

// Hybrid Gauss-Seidel schedule of one level in hierarchical (nested-aggregate)
// order, blocks of nb consecutive rows: every row's depth in its block's
// forward (earlier rows) and backward (later rows) dependency graph (rows of
// one depth are independent, so a sweep runs depth by depth), each block's
// largest depth per direction, and 1 / a_ii.
struct GsLevel {
    std::vector<uint8_t> depth_f, depth_b;
    std::vector<int32_t> maxd;      // 2 per block: forward, backward
    std::vector<double> ainv;       // 1 / a_ii
    // 2 per row: the first entry whose column is in the row's block, and
    // nf | nb << 8 | diag << 16 with nf (nb) the entries of columns in the
    // block before (after) the row and diag 1 if the row stores a_ii: the
    // in-block entries are consecutive in the sorted row, so a sweep reads
    // only them
    std::vector<int32_t> fresh;
};

struct LayoutLevel {
    std::vector<int32_t> perm;      // canonical -> hierarchical index
    std::vector<int32_t> iperm;     // hierarchical -> canonical
    std::vector<int32_t> rp, ci;    // permuted CSR, columns ascending
    std::vector<double> v;
    std::vector<double> vd;         // column-scaled values a_ij / d_j (restriction pass, l < L)
    std::vector<double> dinv, p;    // permuted
    std::vector<int32_t> aggptr;    // n_{l+1}+1: members of coarse row I are rows [aggptr[I], aggptr[I+1])
    int items = 8;                  // tile capacity of this level: items * kBlock entries
    std::vector<int32_t> down_tiles;  // 4 ints per restriction tile: k0, k1, c0, c1 (l < L)
    std::vector<int32_t> up_tiles;    // 4 ints per row tile: k0, k1, r0, r1
    // Column dictionaries of the tiles: the distinct columns of a tile's
    // entries, ascending, gathered once per tile into LDS; every entry stores
    // the 16-bit position of its column in its tile's dictionary.  A tile
    // holding one row / aggregate longer than a tile has no dictionary.
    TileDict up_dict, down_dict;
    GsLevel gs;                     // hybrid Gauss-Seidel smoother only (l < L)
    // smoothed prolongator only (l < L): P (rows of this level, columns of the
    // next, both hierarchical, columns ascending) and P^T
    std::vector<int32_t> sa_prp, sa_pci, sa_trp, sa_tci;
    std::vector<double> sa_pv, sa_tv;
    TiledRows sa_ptile, sa_ttile;   // their row tiles and column dictionaries
};

constexpr int kBlock = 256;          // threads per workgroup of the tile kernels
constexpr int kMaxItems = 16;        // matrix entries per thread per tile (largest tiles)
constexpr int kDictItems = 8;        // tiles of at least this many items per thread use column dictionaries
constexpr int kDictMaxLarge = 2048;  // longest dictionary accepted for the largest tiles (prefetch slots)
constexpr int kTileRows = kBlock;    // at most one row (or aggregate) per thread in a tile
constexpr int kMaxAggSteps = 4;      // composed aggregates hold at most 2^4 fine rows
constexpr int kTargetTiles = 1024;   // small levels shrink their tiles to keep >= this many

// setup.cpp
void validate_csr(const pamg_csr& A, bool check_symmetry);
void validate_csr_header(const pamg_csr& A);
// The message of row check `code` (1..6 as validate_csr numbers them) failing in `row`.
std::string csr_error(int code, int64_t row);
HostHierarchy build_hierarchy(const pamg_csr& A, const pamg_params& prm);
void extend_hierarchy(HostHierarchy& H, const pamg_params& prm);
// Keep levels 0, s, 2s, ... and the last of a pairwise hierarchy, composing
// aggregates and prolongators in between (the pairwise chain kept in H.chain).
void compose_levels(HostHierarchy& H, int s);
std::vector<LayoutLevel> build_layout(const HostHierarchy& H);
int first_tile_items(int64_t nnz);
void make_tiles(const std::vector<int32_t>& rp, const std::vector<int32_t>& aggptr, int32_t n, int32_t nc,
                int32_t cap, std::vector<int32_t>& up, std::vector<int32_t>& down);

// Smoothed prolongator of level l in hierarchical numbering (P and P^T).
void sa_layout(const HostCSR& P, const LayoutLevel& fine, const LayoutLevel& coarse, LayoutLevel& out);
// Row tiles and dictionaries of an n-row CSR matrix with ncols columns.
TiledRows tile_rows(const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, int32_t n, int32_t ncols);

// Hybrid Gauss-Seidel schedule of a laid-out level (blocks of nb <= 256 rows).
GsLevel gs_schedule(const LayoutLevel& L, int nb);

// Coefficient-only reuse.  The Galerkin sum of one pairwise step as a plan:
// for every coarse entry (canonical CSR order of Ac) the fine entries of A
// that sum into it, in the setup's order, each with its factor p_i p_j (the
// setup's term is a_ij (p_i p_j)).  A and Ac are used for their patterns.
struct GalerkinPlan {
    std::vector<int32_t> ptr;   // nnz(Ac) + 1: terms of coarse entry e are [ptr[e], ptr[e+1])
    std::vector<int32_t> k;     // nnz(A): fine entry of each term
    std::vector<double> pp;     // nnz(A): p_i p_j of each term
};
GalerkinPlan galerkin_plan(const HostCSR& A, const std::vector<int32_t>& agg, const std::vector<double>& p,
                           const HostCSR& Ac);
// For every entry of a level's hierarchical CSR, its canonical entry index.
std::vector<int32_t> entry_order(const HostCSR& A, const std::vector<int32_t>& perm,
                                 const std::vector<int32_t>& iperm);

// parallel helpers
int num_threads();
void set_num_threads(int t);

template <class F>
void parallel_for(int64_t n, F&& f, int64_t grain = 4096) {
    int nt = num_threads();
    if (nt <= 1 || n < 2 * grain) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    int64_t chunks = (n + grain - 1) / grain;
    if (chunks < nt) nt = (int)chunks;
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) {
        th.emplace_back([&, t]() {
            int64_t b = n * t / nt, e = n * (t + 1) / nt;
            for (int64_t i = b; i < e; ++i) f(i);
        });
    }
    for (auto& x : th) x.join();
}

// Run f(t) on nt threads, t = 0 .. nt-1 (the calling thread runs t = 0).
template <class F>
void parallel_workers(int nt, F&& f) {
    if (nt <= 1) {
        f(0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) th.emplace_back([&f, t]() { f(t); });
    f(0);
    for (auto& x : th) x.join();
}

// Run f(t, begin, end) over chunks of consecutive indices of [0, n) that up
// to num_threads() threads take from a shared counter (t: the thread,
// 0-based), for loops whose iterations differ widely in cost.  A chunk holds
// about n / (64 threads) indices, at least min_grab.
template <class F>
void parallel_chunks(int64_t n, int64_t min_grab, F&& f) {
    const int64_t grab = std::max<int64_t>(min_grab, n / (64 * (int64_t)num_threads()));
    std::atomic<int64_t> next{0};
    const int nt = (int)std::min<int64_t>(num_threads(), (n + grab - 1) / grab);
    parallel_workers(nt, [&](int t) {
        for (;;) {
            const int64_t b = next.fetch_add(grab);
            if (b >= n) break;
            f(t, b, std::min(n, b + grab));
        }
    });
}

// Run f(t, begin, end) over nt contiguous ranges.
template <class F>
void parallel_ranges(int64_t n, F&& f) {
    int nt = num_threads();
    if (n < 8192) nt = 1;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        int64_t b = n * t / nt, e = n * (t + 1) / nt;
        if (nt == 1) { f(0, b, e); return; }
        th.emplace_back([&f, t, b, e]() { f(t, b, e); });
    }
    for (auto& x : th) x.join();
}

}  // namespace pamg
