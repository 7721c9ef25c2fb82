// Host-side layout checks, run by tests/test_host_layout_cpu.py (CPU only):
//  * the hybrid Gauss-Seidel schedule (gs_schedule): every row's depth is one
//    more than the deepest in-block neighbour before (after) it, each block's
//    largest depths, 1 / a_ii, and the in-block entry ranges (consecutive in
//    the sorted row) agree with a brute-force scan of the row;
//  * the row tiles and column dictionaries of a rectangular CSR matrix
//    (tile_rows, used for the smoothed prolongator's P and P^T): the tiles
//    cover the rows in order within their row and entry limits, and every
//    entry's 16-bit dictionary position names its own column.
// Exit status 0 when every check holds; the first failures are printed.
#include <algorithm>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "common.hpp"

using namespace pamg;

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            if (++failures <= 10) {               \
                std::printf(__VA_ARGS__);         \
                std::printf("\n");                \
            }                                     \
        }                                         \
    } while (0)

// A random CSR with ncols columns; square: the diagonal is stored (positive)
// and the columns cluster around it, like a mesh matrix in a local order.
static void random_csr(std::mt19937& rng, int n, int ncols, bool square, int maxlen, std::vector<int32_t>& rp,
                       std::vector<int32_t>& ci, std::vector<double>& v) {
    rp.assign(n + 1, 0);
    ci.clear();
    v.clear();
    for (int i = 0; i < n; ++i) {
        std::set<int> cols;
        if (square) cols.insert(i);
        const int len = (int)(rng() % (unsigned)maxlen);
        for (int q = 0; q < len; ++q) {
            const int base = square ? i : (int)((long long)i * ncols / n);
            const int j = (rng() % 4 == 0) ? (int)(rng() % (unsigned)ncols)
                                           : (base + (int)(rng() % 61) - 30 + ncols) % ncols;
            cols.insert(j);
        }
        for (int j : cols) {
            ci.push_back(j);
            v.push_back(square && j == i ? 4.0 + (double)(rng() % 100) : -0.01 * (double)(1 + rng() % 50));
        }
        rp[i + 1] = (int32_t)ci.size();
    }
}

static void check_gs(std::mt19937& rng) {
    for (int trial = 0; trial < 30; ++trial) {
        const int n = 1 + (int)(rng() % 1500);
        const int nb = 1 + (int)(rng() % 256);
        LayoutLevel L;
        random_csr(rng, n, n, true, 40, L.rp, L.ci, L.v);
        L.dinv.assign(n, 0.25);
        const GsLevel g = gs_schedule(L, nb);
        const int nblk = (n + nb - 1) / nb;
        CHECK((int)g.maxd.size() == 2 * nblk, "gs trial %d: %zu maxd entries for %d blocks", trial, g.maxd.size(), nblk);
        std::vector<int> df(n), dbk(n);
        for (int p = 0; p < nblk; ++p) {
            const int b0 = p * nb, b1 = std::min(n, b0 + nb);
            int mf = 0, mb = 0;
            for (int i = b0; i < b1; ++i) {
                int d = 0;
                for (int k = L.rp[i]; k < L.rp[i + 1]; ++k)
                    if (L.ci[k] >= b0 && L.ci[k] < i) d = std::max(d, df[L.ci[k]] + 1);
                df[i] = d;
                mf = std::max(mf, d);
            }
            for (int i = b1 - 1; i >= b0; --i) {
                int d = 0;
                for (int k = L.rp[i]; k < L.rp[i + 1]; ++k)
                    if (L.ci[k] > i && L.ci[k] < b1) d = std::max(d, dbk[L.ci[k]] + 1);
                dbk[i] = d;
                mb = std::max(mb, d);
            }
            CHECK(g.maxd[2 * p] == mf && g.maxd[2 * p + 1] == mb, "gs trial %d block %d: largest depths", trial, p);
            for (int i = b0; i < b1; ++i) {
                CHECK(g.depth_f[i] == df[i] && g.depth_b[i] == dbk[i], "gs trial %d row %d: depth", trial, i);
                std::vector<int> before, after;
                double aii = 0.0;
                for (int k = L.rp[i]; k < L.rp[i + 1]; ++k) {
                    const int j = L.ci[k];
                    if (j >= b0 && j < i) before.push_back(k);
                    if (j > i && j < b1) after.push_back(k);
                    if (j == i) aii = L.v[k];
                }
                const int f0 = g.fresh[2 * (size_t)i], y = g.fresh[2 * (size_t)i + 1];
                const int nbf = y & 0xff, naf = (y >> 8) & 0xff, diag = (y >> 16) & 1;
                std::vector<int> before2, after2;
                for (int u = 0; u < nbf; ++u) before2.push_back(f0 + u);
                for (int u = 0; u < naf; ++u) after2.push_back(f0 + nbf + diag + u);
                CHECK(before == before2 && after == after2 && diag == 1, "gs trial %d row %d: in-block range", trial, i);
                CHECK(g.ainv[i] == 1.0 / aii, "gs trial %d row %d: 1 / a_ii", trial, i);
            }
        }
    }
}

static int dict_items_seen = 0;

static void check_tiles(std::mt19937& rng) {
    for (int trial = 0; trial < 33; ++trial) {
        // small matrices (one-row tiles of 256 entries and rows longer than
        // that), then large ones whose tiles carry dictionaries (8 and 16
        // entries per thread)
        const bool big = trial >= 30;
        const int n = big ? 60000 + 40000 * (trial - 30) : 1 + (int)(rng() % 3000);
        const int ncols = big ? n / 2 : 1 + (int)(rng() % 3000);
        const int maxlen = big ? 90 : (trial % 3 == 0 ? 600 : 60);
        std::vector<int32_t> rp, ci;
        std::vector<double> v;
        random_csr(rng, n, ncols, false, maxlen, rp, ci, v);
        const TiledRows T = tile_rows(rp, ci, n, ncols);
        const int cap = T.items * kBlock;
        CHECK(T.items >= 1 && T.items <= kMaxItems && (T.items & (T.items - 1)) == 0, "tiles trial %d: items %d",
              trial, T.items);
        const int nt = (int)T.tiles.size() / 4;
        int next_row = 0;
        for (int t = 0; t < nt; ++t) {
            const int k0 = T.tiles[4 * t], k1 = T.tiles[4 * t + 1], r0 = T.tiles[4 * t + 2], r1 = T.tiles[4 * t + 3];
            CHECK(r0 == next_row && r1 > r0 && r1 <= n, "tiles trial %d tile %d: rows %d..%d", trial, t, r0, r1);
            CHECK(k0 == rp[r0] && k1 == rp[r1], "tiles trial %d tile %d: entry range", trial, t);
            CHECK(r1 - r0 <= kTileRows, "tiles trial %d tile %d: %d rows", trial, t, r1 - r0);
            CHECK(k1 - k0 <= cap || r1 - r0 == 1, "tiles trial %d tile %d: %d entries over %d", trial, t, k1 - k0, cap);
            next_row = r1;
            if (T.items >= kDictItems && k1 - k0 <= cap) {
                const int s0 = T.dict.span[2 * t], len = T.dict.span[2 * t + 1];
                std::set<int> cols(ci.begin() + k0, ci.begin() + k1);
                std::vector<int> d(T.dict.col.begin() + s0, T.dict.col.begin() + s0 + len);
                CHECK(std::vector<int>(cols.begin(), cols.end()) == d, "tiles trial %d tile %d: dictionary", trial, t);
                for (int k = k0; k < k1; ++k)
                    CHECK(T.dict.local[k] < len && d[T.dict.local[k]] == ci[k], "tiles trial %d entry %d: position",
                          trial, k);
                CHECK(len <= T.dict.max_len, "tiles trial %d tile %d: longest dictionary", trial, t);
            }
        }
        CHECK(next_row == n, "tiles trial %d: rows covered up to %d of %d", trial, next_row, n);
        if (big) {
            CHECK(T.items >= kDictItems, "tiles trial %d: %lld entries gave %d items", trial, (long long)rp[n], T.items);
            dict_items_seen |= T.items;
        }
        if (T.items == kMaxItems) CHECK(T.dict.max_len <= kDictMaxLarge, "tiles trial %d: dictionary too long", trial);
    }
}

int main() {
    std::mt19937 rng(20260312);
    check_gs(rng);
    check_tiles(rng);
    CHECK((dict_items_seen & kMaxItems) && (dict_items_seen & kDictItems), "dictionary tile sizes seen: %d",
          dict_items_seen);
    std::printf("%d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
