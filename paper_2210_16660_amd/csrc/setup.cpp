// Host construction of the AMG hierarchy (arXiv 2210.16660, Sec. 3.1).
//
// Compiled with -ffp-contract=off: every floating-point expression below is
// evaluated one IEEE binary64 operation at a time, in the written order, so
// that weights, prolongator entries and Galerkin sums are bitwise
// reproducible.  The definitions followed (canonical numbering):
//   * l1 diagonal d_i = sum_j |a_ij| (ascending columns); dinv = 1/d.
//   * edge weight of eq. (weights) for a stored upper entry (lo, hi):
//       num = ((2 a_lohi) w_lo) w_hi, den = (a_lolo w_lo) w_lo + (a_hihi w_hi) w_hi,
//       c = 1 - num/den;  an edge may be matched iff c > 1.
//   * matching: the greedy matching under the strict order (c desc, lo asc,
//     hi asc), which is what eq. (approximatematch) approximates within 1/2.
//     Computed here with the parallel Suitor algorithm (Manne & Halappanavar,
//     IPDPS 2014), which yields exactly the greedy matching for a strict
//     total order on the edges.
//   * aggregates: matched pairs and singletons, numbered by smallest member.
//   * tentative prolongator of eq. (prolongator): pair: nu = sqrt(w_lo^2 + w_hi^2),
//     p = w/nu, w_c = nu; singleton: p = w/|w|, w_c = |w|.
//   * Galerkin A_{l+1} = P^T A P: entry (I, J) is the sum of a_ij (p_i p_j)
//     over stored (i, j) with agg(i) = I, agg(j) = J, added left to right in
//     ascending (min(i,j), max(i,j), i); structural zeros are kept.
//   * coarsen while n_l > max_coarse; a level without pairs is the coarsest,
//     and so is a level within the dense limit whose matching would shrink it
//     by less than min_ratio (stalled coarsening).
//   * the coarsest matrix is factorized on the device (Cholesky and explicit
//     inverse, dense.hip).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "common.hpp"

namespace pamg {

static thread_local int g_threads = 0;

int num_threads() {
    if (g_threads > 0) return g_threads;
    unsigned h = std::thread::hardware_concurrency();
    return h == 0 ? 1 : (int)std::min(h, 64u);
}
void set_num_threads(int t) { g_threads = t; }

std::string csr_error(int code, int64_t row) {
    static const char* msg[] = {"", "row_ptr not monotone", "column index out of range",
                                "columns not strictly ascending", "non-positive diagonal",
                                "missing diagonal entry", "non-finite value"};
    return std::string(msg[code]) + " in row " + std::to_string(row);
}

// The checks of validate_csr that read no row (pointers, sizes, row_ptr ends).
void validate_csr_header(const pamg_csr& A) {
    if (A.n <= 0) throw Error(PAMG_E_INVALID, "n must be positive");
    if (!A.row_ptr || !A.col_idx || !A.val) throw Error(PAMG_E_INVALID, "null CSR pointer");
    if (A.nnz < A.n || A.nnz >= (int64_t(1) << 31)) throw Error(PAMG_E_INVALID, "nnz out of range (need n <= nnz < 2^31)");
    if (A.row_ptr[0] != 0 || A.row_ptr[A.n] != A.nnz) throw Error(PAMG_E_INVALID, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
}

void validate_csr(const pamg_csr& A, bool check_symmetry) {
    validate_csr_header(A);
    // the smallest failing row and its check, as (row << 8) | check
    std::atomic<int64_t> first{INT64_MAX};
    parallel_for(A.n, [&](int64_t i) {
        int32_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
        int err = 0;
        if (e < b || b < 0 || e > A.nnz) err = 1;   // no entry of such a row is read
        bool diag = false;
        for (int32_t k = b; k < e && !err; ++k) {
            int32_t c = A.col_idx[k];
            if (c < 0 || c >= A.n) err = 2;
            else if (k > b && c <= A.col_idx[k - 1]) err = 3;
            else if (c == i) {
                diag = true;
                if (!(A.val[k] > 0.0)) err = 4;
            }
            if (!std::isfinite(A.val[k])) err = 6;
        }
        if (!err && !diag) err = 5;
        if (err) {
            const int64_t key = (i << 8) | err;
            int64_t cur = first.load();
            while (key < cur && !first.compare_exchange_weak(cur, key)) {
            }
        }
    });
    if (first.load() != INT64_MAX) throw Error(PAMG_E_INVALID, csr_error((int)(first.load() & 0xff), first.load() >> 8));
    if (check_symmetry) {
        std::atomic<int> asym{0};
        parallel_for(A.n, [&](int64_t i) {
            for (int32_t k = A.row_ptr[i]; k < A.row_ptr[i + 1]; ++k) {
                int32_t j = A.col_idx[k];
                const int32_t* b = A.col_idx + A.row_ptr[j];
                const int32_t* e = A.col_idx + A.row_ptr[j + 1];
                const int32_t* f = std::lower_bound(b, e, (int32_t)i);
                if (f == e || *f != i || std::memcmp(&A.val[f - A.col_idx], &A.val[k], 8) != 0) asym.store(1);
            }
        });
        if (asym.load()) throw Error(PAMG_E_INVALID, "matrix is not bitwise symmetric");
    }
}

// ---------------------------------------------------------------- weights

static inline double edge_weight(double a_lohi, double a_lolo, double a_hihi, double w_lo, double w_hi) {
    double num = ((2.0 * a_lohi) * w_lo) * w_hi;
    double den = (a_lolo * w_lo) * w_lo + (a_hihi * w_hi) * w_hi;
    return 1.0 - num / den;
}

// strict total order on edges: true if (c1, lo1, hi1) is heavier than (c2, lo2, hi2)
static inline bool heavier(double c1, int32_t lo1, int32_t hi1, double c2, int32_t lo2, int32_t hi2) {
    if (c1 != c2) return c1 > c2;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

struct Adj {
    std::vector<int64_t> ptr;    // n+1
    std::vector<int32_t> nbr;
    std::vector<double> c;
};

// Eligible edges of the graph of A with their weights, both directions,
// each vertex's list sorted heaviest first.
static Adj eligible_adjacency(const HostCSR& A, const std::vector<double>& diag, const std::vector<double>& w,
                              bool match_all) {
    const int32_t n = A.n;
    Adj g;
    std::vector<int32_t> deg(n, 0);
    // upper entries: eligible flag per stored entry (both arrays written
    // here for every entry, first touched by the threads; a weight is read
    // only where its flag is set)
    std::unique_ptr<double[]> cval(new double[A.nnz()]);
    std::unique_ptr<uint8_t[]> elig(new uint8_t[A.nnz()]);
    parallel_for(n, [&](int64_t i) {
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            int32_t j = A.ci[k];
            if (j <= i) {
                cval[k] = 0.0;
                elig[k] = 0;
                continue;
            }
            double c = edge_weight(A.v[k], diag[i], diag[j], w[i], w[j]);
            cval[k] = c;
            elig[k] = (match_all || c > 1.0) ? 1 : 0;
        }
    });
    // degree count (both endpoints) and fill, rows over threads with atomic
    // counters: the order in which a vertex's list is filled does not
    // matter, since the list is then sorted under a strict total order
    // (weight, then the lower and the higher endpoint)
    parallel_for(n, [&](int64_t i) {
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (elig[k]) {
                __atomic_fetch_add(&deg[i], 1, __ATOMIC_RELAXED);
                __atomic_fetch_add(&deg[A.ci[k]], 1, __ATOMIC_RELAXED);
            }
    });
    g.ptr.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) g.ptr[i + 1] = g.ptr[i] + deg[i];
    g.nbr.resize(g.ptr[n]);
    g.c.resize(g.ptr[n]);
    std::vector<int64_t> pos(g.ptr.begin(), g.ptr.end() - 1);
    parallel_for(n, [&](int64_t i) {
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (elig[k]) {
                const int32_t j = A.ci[k];
                const int64_t pi = __atomic_fetch_add(&pos[i], 1, __ATOMIC_RELAXED);
                const int64_t pj = __atomic_fetch_add(&pos[j], 1, __ATOMIC_RELAXED);
                g.nbr[pi] = j;
                g.c[pi] = cval[k];
                g.nbr[pj] = (int32_t)i;
                g.c[pj] = cval[k];
            }
    });
    struct alignas(64) SortBuf {  // one cache line (or more) per thread
        std::vector<std::pair<double, int32_t>> t;
    };
    std::vector<SortBuf> buf(num_threads());
    parallel_chunks(n, 1024, [&](int th, int64_t rb, int64_t re) {
        std::vector<std::pair<double, int32_t>>& t = buf[th].t;
        for (int64_t i = rb; i < re; ++i) {
            int64_t b = g.ptr[i], e = g.ptr[i + 1];
            if (e - b < 2) continue;
            t.clear();
            for (int64_t k = b; k < e; ++k) t.emplace_back(g.c[k], g.nbr[k]);
            int32_t u = (int32_t)i;
            std::sort(t.begin(), t.end(), [u](const std::pair<double, int32_t>& x, const std::pair<double, int32_t>& y) {
                return heavier(x.first, std::min(u, x.second), std::max(u, x.second),
                               y.first, std::min(u, y.second), std::max(u, y.second));
            });
            for (int64_t k = b; k < e; ++k) { g.c[k] = t[k - b].first; g.nbr[k] = t[k - b].second; }
        }
    });
    return g;
}

// Parallel Suitor matching.  mate[i] = partner or -1; returns number of pairs.
static int64_t suitor_matching(const Adj& g, int32_t n, std::vector<int32_t>& mate) {
    std::vector<int32_t> suitor(n, -1);
    std::vector<double> ws(n, 0.0);                 // weight of the suitor's edge (valid if suitor >= 0)
    std::unique_ptr<std::atomic<uint8_t>[]> lock(new std::atomic<uint8_t>[n]);
    for (int32_t i = 0; i < n; ++i) lock[i].store(0, std::memory_order_relaxed);
    std::vector<int64_t> next(g.ptr.begin(), g.ptr.end() - 1);   // scan position per vertex

    auto propose = [&](int32_t u0) {
        int32_t cur = u0;
        while (cur >= 0) {
            int32_t displaced = -1;
            bool placed = false;
            for (int64_t k = next[cur]; k < g.ptr[cur + 1]; ++k) {
                int32_t v = g.nbr[k];
                double c = g.c[k];
                int32_t lo = std::min(cur, v), hi = std::max(cur, v);
                while (lock[v].exchange(1, std::memory_order_acquire)) { }
                int32_t s = suitor[v];
                bool beats = (s < 0) || heavier(c, lo, hi, ws[v], std::min(s, v), std::max(s, v));
                if (beats) {
                    displaced = s;
                    suitor[v] = cur;
                    ws[v] = c;
                    // publish the scan position before cur can be displaced by another thread
                    next[cur] = k + 1;
                }
                lock[v].store(0, std::memory_order_release);
                if (beats) { placed = true; break; }
            }
            if (!placed) next[cur] = g.ptr[cur + 1];
            cur = placed ? displaced : -1;
        }
    };
    parallel_ranges(n, [&](int, int64_t b, int64_t e) {
        for (int64_t u = b; u < e; ++u) propose((int32_t)u);
    });
    int64_t pairs = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t s = suitor[i];
        mate[i] = (s >= 0 && suitor[s] == i) ? s : -1;
        if (mate[i] > i) ++pairs;
    }
    return pairs;
}

// ---------------------------------------------------------------- Galerkin

struct Term {
    int32_t J, k1, k2, k3;
    double t;
};

static void galerkin(const HostCSR& A, const std::vector<int32_t>& agg, const std::vector<double>& p,
                     const std::vector<int32_t>& mem_ptr, const std::vector<int32_t>& mem, HostCSR& Ac) {
    const int32_t nc = (int32_t)mem_ptr.size() - 1;
    auto row_terms = [&](int32_t I, std::vector<Term>& t) {
        t.clear();
        for (int32_t q = mem_ptr[I]; q < mem_ptr[I + 1]; ++q) {
            int32_t i = mem[q];
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                int32_t j = A.ci[k];
                Term x;
                x.J = agg[j];
                x.k1 = std::min(i, j);
                x.k2 = std::max(i, j);
                x.k3 = i;
                x.t = A.v[k] * (p[i] * p[j]);
                t.push_back(x);
            }
        }
        std::sort(t.begin(), t.end(), [](const Term& a, const Term& b) {
            if (a.J != b.J) return a.J < b.J;
            if (a.k1 != b.k1) return a.k1 < b.k1;
            if (a.k2 != b.k2) return a.k2 < b.k2;
            return a.k3 < b.k3;
        });
    };
    // coarse rows in chunks from a shared counter: near the coarsest level the
    // rows are few and long
    constexpr int64_t kGrab = 16;
    struct alignas(64) Scratch {  // one cache line (or more) per thread
        std::vector<Term> t;
    };
    std::vector<Scratch> scratch(num_threads());
    std::vector<int32_t> cnt(nc, 0);
    parallel_chunks(nc, kGrab, [&](int th, int64_t b, int64_t e) {
        std::vector<Term>& t = scratch[th].t;
        for (int64_t I = b; I < e; ++I) {
            row_terms((int32_t)I, t);
            int32_t d = 0;
            for (size_t s = 0; s < t.size(); ++s)
                if (s == 0 || t[s].J != t[s - 1].J) ++d;
            cnt[I] = d;
        }
    });
    Ac.n = nc;
    Ac.rp.assign(nc + 1, 0);
    for (int32_t I = 0; I < nc; ++I) {
        int64_t nx = (int64_t)Ac.rp[I] + cnt[I];
        if (nx >= (int64_t(1) << 31)) throw Error(PAMG_E_OOM, "coarse matrix exceeds 2^31 entries");
        Ac.rp[I + 1] = (int32_t)nx;
    }
    Ac.ci.resize(Ac.rp[nc]);
    Ac.v.resize(Ac.rp[nc]);
    parallel_chunks(nc, kGrab, [&](int th, int64_t b, int64_t e) {
        std::vector<Term>& t = scratch[th].t;
        for (int64_t I = b; I < e; ++I) {
            row_terms((int32_t)I, t);
            int32_t q = Ac.rp[I] - 1;
            for (size_t s = 0; s < t.size(); ++s) {
                if (s == 0 || t[s].J != t[s - 1].J) {
                    ++q;
                    Ac.ci[q] = t[s].J;
                    Ac.v[q] = t[s].t;
                } else {
                    Ac.v[q] = Ac.v[q] + t[s].t;
                }
            }
        }
    });
}

// ------------------------------------------------ smoothed prolongator

// P = (I - omega D^-1 A) P^ (Sec. 3.1), D = diag(A), omega = 1/||D^-1 A||_inf.
// Row i: P_iJ = [J = agg(i)] p_i - sum_{j: agg(j) = J} (omega (a_ij / a_ii)) p_j,
// subtracted in ascending j; pattern {agg(j) : a_ij stored}, ascending.
static void smoothed_prolongator(const HostCSR& A, const std::vector<int32_t>& agg, const std::vector<double>& p,
                                 HostCSR& P, double& omega) {
    const int32_t n = A.n;
    // the rows of a coarse level are long: small levels are split too
    constexpr int64_t kSmoothGrain = 64;
    std::vector<double> ratio(n);
    parallel_for(n, [&](int64_t i) {
        double s = 0.0, aii = 0.0;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            s += std::fabs(A.v[k]);
            if (A.ci[k] == i) aii = A.v[k];
        }
        ratio[i] = s / aii;
    }, kSmoothGrain);
    double mx = 0.0;
    for (int32_t i = 0; i < n; ++i)
        if (ratio[i] > mx) mx = ratio[i];
    omega = 1.0 / mx;
    const double om = omega;
    std::vector<std::vector<int32_t>> cols(n);
    std::vector<std::vector<double>> vals(n);
    parallel_for(n, [&](int64_t i) {
        std::vector<int32_t>& c = cols[i];
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) c.push_back(agg[A.ci[k]]);
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        std::vector<double>& v = vals[i];
        v.assign(c.size(), 0.0);
        double aii = 0.0;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] == i) aii = A.v[k];
        for (size_t u = 0; u < c.size(); ++u) v[u] = c[u] == agg[i] ? p[i] : 0.0;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.ci[k];
            const size_t u = std::lower_bound(c.begin(), c.end(), agg[j]) - c.begin();
            v[u] = v[u] - (om * (A.v[k] / aii)) * p[j];
        }
    }, kSmoothGrain);
    P.n = n;
    P.rp.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) P.rp[i + 1] = P.rp[i] + (int32_t)cols[i].size();
    P.ci.resize(P.rp[n]);
    P.v.resize(P.rp[n]);
    parallel_for(n, [&](int64_t i) {
        std::copy(cols[i].begin(), cols[i].end(), P.ci.begin() + P.rp[i]);
        std::copy(vals[i].begin(), vals[i].end(), P.v.begin() + P.rp[i]);
    });
}

// Rows of a sparse product accumulated in a fixed order: out row r =
// sum over the listed (coefficient, source row) pairs, in list order, of
// coefficient * source row; keep(J) filters the columns; 0.0 starts each sum.
// Rows are built by `emit(r, visit)` where visit(coef, row_ptr, row_col, row_val).
template <class Emit>
static void accumulate_rows(int32_t nrows, int32_t ncols, Emit emit, HostCSR& out) {
    std::vector<std::vector<int32_t>> cols(nrows);
    std::vector<std::vector<double>> vals(nrows);
    // rows taken kGrab at a time from a shared counter: the rows of a coarse
    // smoothed level are long and few, so equal row ranges (or one thread
    // for a small level) leave most threads idle; each row is still summed by
    // one thread in list order
    constexpr int64_t kGrab = 16;
    struct alignas(64) Scratch {  // one cache line (or more) per thread
        std::vector<double> acc;
        std::vector<int32_t> mark, list;
    };
    std::vector<Scratch> scratch(num_threads());
    parallel_chunks(nrows, kGrab, [&](int th, int64_t b, int64_t e) {
        Scratch& S = scratch[th];
        if (S.mark.empty()) {
            S.acc.assign(ncols, 0.0);
            S.mark.assign(ncols, -1);
        }
        std::vector<double>& acc = S.acc;
        std::vector<int32_t>& mark = S.mark;
        std::vector<int32_t>& list = S.list;
        for (int64_t r = b; r < e; ++r) {
            list.clear();
            emit((int32_t)r, [&](int32_t J, double term) {
                if (mark[J] != r) {
                    mark[J] = (int32_t)r;
                    acc[J] = 0.0;
                    list.push_back(J);
                }
                acc[J] = acc[J] + term;
            });
            std::sort(list.begin(), list.end());
            cols[r] = list;
            vals[r].resize(list.size());
            for (size_t u = 0; u < list.size(); ++u) vals[r][u] = acc[list[u]];
        }
    });
    out.n = nrows;
    out.rp.assign(nrows + 1, 0);
    for (int32_t r = 0; r < nrows; ++r) {
        const int64_t nx = (int64_t)out.rp[r] + (int64_t)cols[r].size();
        if (nx >= (int64_t(1) << 31)) throw Error(PAMG_E_OOM, "smoothed Galerkin product exceeds 2^31 entries");
        out.rp[r + 1] = (int32_t)nx;
    }
    out.ci.resize(out.rp[nrows]);
    out.v.resize(out.rp[nrows]);
    parallel_for(nrows, [&](int64_t r) {
        std::copy(cols[r].begin(), cols[r].end(), out.ci.begin() + out.rp[r]);
        std::copy(vals[r].begin(), vals[r].end(), out.v.begin() + out.rp[r]);
    });
}

// Out row J lists (i, v_iJ) over the stored entries (i, J) of rows 0..n-1
// that keep(i, J) accepts, i ascending: a stable counting sort by column over
// contiguous row ranges, one per thread, each thread filling its own slots
// (column J holds thread 0's rows first, then thread 1's, ...).
template <class Keep>
static void transpose_rows(int32_t n, int32_t m, const int32_t* rp, const int32_t* ci, const double* v, Keep keep,
                           std::vector<int32_t>& orp, std::vector<int32_t>& oci, std::vector<double>& ov) {
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(num_threads(), n / 1024));
    std::vector<std::vector<int32_t>> slot(nt);
    auto rows_of = [&](int t, int64_t& b, int64_t& e) {
        b = (int64_t)n * t / nt;
        e = (int64_t)n * (t + 1) / nt;
    };
    parallel_workers(nt, [&](int t) {
        int64_t b, e;
        rows_of(t, b, e);
        std::vector<int32_t>& c = slot[t];
        c.assign(m, 0);
        for (int64_t i = b; i < e; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (keep((int32_t)i, ci[k])) ++c[ci[k]];
    });
    orp.assign(m + 1, 0);
    for (int32_t J = 0; J < m; ++J) {
        int64_t at = orp[J];
        for (int t = 0; t < nt; ++t) {
            const int32_t c = slot[t][J];
            slot[t][J] = (int32_t)at;
            at += c;
        }
        if (at >= (int64_t(1) << 31)) throw Error(PAMG_E_OOM, "transposed matrix exceeds 2^31 entries");
        orp[J + 1] = (int32_t)at;
    }
    oci.resize(orp[m]);
    ov.resize(orp[m]);
    parallel_workers(nt, [&](int t) {
        int64_t b, e;
        rows_of(t, b, e);
        std::vector<int32_t>& pos = slot[t];
        for (int64_t i = b; i < e; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t J = ci[k];
                if (!keep((int32_t)i, J)) continue;
                oci[pos[J]] = (int32_t)i;
                ov[pos[J]] = v[k];
                ++pos[J];
            }
    });
}

// A_c = P^T A P: B = A P (B_kJ = 0.0 + sum over j ascending of a_kj P_jJ), then
// for I <= J: A_c[I,J] = 0.0 + sum over i ascending of P_iI B_iJ; mirrored.
static void galerkin_smoothed(const HostCSR& A, const HostCSR& P, int32_t nc, HostCSR& Ac) {
    const int32_t n = A.n;
    HostCSR B;
    accumulate_rows(n, nc, [&](int32_t k, auto&& add) {
        for (int32_t e = A.rp[k]; e < A.rp[k + 1]; ++e) {
            const int32_t j = A.ci[e];
            for (int32_t u = P.rp[j]; u < P.rp[j + 1]; ++u) add(P.ci[u], A.v[e] * P.v[u]);
        }
    }, B);
    // P^T: rows I, entries (i, P_iI) with i ascending
    std::vector<int32_t> tp, ti;
    std::vector<double> tv;
    transpose_rows(n, nc, P.rp.data(), P.ci.data(), P.v.data(), [](int32_t, int32_t) { return true; }, tp, ti, tv);
    HostCSR U;
    accumulate_rows(nc, nc, [&](int32_t I, auto&& add) {
        for (int32_t x = tp[I]; x < tp[I + 1]; ++x) {
            const int32_t i = ti[x];
            for (int32_t u = B.rp[i]; u < B.rp[i + 1]; ++u)
                if (B.ci[u] >= I) add(B.ci[u], tv[x] * B.v[u]);
        }
    }, U);
    // full rows: mirrored entries (ascending source row), then the upper row
    std::vector<int32_t> mp, mi;
    std::vector<double> mv;
    transpose_rows(nc, nc, U.rp.data(), U.ci.data(), U.v.data(), [](int32_t I, int32_t J) { return J != I; }, mp, mi,
                   mv);
    Ac.n = nc;
    Ac.rp.assign(nc + 1, 0);
    for (int32_t I = 0; I < nc; ++I) {
        const int64_t nx = (int64_t)Ac.rp[I] + (mp[I + 1] - mp[I]) + (U.rp[I + 1] - U.rp[I]);
        if (nx >= (int64_t(1) << 31)) throw Error(PAMG_E_OOM, "coarse matrix exceeds 2^31 entries");
        Ac.rp[I + 1] = (int32_t)nx;
    }
    Ac.ci.resize(Ac.rp[nc]);
    Ac.v.resize(Ac.rp[nc]);
    parallel_for(nc, [&](int64_t I) {
        int32_t q = Ac.rp[I];
        for (int32_t u = mp[I]; u < mp[I + 1]; ++u, ++q) {
            Ac.ci[q] = mi[u];
            Ac.v[q] = mv[u];
        }
        for (int32_t u = U.rp[I]; u < U.rp[I + 1]; ++u, ++q) {
            Ac.ci[q] = U.ci[u];
            Ac.v[q] = U.v[u];
        }
    }, 256);
}

// ------------------------------------------ aggregate-size composition

// Keep levels 0, s, 2s, ... and the coarsest of the pairwise hierarchy; the
// prolongator between kept levels is the product of the pairwise ones in
// between (Sec. 3.1): agg follows the chain, p is multiplied finest first.
void compose_levels(HostHierarchy& H, int s) {
    const int L = (int)H.lev.size() - 1;
    std::vector<int> kept;
    for (int l = 0; l < L; l += s) kept.push_back(l);
    kept.push_back(L);
    std::vector<HostLevel> out(kept.size());
    for (size_t j = 0; j < kept.size(); ++j) {
        const int a = kept[j];
        HostLevel& o = out[j];
        o.A = std::move(H.lev[a].A);
        o.w = std::move(H.lev[a].w);
        o.dinv = std::move(H.lev[a].dinv);
        o.pairs = H.lev[a].pairs;
        if (j + 1 == kept.size()) break;
        const int b = kept[j + 1];
        const int32_t n = o.A.n;
        o.agg.resize(n);
        o.p.resize(n);
        parallel_for(n, [&](int64_t i) {
            int32_t I = H.lev[a].agg[i];
            double pc = H.lev[a].p[i];
            for (int m = a + 1; m < b; ++m) {
                pc = pc * H.lev[m].p[I];
                I = H.lev[m].agg[I];
            }
            o.agg[i] = I;
            o.p[i] = pc;
        });
    }
    // the pairwise chain stays behind the kept levels (coefficient-only reuse)
    H.chain.assign(L + 1, PairLevel());
    for (size_t j = 0; j < kept.size(); ++j) H.chain[kept[j]].kept = (int32_t)j;
    for (int m = 0; m <= L; ++m) {
        PairLevel& c = H.chain[m];
        if (c.kept < 0) {
            c.S.n = H.lev[m].A.n;
            c.S.rp = std::move(H.lev[m].A.rp);
            c.S.ci = std::move(H.lev[m].A.ci);
        }
        c.agg = std::move(H.lev[m].agg);
        c.p = std::move(H.lev[m].p);
    }
    H.lev = std::move(out);
}

// ------------------------------- smoothed prolongators with composition

// One pairwise step on A with near-null vector w: matching, stop rules and
// aggregates, as in the pairwise loop of build_hierarchy.  False when A is
// the coarsest level.
struct PairStepOut {
    std::vector<int32_t> agg, mem_ptr, mem;
    std::vector<double> p, wc;
    int32_t nc = 0;
    int64_t pairs = 0;
};

static bool pairwise_step(const HostCSR& A, const std::vector<double>& w, const pamg_params& prm, PairStepOut& o) {
    const int32_t n = A.n;
    std::vector<double> diag(n, 0.0);
    parallel_for(n, [&](int64_t i) {
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
            if (A.ci[k] == i) diag[i] = A.v[k];
    });
    Adj g = eligible_adjacency(A, diag, w, prm.match_all_edges != 0);
    std::vector<int32_t> mate(n, -1);
    const int64_t pairs = suitor_matching(g, n, mate);
    if (pairs == 0) return false;
    if (n <= prm.max_dense && (double)n < prm.min_ratio * (double)(n - pairs)) return false;
    o.pairs = pairs;
    o.agg.assign(n, -1);
    o.p.assign(n, 0.0);
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (mate[i] < 0 || mate[i] > i) ++nc;
    o.nc = nc;
    o.wc.resize(nc);
    o.mem_ptr.resize(nc + 1);
    o.mem.resize(n);
    int32_t I = 0, q = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t m = mate[i];
        if (m >= 0 && m < i) continue;
        o.mem_ptr[I] = q;
        if (m < 0) {
            o.agg[i] = I;
            o.p[i] = w[i] / std::fabs(w[i]);
            o.wc[I] = std::fabs(w[i]);
            o.mem[q++] = i;
        } else {
            const double nu = std::sqrt(w[i] * w[i] + w[m] * w[m]);
            o.agg[i] = I;
            o.agg[m] = I;
            o.p[i] = w[i] / nu;
            o.p[m] = w[m] / nu;
            o.wc[I] = nu;
            o.mem[q++] = i;
            o.mem[q++] = m;
        }
        ++I;
    }
    o.mem_ptr[nc] = q;
    return true;
}

// Kept levels one at a time: from kept level K, up to s pairwise steps
// (tentative Galerkin products between them) give K's composed aggregates and
// p (finest first); K's prolongator is the composed tentative one smoothed
// with K, and the next kept level is P^T K P.
static void build_smoothed_composed(HostHierarchy& H, const pamg_params& prm) {
    const int s = prm.agg_steps;
    for (int j = 0;; ++j) {
        {
            HostLevel& K = H.lev[j];
            const HostCSR& A = K.A;
            K.dinv.resize(A.n);
            parallel_for(A.n, [&](int64_t i) {
                double d = 0.0;
                for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) d += std::fabs(A.v[k]);
                K.dinv[i] = 1.0 / d;
            });
            if (A.n <= prm.max_coarse || j + 1 >= prm.max_levels) break;
        }
        const HostCSR& KA = H.lev[j].A;
        const int32_t n = KA.n;
        std::vector<int32_t> cagg;
        std::vector<double> cp, wcur = H.lev[j].w;
        const HostCSR* C = &KA;
        HostCSR own;
        int steps = 0;
        int32_t nc = 0;
        int64_t first_pairs = 0;
        for (int m = 0; m < s; ++m) {
            if (m > 0 && C->n <= prm.max_coarse) break;
            PairStepOut o;
            if (!pairwise_step(*C, wcur, prm, o)) break;
            if (m == 0) {
                first_pairs = o.pairs;
                cagg = o.agg;
                cp = o.p;
            } else {
                parallel_for(n, [&](int64_t i) {
                    const int32_t I = cagg[i];
                    cp[i] = cp[i] * o.p[I];
                    cagg[i] = o.agg[I];
                });
            }
            nc = o.nc;
            HostCSR next;
            if (m + 1 < s)
                galerkin(*C, o.agg, o.p, o.mem_ptr, o.mem, next);
            else
                next.n = nc;
            own = std::move(next);
            C = &own;
            wcur = std::move(o.wc);
            ++steps;
        }
        if (steps == 0) break;
        HostLevel next;
        {
            HostLevel& K = H.lev[j];
            K.pairs = (int32_t)first_pairs;
            K.agg = std::move(cagg);
            K.p = std::move(cp);
            smoothed_prolongator(K.A, K.agg, K.p, K.P, K.omega_p);
            galerkin_smoothed(K.A, K.P, nc, next.A);
        }
        next.w = std::move(wcur);
        H.lev.push_back(std::move(next));
    }
}

// ---------------------------------------------------------------- driver

HostHierarchy build_hierarchy(const pamg_csr& Ain, const pamg_params& prm) {
    HostHierarchy H;
    H.lev.emplace_back();
    {
        HostLevel& L0 = H.lev[0];
        L0.A.n = Ain.n;
        L0.A.rp.assign(Ain.row_ptr, Ain.row_ptr + Ain.n + 1);
        L0.A.ci.assign(Ain.col_idx, Ain.col_idx + Ain.nnz);
        L0.A.v.assign(Ain.val, Ain.val + Ain.nnz);
        L0.w.assign(Ain.n, 1.0);
    }
    if (prm.smooth_prolongator && prm.agg_steps > 1) {
        build_smoothed_composed(H, prm);
        if (H.lev.back().A.n > prm.max_dense)
            throw Error(PAMG_E_STALLED, "coarsening stalled at " + std::to_string(H.lev.back().A.n) +
                                            " unknowns, above the dense-solve limit");
        return H;
    }
    extend_hierarchy(H, prm);
    const HostCSR& AL = H.lev.back().A;
    if (AL.n > prm.max_dense)
        throw Error(PAMG_E_STALLED, "coarsening stalled at " + std::to_string(AL.n) +
                                        " unknowns, above the dense-solve limit");
    if (prm.agg_steps > 1) compose_levels(H, prm.agg_steps);
    return H;
}

// The pairwise loop of build_hierarchy from the last level of H (its A and w
// set): l1 diagonal, matching, stop rules, aggregates, Galerkin product.  The
// levels of H count towards max_levels.
void extend_hierarchy(HostHierarchy& H, const pamg_params& prm) {
    for (int l = (int)H.lev.size() - 1;; ++l) {
        HostLevel& cur = H.lev[l];
        const HostCSR& A = cur.A;
        const int32_t n = A.n;
        std::vector<double> diag(n, 0.0);
        cur.dinv.resize(n);
        parallel_for(n, [&](int64_t i) {
            double d = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                d += std::fabs(A.v[k]);
                if (A.ci[k] == i) diag[i] = A.v[k];
            }
            cur.dinv[i] = 1.0 / d;
        });
        if (n <= prm.max_coarse || l + 1 >= prm.max_levels) break;
        Adj g = eligible_adjacency(A, diag, cur.w, prm.match_all_edges != 0);
        std::vector<int32_t> mate(n, -1);
        int64_t pairs = suitor_matching(g, n, mate);
        if (pairs == 0) break;
        // too little reduction on a level the dense solve can take: coarsest
        if (n <= prm.max_dense && (double)n < prm.min_ratio * (double)(n - pairs)) break;
        cur.pairs = (int32_t)pairs;
        // aggregates numbered by smallest member
        cur.agg.assign(n, -1);
        cur.p.assign(n, 0.0);
        int32_t nc = 0;
        for (int32_t i = 0; i < n; ++i)
            if (mate[i] < 0 || mate[i] > i) ++nc;
        std::vector<double> wc(nc);
        std::vector<int32_t> mem_ptr(nc + 1), mem(n);
        int32_t I = 0, q = 0;
        for (int32_t i = 0; i < n; ++i) {
            int32_t m = mate[i];
            if (m >= 0 && m < i) continue;
            mem_ptr[I] = q;
            if (m < 0) {
                cur.agg[i] = I;
                cur.p[i] = cur.w[i] / std::fabs(cur.w[i]);
                wc[I] = std::fabs(cur.w[i]);
                mem[q++] = i;
            } else {
                double nu = std::sqrt(cur.w[i] * cur.w[i] + cur.w[m] * cur.w[m]);
                cur.agg[i] = I; cur.agg[m] = I;
                cur.p[i] = cur.w[i] / nu;
                cur.p[m] = cur.w[m] / nu;
                wc[I] = nu;
                mem[q++] = i; mem[q++] = m;
            }
            ++I;
        }
        mem_ptr[nc] = q;
        HostLevel next;
        if (prm.smooth_prolongator) {
            smoothed_prolongator(A, cur.agg, cur.p, cur.P, cur.omega_p);
            galerkin_smoothed(A, cur.P, nc, next.A);
        } else {
            galerkin(A, cur.agg, cur.p, mem_ptr, mem, next.A);
        }
        next.w = std::move(wc);
        H.lev.push_back(std::move(next));
    }
}

// ------------------------------------------- smoothed prolongator layout

void sa_layout(const HostCSR& P, const LayoutLevel& fine, const LayoutLevel& coarse, LayoutLevel& out) {
    const int32_t n = P.n, nc = (int32_t)coarse.perm.size();
    out.sa_prp.assign(n + 1, 0);
    for (int32_t ip = 0; ip < n; ++ip) {
        const int32_t i = fine.iperm[ip];
        out.sa_prp[ip + 1] = out.sa_prp[ip] + (P.rp[i + 1] - P.rp[i]);
    }
    out.sa_pci.resize(out.sa_prp[n]);
    out.sa_pv.resize(out.sa_prp[n]);
    parallel_ranges(n, [&](int, int64_t b, int64_t e) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t ip = b; ip < e; ++ip) {
            const int32_t i = fine.iperm[ip];
            row.clear();
            for (int32_t u = P.rp[i]; u < P.rp[i + 1]; ++u) row.emplace_back(coarse.perm[P.ci[u]], P.v[u]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
            for (size_t u = 0; u < row.size(); ++u) {
                out.sa_pci[out.sa_prp[ip] + u] = row[u].first;
                out.sa_pv[out.sa_prp[ip] + u] = row[u].second;
            }
        }
    });
    // P^T: rows = coarse (hierarchical), entries = fine rows ascending
    out.sa_trp.assign(nc + 1, 0);
    for (int32_t u = 0; u < out.sa_prp[n]; ++u) ++out.sa_trp[out.sa_pci[u] + 1];
    for (int32_t I = 0; I < nc; ++I) out.sa_trp[I + 1] += out.sa_trp[I];
    out.sa_tci.resize(out.sa_prp[n]);
    out.sa_tv.resize(out.sa_prp[n]);
    std::vector<int32_t> fill(out.sa_trp.begin(), out.sa_trp.end() - 1);
    for (int32_t ip = 0; ip < n; ++ip)
        for (int32_t u = out.sa_prp[ip]; u < out.sa_prp[ip + 1]; ++u) {
            const int32_t I = out.sa_pci[u];
            out.sa_tci[fill[I]] = ip;
            out.sa_tv[fill[I]] = out.sa_pv[u];
            ++fill[I];
        }
    out.sa_ptile = tile_rows(out.sa_prp, out.sa_pci, n, nc);
    out.sa_ttile = tile_rows(out.sa_trp, out.sa_tci, nc, n);
}

// ------------------------------------------- hybrid Gauss-Seidel schedule

GsLevel gs_schedule(const LayoutLevel& L, int nb) {
    const int32_t n = (int32_t)L.dinv.size();
    const int32_t nblk = (n + nb - 1) / nb;
    GsLevel g;
    g.depth_f.assign(n, 0);
    g.depth_b.assign(n, 0);
    g.maxd.assign(2 * (size_t)nblk, 0);
    g.ainv.assign(n, 0.0);
    g.fresh.assign(2 * (size_t)n, 0);
    std::atomic<int> bad{0};
    parallel_for(nblk, [&](int64_t p) {
        const int32_t b0 = (int32_t)p * nb, b1 = std::min(n, b0 + nb);
        int32_t mf = 0, mb = 0;
        for (int32_t i = b0; i < b1; ++i) {
            int32_t d = 0, first = -1, nbefore = 0, nafter = 0, diag = 0;
            for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) {
                const int32_t j = L.ci[k];
                if (j >= b0 && j < b1 && first < 0) first = k;
                if (j >= b0 && j < i) {
                    d = std::max(d, g.depth_f[j] + 1);
                    ++nbefore;
                }
                if (j > i && j < b1) ++nafter;
                if (j == i) {
                    if (!(L.v[k] > 0.0)) bad.store(1);
                    g.ainv[i] = 1.0 / L.v[k];
                    diag = 1;
                }
            }
            g.fresh[2 * (size_t)i] = first < 0 ? L.rp[i] : first;
            g.fresh[2 * (size_t)i + 1] = nbefore | nafter << 8 | diag << 16;
            g.depth_f[i] = (uint8_t)d;
            mf = std::max(mf, d);
        }
        for (int32_t i = b1 - 1; i >= b0; --i) {
            int32_t d = 0;
            for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) {
                const int32_t j = L.ci[k];
                if (j > i && j < b1) d = std::max(d, g.depth_b[j] + 1);
            }
            g.depth_b[i] = (uint8_t)d;
            mb = std::max(mb, d);
        }
        g.maxd[2 * p] = mf;
        g.maxd[2 * p + 1] = mb;
    });
    if (bad.load()) throw Error(PAMG_E_NOT_SPD, "non-positive diagonal on a coarse level (Gauss-Seidel smoother)");
    return g;
}

// ------------------------------------------------ coefficient-only reuse

GalerkinPlan galerkin_plan(const HostCSR& A, const std::vector<int32_t>& agg, const std::vector<double>& p,
                           const HostCSR& Ac) {
    const int32_t n = A.n, nc = Ac.n;
    std::vector<int32_t> mptr(nc + 1, 0), mem(n);
    for (int32_t i = 0; i < n; ++i) ++mptr[agg[i] + 1];
    for (int32_t I = 0; I < nc; ++I) mptr[I + 1] += mptr[I];
    {
        std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1);
        for (int32_t i = 0; i < n; ++i) mem[fill[agg[i]]++] = i;
    }
    // first term of each coarse row: the terms of a row are its members' entries
    std::vector<int64_t> toff(nc + 1, 0);
    for (int32_t I = 0; I < nc; ++I) {
        int64_t c = 0;
        for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) c += A.rp[mem[q] + 1] - A.rp[mem[q]];
        toff[I + 1] = toff[I] + c;
    }
    GalerkinPlan g;
    g.ptr.assign(Ac.nnz() + 1, 0);
    g.k.resize(A.nnz());
    g.pp.resize(A.nnz());
    std::atomic<int> bad{0};
    parallel_ranges(nc, [&](int, int64_t b, int64_t e) {
        struct Key {
            int32_t J, k1, k2, k3, k;
        };
        std::vector<Key> t;
        for (int64_t I = b; I < e; ++I) {
            t.clear();
            for (int32_t q = mptr[I]; q < mptr[I + 1]; ++q) {
                const int32_t i = mem[q];
                for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                    const int32_t j = A.ci[k];
                    t.push_back({agg[j], std::min(i, j), std::max(i, j), i, k});
                }
            }
            // the order of the setup's Galerkin sum (a strict total order)
            std::sort(t.begin(), t.end(), [](const Key& x, const Key& y) {
                if (x.J != y.J) return x.J < y.J;
                if (x.k1 != y.k1) return x.k1 < y.k1;
                if (x.k2 != y.k2) return x.k2 < y.k2;
                return x.k3 < y.k3;
            });
            int64_t q = toff[I];
            int32_t c = Ac.rp[I] - 1;
            for (size_t u = 0; u < t.size(); ++u, ++q) {
                if (u == 0 || t[u].J != t[u - 1].J) {
                    ++c;
                    if (c >= Ac.rp[I + 1] || Ac.ci[c] != t[u].J) bad.store(1);
                    else g.ptr[c] = (int32_t)q;
                }
                g.k[q] = t[u].k;
                g.pp[q] = p[t[u].k3] * p[A.ci[t[u].k]];
            }
            if (c != Ac.rp[I + 1] - 1) bad.store(1);
        }
    });
    if (bad.load()) throw Error(PAMG_E_DEVICE, "Galerkin plan does not match the coarse pattern");
    g.ptr[Ac.nnz()] = (int32_t)A.nnz();
    return g;
}

std::vector<int32_t> entry_order(const HostCSR& A, const std::vector<int32_t>& perm,
                                 const std::vector<int32_t>& iperm) {
    const int32_t n = A.n;
    std::vector<int32_t> rp(n + 1, 0);
    for (int32_t ip = 0; ip < n; ++ip) rp[ip + 1] = rp[ip] + (A.rp[iperm[ip] + 1] - A.rp[iperm[ip]]);
    std::vector<int32_t> out(A.nnz());
    parallel_ranges(n, [&](int, int64_t b, int64_t e) {
        std::vector<std::pair<int32_t, int32_t>> row;
        for (int64_t ip = b; ip < e; ++ip) {
            const int32_t i = iperm[ip];
            row.clear();
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) row.emplace_back(perm[A.ci[k]], k);
            std::sort(row.begin(), row.end());
            for (size_t u = 0; u < row.size(); ++u) out[rp[ip] + u] = row[u].second;
        }
    });
    return out;
}

// ---------------------------------------------------------------- layout

// Column dictionary of every tile (tiles given as 4 ints k0, k1, *, *).
// Per tile: the distinct columns are collected with a per-worker position
// array (n entries, reset after each tile), sorted, and every entry's column
// is then looked up directly.
static TileDict build_dicts(const std::vector<int32_t>& tiles, const std::vector<int32_t>& ci, int32_t n,
                            int32_t cap) {
    TileDict D;
    const int64_t nt = (int64_t)tiles.size() / 4;
    D.span.assign(2 * nt, 0);
    D.local.assign(ci.size(), 0);
    std::vector<std::vector<int32_t>> dict(nt);
    // tiles in chunks from a shared counter (a level has few tiles when its
    // matrix is small, not when its tiles are cheap)
    struct alignas(64) PosBuf {  // one cache line (or more) per thread
        std::vector<int32_t> pos;
    };
    std::vector<PosBuf> pbuf(num_threads());
    parallel_chunks(nt, 4, [&](int th, int64_t b, int64_t e) {
        std::vector<int32_t>& pos = pbuf[th].pos;
        if (pos.empty()) pos.assign(n, -1);
        for (int64_t t = b; t < e; ++t) {
            const int32_t k0 = tiles[4 * t], k1 = tiles[4 * t + 1];
            if (k1 - k0 > cap) continue;
            std::vector<int32_t>& u = dict[t];
            for (int32_t k = k0; k < k1; ++k)
                if (pos[ci[k]] < 0) {
                    pos[ci[k]] = 0;
                    u.push_back(ci[k]);
                }
            std::sort(u.begin(), u.end());
            for (size_t j = 0; j < u.size(); ++j) pos[u[j]] = (int32_t)j;
            for (int32_t k = k0; k < k1; ++k) D.local[k] = (uint16_t)pos[ci[k]];
            for (int32_t c : u) pos[c] = -1;
        }
    });
    int64_t total = 0;
    for (int64_t t = 0; t < nt; ++t) {
        D.span[2 * t] = (int32_t)total;
        D.span[2 * t + 1] = (int32_t)dict[t].size();
        D.max_len = std::max<int32_t>(D.max_len, (int32_t)dict[t].size());
        total += (int64_t)dict[t].size();
    }
    if (total >= (int64_t(1) << 31)) throw Error(PAMG_E_OOM, "tile dictionaries exceed 2^31 entries");
    D.col.resize(total);
    parallel_ranges(nt, [&](int, int64_t b, int64_t e) {
        for (int64_t t = b; t < e; ++t) std::copy(dict[t].begin(), dict[t].end(), D.col.begin() + D.span[2 * t]);
    });
    return D;
}

// Tile capacity of a level: the largest power of two <= kMaxItems with at
// least kTargetTiles tiles' worth of entries (small levels get small tiles).
int first_tile_items(int64_t nnz) {
    int items = kMaxItems;
    while (items > 1 && (int64_t)items * kBlock * kTargetTiles > nnz) items /= 2;
    return items;
}

// Row tiles: <= kTileRows rows and <= cap entries, or a single long row.
// Restriction tiles over coarse rows: the <= kTileRows fine rows of
// <= kTileRows aggregates holding <= cap entries, or a single aggregate (at
// most 2^kMaxAggSteps members).  4 ints per tile: k0, k1, first, end.
void make_tiles(const std::vector<int32_t>& rp, const std::vector<int32_t>& aggptr, int32_t n, int32_t nc,
                int32_t cap, std::vector<int32_t>& up, std::vector<int32_t>& down) {
    up.clear();
    int32_t start = 0;
    while (start < n) {
        int32_t end = start + 1;
        while (end < n && end - start < kTileRows && rp[end + 1] - rp[start] <= cap) ++end;
        up.insert(up.end(), {rp[start], rp[end], start, end});
        start = end;
    }
    down.clear();
    start = 0;
    while (start < nc) {
        int32_t end = start + 1;
        while (end < nc && end - start < kTileRows && aggptr[end + 1] - aggptr[start] <= kTileRows &&
               rp[aggptr[end + 1]] - rp[aggptr[start]] <= cap)
            ++end;
        down.insert(down.end(), {rp[aggptr[start]], rp[aggptr[end]], start, end});
        start = end;
    }
}

// Row tiles of an n-row matrix with ncols columns, capacity chosen as for a
// level's own matrix: the first capacity whose dictionaries fit the
// prefetch slots (halving from first_tile_items), dictionaries only for
// tiles of at least kDictItems items per thread.
TiledRows tile_rows(const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, int32_t n, int32_t ncols) {
    TiledRows T;
    const std::vector<int32_t> no_aggregates;
    std::vector<int32_t> no_down;
    int items = first_tile_items((int64_t)rp[n]);
    for (;;) {
        T.items = items;
        const int32_t cap = items * kBlock;
        make_tiles(rp, no_aggregates, n, 0, cap, T.tiles, no_down);
        if (items < kDictItems) break;
        T.dict = build_dicts(T.tiles, ci, ncols, cap);
        if (items == kDictItems || T.dict.max_len <= kDictMaxLarge) break;
        items /= 2;
        T.dict = TileDict();
    }
    return T;
}

// Hierarchical numbering: the coarsest level keeps its numbering; on every
// finer level the members of each aggregate are placed next to each other,
// in the order of their aggregate's (already permuted) coarse index, members
// ascending.  Restriction and prolongation then touch contiguous rows.
std::vector<LayoutLevel> build_layout(const HostHierarchy& H) {
    const int nl = (int)H.lev.size();
    std::vector<LayoutLevel> out(nl);
    {
        LayoutLevel& c = out[nl - 1];
        int32_t n = H.lev[nl - 1].A.n;
        c.perm.resize(n);
        c.iperm.resize(n);
        std::iota(c.perm.begin(), c.perm.end(), 0);
        std::iota(c.iperm.begin(), c.iperm.end(), 0);
    }
    for (int l = nl - 2; l >= 0; --l) {
        const HostLevel& hl = H.lev[l];
        const int32_t n = hl.A.n, nc = H.lev[l + 1].A.n;
        // canonical members of each canonical aggregate, ascending (pairs,
        // or up to 2^s members with aggregate-size composition)
        std::vector<int32_t> mptr(nc + 1, 0), mem(n);
        for (int32_t i = 0; i < n; ++i) ++mptr[hl.agg[i] + 1];
        for (int32_t I = 0; I < nc; ++I) mptr[I + 1] += mptr[I];
        {
            std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1);
            for (int32_t i = 0; i < n; ++i) mem[fill[hl.agg[i]]++] = i;
        }
        LayoutLevel& L = out[l];
        L.iperm.resize(n);
        L.perm.resize(n);
        L.aggptr.resize(nc + 1);
        const std::vector<int32_t>& cip = out[l + 1].iperm;
        int32_t q = 0;
        for (int32_t Ip = 0; Ip < nc; ++Ip) {
            int32_t I = cip[Ip];
            L.aggptr[Ip] = q;
            for (int32_t k = mptr[I]; k < mptr[I + 1]; ++k) L.iperm[q++] = mem[k];
        }
        L.aggptr[nc] = q;
        for (int32_t ip = 0; ip < n; ++ip) L.perm[L.iperm[ip]] = ip;
    }
    for (int l = 0; l < nl; ++l) {
        const HostLevel& hl = H.lev[l];
        LayoutLevel& L = out[l];
        const int32_t n = hl.A.n;
        L.rp.resize(n + 1);
        L.rp[0] = 0;
        for (int32_t ip = 0; ip < n; ++ip) {
            int32_t i = L.iperm[ip];
            L.rp[ip + 1] = L.rp[ip] + (hl.A.rp[i + 1] - hl.A.rp[i]);
        }
        L.ci.resize(hl.A.nnz());
        L.v.resize(hl.A.nnz());
        L.dinv.resize(n);
        if (l + 1 < nl) L.p.resize(n);
        // rows in chunks from a shared counter (small coarse levels have long rows)
        struct alignas(64) RowBuf {  // one cache line (or more) per thread
            std::vector<std::pair<int32_t, double>> row;
        };
        std::vector<RowBuf> rbuf(num_threads());
        parallel_chunks(n, 16, [&](int th, int64_t b, int64_t e) {
            std::vector<std::pair<int32_t, double>>& row = rbuf[th].row;
            for (int64_t ip = b; ip < e; ++ip) {
                int32_t i = L.iperm[ip];
                row.clear();
                for (int32_t k = hl.A.rp[i]; k < hl.A.rp[i + 1]; ++k) row.emplace_back(L.perm[hl.A.ci[k]], hl.A.v[k]);
                std::sort(row.begin(), row.end(),
                          [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b2) { return a.first < b2.first; });
                int32_t o = L.rp[ip];
                for (size_t s = 0; s < row.size(); ++s) { L.ci[o + s] = row[s].first; L.v[o + s] = row[s].second; }
                L.dinv[ip] = hl.dinv[i];
                if (l + 1 < nl) L.p[ip] = hl.p[i];
            }
        });
        int items = first_tile_items((int64_t)L.rp[n]);
        const int32_t nc = l + 1 < nl ? H.lev[l + 1].A.n : 0;
        for (;;) {
            L.items = items;
            const int32_t cap = items * kBlock;
            make_tiles(L.rp, L.aggptr, n, nc, cap, L.up_tiles, L.down_tiles);
            if (items < kDictItems) break;            // small tiles gather per entry
            L.up_dict = build_dicts(L.up_tiles, L.ci, n, cap);
            if (nc > 0) L.down_dict = build_dicts(L.down_tiles, L.ci, n, cap);
            // the largest tiles keep their dictionary within LDS, else halve them
            if (items == kDictItems || std::max(L.up_dict.max_len, L.down_dict.max_len) <= kDictMaxLarge) break;
            items /= 2;
            L.up_dict = TileDict();
            L.down_dict = TileDict();
        }
        if (l + 1 < nl) {
            // column-scaled values for the restriction pass: a_ij / d_j
            L.vd.resize(L.v.size());
            parallel_for(n, [&](int64_t ip) {
                for (int32_t k = L.rp[ip]; k < L.rp[ip + 1]; ++k) L.vd[k] = L.v[k] * L.dinv[L.ci[k]];
            }, 64);
        }
    }
    return out;
}

}  // namespace pamg
