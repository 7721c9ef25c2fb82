/*
 * CPU FP64 ORACLE for the PCG/FCG + matching-aggregation AMG solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the library; only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  The product path
 * never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no
 * fast-math: every floating-point operation below is one IEEE-754 binary64
 * operation in the order written).
 *
 * What it computes (paper: "Alya towards Exascale: Algorithmic Scalability
 * using PSCToolkit", arXiv 2210.16660):
 *   - the AMG hierarchy of Sec. 3.1: Galerkin coarse matrices
 *     A_{l+1} = P_l^T A_l P_l, edge weights of eq. (weights), an
 *     approximate maximum-product matching (eq. approximatematch), aggregates
 *     made of matched pairs and singletons, and the tentative prolongator of
 *     eq. (prolongator) (piecewise constant, w in its range);
 *   - the V-cycle of eq. (multiplicative_composition) with nu = 1 and the
 *     l1-Jacobi smoother M_l = diag(sum_j |a_ij|), and a direct (dense
 *     Cholesky) coarsest solve B_L = A_L^{-1};
 *   - preconditioned CG, or flexible CG with truncation 1 (Sec. 5 uses FCG),
 *     stopped when ||r||_2 <= tol * ||b||_2.
 *
 * Readings where the paper is silent (each is the definition used below):
 *   R1 smoother: l1-Jacobi, D_ii = sum_j |a_ij| summed in ascending column
 *      order, one undamped pre- and one post-sweep, zero initial guess.
 *   R2 w_0 = 1 (the "arbitrary vector w" of the weights).
 *   R3 eligible edges: c_ij > 1 as computed (only those raise the product).
 *   R4 weight evaluation order: num = ((2*a)*w_lo)*w_hi,
 *      den = (a_lolo*w_lo)*w_lo + (a_hihi*w_hi)*w_hi, c = 1 - num/den.
 *   R5 matching: greedy over eligible edges sorted by (c descending, lo
 *      ascending, hi ascending); an edge is taken iff both ends are free.
 *      Under this strict total order the result is unique and is a
 *      half-approximation of the maximum product (the bound the paper quotes
 *      for its matching library).
 *   R6 coarse numbering: aggregates numbered by ascending smallest member.
 *   R7 prolongator: pair (lo, hi): nu = sqrt(w_lo*w_lo + w_hi*w_hi),
 *      p = w/nu, w_c = nu;  singleton s: p = w_s/|w_s|, w_c = |w_s|.
 *   R8 Galerkin rounding: A_{l+1}[I,J] = sum of a_ij*(p_i*p_j) over stored
 *      (i,j) with agg(i)=I, agg(j)=J, added left to right in ascending order
 *      of (min(i,j), max(i,j), i); every structural entry kept (even 0.0).
 *   R9 levels: coarsen while n_l > max_coarse (200); a level whose matching
 *      has no pair is the coarsest (error STALLED if it exceeds max_dense);
 *      at most max_levels levels.  Levels are 0..L; smoothing on 0..L-1.
 *   R11 stalled coarsening: a level with n_l <= max_dense whose matching
 *      would give n_{l+1} with n_l < min_ratio * n_{l+1} (default 1.5) is
 *      the coarsest; its matching is discarded.  (Weakly coupled vertices
 *      can stay singletons on every level while everything else merges, so
 *      that later levels shed one pair each.)  min_ratio <= 1 turns the
 *      rule off; above max_dense coarsening always continues.
 *   R12 aggregate-size composition (Sec. 3.1: aggregates larger than pairs
 *      by multiplying successive pairwise prolongators): with agg_steps = s,
 *      the pairwise hierarchy is built as above and only levels 0, s, 2s, ...
 *      and the coarsest are kept; the prolongator from a kept level to the
 *      next is the product of the pairwise ones in between, itself piecewise
 *      constant: agg(i) follows the chain of aggregates and p(i) is the
 *      product of the chain's p values, multiplied finest first.  The kept
 *      coarse matrices are the pairwise Galerkin matrices (the same sums).
 *   R10 Krylov: PCG, or FCG(1) with beta = -(z.q_old)/delta_old and
 *      alpha = (p.r)/delta; dot products summed in index order.
 *   R13 coefficient-only reuse (Sec. 4: when only the coefficients of A
 *      change, the prolongators are kept and the coarse matrices and
 *      smoothers rebuilt): new values of A_0 with the same pattern; every
 *      pairwise step keeps its aggregates and p, its Galerkin matrix is
 *      recomputed from the new fine values by R8, the l1 diagonals by R1 and
 *      the coarsest factor anew.  With composition (R12) the whole pairwise
 *      chain is recomputed and the kept levels are taken from it, so the
 *      result is the hierarchy a setup would give if its matchings were
 *      those of the original matrix.
 *   R14 hybrid forward/backward Gauss-Seidel smoother (Sec. 3.1, the
 *      smoother the paper uses; optional here, R1 is the default): the
 *      unknowns of a level are taken in nested-aggregate order (the coarsest
 *      level in its own order; a finer level lists the members of each
 *      coarse unknown, coarse unknowns in their nested order, members in
 *      ascending index) and cut into consecutive blocks of nb unknowns, the
 *      row blocks of the paper's row-block distribution.  One sweep is
 *      x <- x + M^-1 (r - A x) with M = blockdiag(omega (L_pp + D_pp)):
 *      within a block, in nested order,
 *      d_i = ((r_i - sum_j a_ij x_j) - sum_{j earlier in the block} a_ij d_j) / a_ii
 *      (both sums in ascending column order), then x_i += d_i / omega.  A
 *      backward sweep runs each block in reverse (M^T).  Pre-smoothing: nu
 *      forward sweeps from zero; post-smoothing: nu backward sweeps, so the
 *      V-cycle stays symmetric.
 *   R15 smoothed prolongator (Sec. 3.1, optional):
 *      P = (I - omega D^-1 A) P^ with D = diag(A) and
 *      omega = 1 / ||D^-1 A||_inf = 1 / max_i ((sum_j |a_ij|) / a_ii).
 *      Row i: P_iJ = [J = agg(i)] p_i - sum_{j: agg(j) = J} (omega (a_ij / a_ii)) p_j,
 *      starting from p_i (or 0.0) and subtracting in ascending j; its pattern
 *      is {agg(j) : a_ij stored}.  Galerkin: B = A P with
 *      B_kJ = 0.0 + sum over j ascending of a_kj P_jJ, then for I <= J
 *      A_{l+1}[I,J] = 0.0 + sum over i ascending of P_iI B_iJ, and
 *      A_{l+1}[J,I] = A_{l+1}[I,J] (bitwise symmetric).  The matching of the
 *      next level runs on this matrix with the tentative coarse w.
 *      Restriction is P^T (sums over ascending i), prolongation P.  With
 *      composition (R12, agg_steps = s > 1) the levels are built one kept
 *      level at a time: from kept level K, up to s pairwise steps (matching,
 *      aggregates, tentative Galerkin between steps, every stop rule applied
 *      to every step) give the composed aggregates and p; K's prolongator is
 *      that composed tentative prolongator smoothed with K, and the next kept
 *      level is P^T K P.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_E_INVALID (-1)
#define OR_E_NOT_SPD (-2)
#define OR_E_NUMERIC (-3)
#define OR_E_OOM (-4)
#define OR_E_STALLED (-6)

#define OR_MAX_LEVELS 64

typedef struct {
    int n;
    long nnz;
    int *rp;
    int *ci;
    double *v;
} or_csr;

typedef struct {
    int nlev;                       /* levels 0 .. nlev-1; coarsest L = nlev-1 */
    or_csr A[OR_MAX_LEVELS];
    double *w[OR_MAX_LEVELS];       /* near-null vector of level l */
    double *dinv[OR_MAX_LEVELS];    /* 1 / l1 diagonal */
    int *agg[OR_MAX_LEVELS];        /* level l -> level l+1 aggregate index (l < L) */
    double *p[OR_MAX_LEVELS];       /* the single nonzero of row i of P_l (l < L) */
    int n_pairs[OR_MAX_LEVELS];
    double *chol;                   /* lower Cholesky factor of A_L, row-major n_L x n_L */
    /* the pairwise chain before composition (R12), kept for reuse (R13) */
    int pw_nlev;                    /* pairwise levels 0 .. pw_nlev-1 */
    int pw_n[OR_MAX_LEVELS];
    int *pw_agg[OR_MAX_LEVELS];     /* pairwise step m: level m -> m+1 */
    double *pw_p[OR_MAX_LEVELS];
    int kept[OR_MAX_LEVELS];        /* pairwise level of each kept level */
    /* smoothed prolongators (R15): P[l] is n_l x n_{l+1} (l < L) */
    int smoothed;
    or_csr P[OR_MAX_LEVELS];
    double omega_p[OR_MAX_LEVELS];
    /* smoother (R1 l1-Jacobi unless set by oracle_set_smoother, R14) */
    int smoother;                   /* 0: l1-Jacobi, 1: hybrid forward/backward Gauss-Seidel */
    int gs_nu, gs_nb;
    double gs_omega;
} or_hier;

/* ------------------------------------------------------------------ utils */

static void csr_free(or_csr *a) {
    free(a->rp); free(a->ci); free(a->v);
    memset(a, 0, sizeof(*a));
}

void oracle_free(or_hier *h) {
    if (!h) return;
    for (int l = 0; l < OR_MAX_LEVELS; ++l) {
        csr_free(&h->A[l]);
        free(h->w[l]); free(h->dinv[l]); free(h->agg[l]); free(h->p[l]);
        free(h->pw_agg[l]); free(h->pw_p[l]);
        csr_free(&h->P[l]);
    }
    free(h->chol);
    free(h);
}

/* y = A x, each row summed in ascending column order */
/* All-cores timing build (-fopenmp, the CPU baseline only): the row and
 * element loops of the solve phase are split over threads.  Each row or
 * element is still computed by the same operations in the same order and
 * every reduction (dot products, the restriction's scatter) stays serial, so
 * that build's results are bitwise those of the plain build, which ignores
 * the pragma. */
#ifdef _OPENMP
#define OR_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PARALLEL_FOR
#endif

static void csr_mv(const or_csr *a, const double *x, double *y) {
    OR_PARALLEL_FOR
    for (int i = 0; i < a->n; ++i) {
        double s = 0.0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) s += a->v[k] * x[a->ci[k]];
        y[i] = s;
    }
}

static double dot(int n, const double *x, const double *y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

static double diag_entry(const or_csr *a, int i) {
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k)
        if (a->ci[k] == i) return a->v[k];
    return 0.0;
}

/* ----------------------------------------------- matching (Sec. 3.1, R3-R5) */

typedef struct { double c; int lo, hi; } or_edge;

static int edge_order(const void *pa, const void *pb) {
    const or_edge *a = (const or_edge *)pa, *b = (const or_edge *)pb;
    if (a->c > b->c) return -1;          /* weight descending */
    if (a->c < b->c) return 1;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return 0;
}

/* weight c_ij of eq. (weights), evaluated as in R4 */
static double edge_weight(double a_lohi, double a_lolo, double a_hihi, double w_lo, double w_hi) {
    double num = ((2.0 * a_lohi) * w_lo) * w_hi;
    double den = (a_lolo * w_lo) * w_lo + (a_hihi * w_hi) * w_hi;
    return 1.0 - num / den;
}

/* mate[i] = partner or -1.  Returns number of pairs, or -1 on OOM. */
static long greedy_matching(const or_csr *a, const double *w, int match_all, int *mate) {
    int n = a->n;
    double *diag = (double *)malloc(sizeof(double) * (size_t)n);
    if (!diag) return -1;
    for (int i = 0; i < n; ++i) diag[i] = diag_entry(a, i);
    long ne = 0;
    for (int i = 0; i < n; ++i)
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k)
            if (a->ci[k] > i) ++ne;
    or_edge *e = (or_edge *)malloc(sizeof(or_edge) * (size_t)(ne > 0 ? ne : 1));
    if (!e) { free(diag); return -1; }
    long m = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int j = a->ci[k];
            if (j <= i) continue;               /* lo = i, hi = j, a_{lo,hi} stored in row lo */
            double c = edge_weight(a->v[k], diag[i], diag[j], w[i], w[j]);
            if (match_all || c > 1.0) { e[m].c = c; e[m].lo = i; e[m].hi = j; ++m; }
        }
    }
    qsort(e, (size_t)m, sizeof(or_edge), edge_order);
    for (int i = 0; i < n; ++i) mate[i] = -1;
    long pairs = 0;
    for (long t = 0; t < m; ++t) {
        if (mate[e[t].lo] < 0 && mate[e[t].hi] < 0) {
            mate[e[t].lo] = e[t].hi;
            mate[e[t].hi] = e[t].lo;
            ++pairs;
        }
    }
    free(e); free(diag);
    return pairs;
}

/* ------------------------------------ aggregates and prolongator (R6, R7) */

/* returns n_c; fills agg, p (level l) and wc (level l+1) */
static int build_aggregates(int n, const int *mate, const double *w, int *agg, double *p, double *wc) {
    int nc = 0;
    for (int i = 0; i < n; ++i) {
        int m = mate[i];
        if (m < 0) {                              /* singleton: W = diag(w_s/|w_s|) */
            agg[i] = nc;
            p[i] = w[i] / fabs(w[i]);
            wc[nc] = fabs(w[i]);
            ++nc;
        } else if (m > i) {                       /* pair (i, m), i smallest member */
            double nu = sqrt(w[i] * w[i] + w[m] * w[m]);
            agg[i] = nc; agg[m] = nc;
            p[i] = w[i] / nu;
            p[m] = w[m] / nu;
            wc[nc] = nu;
            ++nc;
        }                                          /* m < i: already assigned */
    }
    return nc;
}

/* ------------------------------------------------------- Galerkin (R8) */

typedef struct {
    int I, J;           /* coarse position */
    int k1, k2, k3;     /* min(i,j), max(i,j), i */
    double t;           /* a_ij * (p_i * p_j) */
} or_term;

static int term_order(const void *pa, const void *pb) {
    const or_term *a = (const or_term *)pa, *b = (const or_term *)pb;
    if (a->I != b->I) return a->I < b->I ? -1 : 1;
    if (a->J != b->J) return a->J < b->J ? -1 : 1;
    if (a->k1 != b->k1) return a->k1 < b->k1 ? -1 : 1;
    if (a->k2 != b->k2) return a->k2 < b->k2 ? -1 : 1;
    if (a->k3 != b->k3) return a->k3 < b->k3 ? -1 : 1;
    return 0;
}

static int galerkin(const or_csr *a, const int *agg, const double *p, int nc, or_csr *out) {
    long nnz = a->nnz;
    or_term *t = (or_term *)malloc(sizeof(or_term) * (size_t)nnz);
    if (!t) return OR_E_OOM;
    long m = 0;
    for (int i = 0; i < a->n; ++i) {
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int j = a->ci[k];
            t[m].I = agg[i]; t[m].J = agg[j];
            t[m].k1 = i < j ? i : j;
            t[m].k2 = i < j ? j : i;
            t[m].k3 = i;
            t[m].t = a->v[k] * (p[i] * p[j]);
            ++m;
        }
    }
    qsort(t, (size_t)m, sizeof(or_term), term_order);
    /* count distinct (I, J) */
    long cnt = 0;
    for (long s = 0; s < m; ++s)
        if (s == 0 || t[s].I != t[s - 1].I || t[s].J != t[s - 1].J) ++cnt;
    out->n = nc;
    out->nnz = cnt;
    out->rp = (int *)calloc((size_t)nc + 1, sizeof(int));
    out->ci = (int *)malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
    out->v = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    if (!out->rp || !out->ci || !out->v) { free(t); return OR_E_OOM; }
    long q = -1;
    for (long s = 0; s < m; ++s) {
        if (s == 0 || t[s].I != t[s - 1].I || t[s].J != t[s - 1].J) {
            ++q;
            out->ci[q] = t[s].J;
            out->v[q] = t[s].t;                  /* the first term starts the sum */
            out->rp[t[s].I + 1]++;
        } else {
            out->v[q] = out->v[q] + t[s].t;
        }
    }
    for (int I = 0; I < nc; ++I) out->rp[I + 1] += out->rp[I];
    free(t);
    return OR_OK;
}

/* ------------------------------------------- smoothed prolongator (R15) */

static int smoothed_prolongator(const or_csr *a, const int *agg, const double *p, or_csr *P, double *omega_out) {
    int n = a->n;
    double mx = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0, aii = 0.0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            s += fabs(a->v[k]);
            if (a->ci[k] == i) aii = a->v[k];
        }
        double r = s / aii;
        if (r > mx) mx = r;
    }
    double omega = 1.0 / mx;
    *omega_out = omega;
    /* pattern: the distinct agg(j) of each row, ascending */
    P->n = n;
    P->rp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *cols = (int *)malloc(sizeof(int) * (size_t)(a->nnz > 0 ? a->nnz : 1));
    if (!P->rp || !cols) { free(cols); return OR_E_OOM; }
    long q = 0;
    for (int i = 0; i < n; ++i) {
        long r0 = q;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int J = agg[a->ci[k]], dup = 0;
            for (long u = r0; u < q; ++u)
                if (cols[u] == J) { dup = 1; break; }
            if (!dup) cols[q++] = J;
        }
        for (long u = r0 + 1; u < q; ++u) {        /* insertion sort of the row */
            int c = cols[u];
            long w = u;
            while (w > r0 && cols[w - 1] > c) { cols[w] = cols[w - 1]; --w; }
            cols[w] = c;
        }
        P->rp[i + 1] = (int)q;
    }
    P->nnz = q;
    P->ci = (int *)malloc(sizeof(int) * (size_t)(q > 0 ? q : 1));
    P->v = (double *)malloc(sizeof(double) * (size_t)(q > 0 ? q : 1));
    if (!P->ci || !P->v) { free(cols); return OR_E_OOM; }
    memcpy(P->ci, cols, sizeof(int) * (size_t)q);
    free(cols);
    for (int i = 0; i < n; ++i) {
        double aii = diag_entry(a, i);
        for (int u = P->rp[i]; u < P->rp[i + 1]; ++u) P->v[u] = P->ci[u] == agg[i] ? p[i] : 0.0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int j = a->ci[k], J = agg[j];
            int u = P->rp[i];
            while (P->ci[u] != J) ++u;
            P->v[u] = P->v[u] - (omega * (a->v[k] / aii)) * p[j];
        }
    }
    return OR_OK;
}

static void sort_ints(int *x, int m) {
    for (int u = 1; u < m; ++u) {
        int c = x[u], w = u;
        while (w > 0 && x[w - 1] > c) { x[w] = x[w - 1]; --w; }
        x[w] = c;
    }
}

/* A_c = P^T A P through B = A P; the upper triangle is summed and mirrored (R15) */
static int galerkin_smoothed(const or_csr *a, const or_csr *P, int nc, or_csr *out) {
    int n = a->n, st = OR_OK;
    double *acc = (double *)calloc((size_t)nc, sizeof(double));
    int *mark = (int *)malloc(sizeof(int) * (size_t)nc);
    int *list = (int *)malloc(sizeof(int) * (size_t)nc);
    or_csr B, U;
    memset(&B, 0, sizeof(B));
    memset(&U, 0, sizeof(U));
    B.rp = (int *)calloc((size_t)n + 1, sizeof(int));
    U.rp = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *tp = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *ti = (int *)malloc(sizeof(int) * (size_t)(P->nnz > 0 ? P->nnz : 1));
    double *tv = (double *)malloc(sizeof(double) * (size_t)(P->nnz > 0 ? P->nnz : 1));
    int *fill = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
    long cap = 1024;
    B.ci = (int *)malloc(sizeof(int) * (size_t)cap);
    B.v = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!acc || !mark || !list || !B.rp || !U.rp || !tp || !ti || !tv || !fill || !B.ci || !B.v) {
        st = OR_E_OOM;
        goto done;
    }
    /* B = A P, row k: B_kJ = 0.0 + sum over j ascending of a_kj P_jJ */
    for (int J = 0; J < nc; ++J) mark[J] = -1;
    long used = 0;
    for (int k = 0; k < n; ++k) {
        int m = 0;
        for (int e = a->rp[k]; e < a->rp[k + 1]; ++e) {
            int j = a->ci[e];
            for (int u = P->rp[j]; u < P->rp[j + 1]; ++u) {
                int J = P->ci[u];
                if (mark[J] != k) { mark[J] = k; acc[J] = 0.0; list[m++] = J; }
                acc[J] = acc[J] + a->v[e] * P->v[u];
            }
        }
        sort_ints(list, m);
        if (used + m > cap) {
            while (used + m > cap) cap *= 2;
            B.ci = (int *)realloc(B.ci, sizeof(int) * (size_t)cap);
            B.v = (double *)realloc(B.v, sizeof(double) * (size_t)cap);
            if (!B.ci || !B.v) { st = OR_E_OOM; goto done; }
        }
        for (int x = 0; x < m; ++x) { B.ci[used + x] = list[x]; B.v[used + x] = acc[list[x]]; }
        used += m;
        B.rp[k + 1] = (int)used;
    }
    /* P^T: for each coarse I the rows i with P_iI stored, ascending i */
    for (long u = 0; u < P->nnz; ++u) tp[P->ci[u] + 1]++;
    for (int I = 0; I < nc; ++I) tp[I + 1] += tp[I];
    memcpy(fill, tp, sizeof(int) * (size_t)nc);
    for (int i = 0; i < n; ++i)
        for (int u = P->rp[i]; u < P->rp[i + 1]; ++u) {
            int I = P->ci[u];
            ti[fill[I]] = i;
            tv[fill[I]] = P->v[u];
            fill[I]++;
        }
    /* upper triangle: for J >= I, 0.0 + sum over i ascending of P_iI B_iJ */
    cap = 1024;
    U.ci = (int *)malloc(sizeof(int) * (size_t)cap);
    U.v = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!U.ci || !U.v) { st = OR_E_OOM; goto done; }
    for (int J = 0; J < nc; ++J) mark[J] = -1;
    used = 0;
    for (int I = 0; I < nc; ++I) {
        int m = 0;
        for (int x = tp[I]; x < tp[I + 1]; ++x) {
            int i = ti[x];
            for (int u = B.rp[i]; u < B.rp[i + 1]; ++u) {
                int J = B.ci[u];
                if (J < I) continue;
                if (mark[J] != I) { mark[J] = I; acc[J] = 0.0; list[m++] = J; }
                acc[J] = acc[J] + tv[x] * B.v[u];
            }
        }
        sort_ints(list, m);
        if (used + m > cap) {
            while (used + m > cap) cap *= 2;
            U.ci = (int *)realloc(U.ci, sizeof(int) * (size_t)cap);
            U.v = (double *)realloc(U.v, sizeof(double) * (size_t)cap);
            if (!U.ci || !U.v) { st = OR_E_OOM; goto done; }
        }
        for (int x = 0; x < m; ++x) { U.ci[used + x] = list[x]; U.v[used + x] = acc[list[x]]; }
        used += m;
        U.rp[I + 1] = (int)used;
    }
    /* full rows: the mirrored entries (J < I) in ascending J, then the upper row */
    for (int I = 0; I <= nc; ++I) fill[I] = 0;
    for (int I = 0; I < nc; ++I)
        for (int u = U.rp[I]; u < U.rp[I + 1]; ++u) {
            fill[I + 1]++;
            if (U.ci[u] != I) fill[U.ci[u] + 1]++;
        }
    for (int I = 0; I < nc; ++I) fill[I + 1] += fill[I];
    out->n = nc;
    out->nnz = fill[nc];
    out->rp = (int *)malloc(sizeof(int) * ((size_t)nc + 1));
    out->ci = (int *)malloc(sizeof(int) * (size_t)(out->nnz > 0 ? out->nnz : 1));
    out->v = (double *)malloc(sizeof(double) * (size_t)(out->nnz > 0 ? out->nnz : 1));
    if (!out->rp || !out->ci || !out->v) { st = OR_E_OOM; goto done; }
    memcpy(out->rp, fill, sizeof(int) * ((size_t)nc + 1));
    for (int I = 0; I < nc; ++I) mark[I] = out->rp[I];
    for (int I = 0; I < nc; ++I)
        for (int u = U.rp[I]; u < U.rp[I + 1]; ++u) {
            int J = U.ci[u];
            if (J != I) { out->ci[mark[J]] = I; out->v[mark[J]] = U.v[u]; mark[J]++; }
        }
    for (int I = 0; I < nc; ++I)
        for (int u = U.rp[I]; u < U.rp[I + 1]; ++u) { out->ci[mark[I]] = U.ci[u]; out->v[mark[I]] = U.v[u]; mark[I]++; }
done:
    free(acc); free(mark); free(list); free(tp); free(ti); free(tv); free(fill);
    csr_free(&B); csr_free(&U);
    return st;
}

/* ------------------------------------------------- l1 diagonal (R1) */

static int l1_inverse(const or_csr *a, double *dinv) {
    for (int i = 0; i < a->n; ++i) {
        double d = 0.0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) d += fabs(a->v[k]);
        if (!(d > 0.0)) return OR_E_NUMERIC;
        dinv[i] = 1.0 / d;
    }
    return OR_OK;
}

/* ------------------------------------------ dense Cholesky (coarsest, R9) */

static int dense_cholesky(const or_csr *a, double **out) {
    int n = a->n;
    double *L = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    if (!L) return OR_E_OOM;
    for (int i = 0; i < n; ++i)
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) L[(size_t)i * n + a->ci[k]] = a->v[k];
    /* left-looking column algorithm on the lower triangle */
    for (int j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) { free(L); return OR_E_NOT_SPD; }
        double d = sqrt(s);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / d;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) L[(size_t)i * n + j] = 0.0;
    *out = L;
    return OR_OK;
}

/* ------------------------------------------------------------ setup */

/* ------------------------------------------ aggregate-size composition (R12) */

/* Keep levels 0, s, 2s, ... and the coarsest; compose the prolongators in
 * between (agg along the chain, p multiplied finest first). */
static int compose_levels(or_hier *h, int s) {
    const int L = h->nlev - 1;
    int kept[OR_MAX_LEVELS], nk = 0;
    for (int l = 0; l < L; l += s) kept[nk++] = l;
    kept[nk++] = L;
    for (int j = 0; j < nk; ++j) h->kept[j] = kept[j];
    or_hier tmp;
    memset(&tmp, 0, sizeof(tmp));
    for (int j = 0; j < nk; ++j) {
        const int a = kept[j];
        tmp.A[j] = h->A[a];
        tmp.w[j] = h->w[a];
        tmp.dinv[j] = h->dinv[a];
        h->A[a].rp = NULL; h->A[a].ci = NULL; h->A[a].v = NULL;
        h->w[a] = NULL; h->dinv[a] = NULL;
        if (j + 1 == nk) break;
        const int b = kept[j + 1], n = tmp.A[j].n;
        int *agg = (int *)malloc(sizeof(int) * (size_t)n);
        double *p = (double *)malloc(sizeof(double) * (size_t)n);
        if (!agg || !p) { free(agg); free(p); return OR_E_OOM; }
        for (int i = 0; i < n; ++i) {
            int I = h->agg[a][i];
            double pc = h->p[a][i];
            for (int m = a + 1; m < b; ++m) {
                pc = pc * h->p[m][I];
                I = h->agg[m][I];
            }
            agg[i] = I;
            p[i] = pc;
        }
        tmp.agg[j] = agg;
        tmp.p[j] = p;
        tmp.n_pairs[j] = h->n_pairs[a];
    }
    /* free what was not moved, then install the kept levels */
    for (int l = 0; l < OR_MAX_LEVELS; ++l) {
        csr_free(&h->A[l]);
        free(h->w[l]); free(h->dinv[l]); free(h->agg[l]); free(h->p[l]);
        h->w[l] = NULL; h->dinv[l] = NULL; h->agg[l] = NULL; h->p[l] = NULL; h->n_pairs[l] = 0;
    }
    for (int j = 0; j < nk; ++j) {
        h->A[j] = tmp.A[j];
        h->w[j] = tmp.w[j];
        h->dinv[j] = tmp.dinv[j];
        h->agg[j] = tmp.agg[j];
        h->p[j] = tmp.p[j];
        h->n_pairs[j] = tmp.n_pairs[j];
    }
    h->nlev = nk;
    return OR_OK;
}

/* R15 with aggregate-size composition (R12): from each kept level K, up to
 * s pairwise steps -- matching, aggregates and the tentative Galerkin product
 * between steps, every stop rule applied to every step -- give the composed
 * aggregates and p of K; K's prolongator is that composed tentative one
 * smoothed with K, and the next kept level is P^T K P. */
static int build_smoothed_composed(or_hier *h, int s, int max_coarse, int max_levels, int max_dense,
                                   double min_ratio, int match_all) {
    int j = 0, st = OR_OK;
    for (;;) {
        or_csr *K = &h->A[j];
        h->dinv[j] = (double *)malloc(sizeof(double) * (size_t)K->n);
        if (!h->dinv[j]) return OR_E_OOM;
        st = l1_inverse(K, h->dinv[j]);
        if (st) return st;
        if (K->n <= max_coarse || j + 1 >= max_levels) break;
        int n = K->n, steps = 0, nc = 0;
        long first_pairs = 0;
        int *cagg = (int *)malloc(sizeof(int) * (size_t)n);
        double *cp = (double *)malloc(sizeof(double) * (size_t)n);
        if (!cagg || !cp) { free(cagg); free(cp); return OR_E_OOM; }
        or_csr own;                       /* the chain's current matrix once it is not K */
        memset(&own, 0, sizeof(own));
        const or_csr *C = K;
        double *wc = h->w[j], *w_own = NULL;
        for (int m = 0; m < s; ++m) {
            if (m > 0 && C->n <= max_coarse) break;
            int *mate = (int *)malloc(sizeof(int) * (size_t)C->n);
            if (!mate) { st = OR_E_OOM; break; }
            long pairs = greedy_matching(C, wc, match_all, mate);
            if (pairs < 0) { free(mate); st = OR_E_OOM; break; }
            if (pairs == 0 || (C->n <= max_dense && (double)C->n < min_ratio * (double)(C->n - pairs))) {
                free(mate);
                break;
            }
            if (m == 0) first_pairs = pairs;
            int *agg = (int *)malloc(sizeof(int) * (size_t)C->n);
            double *p = (double *)malloc(sizeof(double) * (size_t)C->n);
            double *wn = (double *)malloc(sizeof(double) * (size_t)C->n);
            if (!agg || !p || !wn) { free(mate); free(agg); free(p); free(wn); st = OR_E_OOM; break; }
            nc = build_aggregates(C->n, mate, wc, agg, p, wn);
            free(mate);
            if (m == 0) {
                memcpy(cagg, agg, sizeof(int) * (size_t)n);
                memcpy(cp, p, sizeof(double) * (size_t)n);
            } else {
                for (int i = 0; i < n; ++i) {          /* finest first, as R12 */
                    int I = cagg[i];
                    cp[i] = cp[i] * p[I];
                    cagg[i] = agg[I];
                }
            }
            or_csr next;
            memset(&next, 0, sizeof(next));
            if (m + 1 < s) st = galerkin(C, agg, p, nc, &next);   /* tentative, for the next step */
            else next.n = nc;
            free(agg); free(p);
            csr_free(&own);
            own = next;
            C = &own;
            free(w_own);
            w_own = wn;
            wc = wn;
            ++steps;
            if (st) break;
        }
        csr_free(&own);
        if (st || steps == 0) {
            free(cagg); free(cp); free(w_own);
            if (st) return st;
            break;                                    /* K is the coarsest level */
        }
        h->n_pairs[j] = (int)first_pairs;
        h->agg[j] = cagg;
        h->p[j] = cp;
        h->w[j + 1] = w_own;
        st = smoothed_prolongator(K, cagg, cp, &h->P[j], &h->omega_p[j]);
        if (!st) st = galerkin_smoothed(K, &h->P[j], nc, &h->A[j + 1]);
        if (st) return st;
        ++j;
    }
    h->nlev = j + 1;
    return OR_OK;
}

/* Copy the pairwise aggregates and prolongators (before any composition). */
static int keep_pairwise_chain(or_hier *h) {
    h->pw_nlev = h->nlev;
    for (int m = 0; m < h->nlev; ++m) {
        h->pw_n[m] = h->A[m].n;
        h->kept[m] = m;
        if (m + 1 == h->nlev) break;
        size_t n = (size_t)h->A[m].n;
        h->pw_agg[m] = (int *)malloc(sizeof(int) * n);
        h->pw_p[m] = (double *)malloc(sizeof(double) * n);
        if (!h->pw_agg[m] || !h->pw_p[m]) return OR_E_OOM;
        memcpy(h->pw_agg[m], h->agg[m], sizeof(int) * n);
        memcpy(h->pw_p[m], h->p[m], sizeof(double) * n);
    }
    return OR_OK;
}

static int validate(int n, const int *rp, const int *ci, const double *v) {
    if (n <= 0 || !rp || !ci || !v) return OR_E_INVALID;
    if (rp[0] != 0) return OR_E_INVALID;
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return OR_E_INVALID;
        int has_diag = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n) return OR_E_INVALID;
            if (k > rp[i] && ci[k] <= ci[k - 1]) return OR_E_INVALID;
            if (ci[k] == i) { has_diag = 1; if (!(v[k] > 0.0)) return OR_E_INVALID; }
        }
        if (!has_diag) return OR_E_INVALID;
    }
    return OR_OK;
}

int oracle_setup(int n, const int *rp, const int *ci, const double *v,
                 int max_coarse, int max_levels, int max_dense, double min_ratio, int match_all,
                 int agg_steps, int smooth_p, or_hier **out) {
    *out = NULL;
    int st = validate(n, rp, ci, v);
    if (st) return st;
    if (max_levels < 1 || max_levels > OR_MAX_LEVELS || agg_steps < 1) return OR_E_INVALID;
    or_hier *h = (or_hier *)calloc(1, sizeof(or_hier));
    if (!h) return OR_E_OOM;
    or_csr *A0 = &h->A[0];
    long nnz = rp[n];
    A0->n = n; A0->nnz = nnz;
    A0->rp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    A0->ci = (int *)malloc(sizeof(int) * (size_t)nnz);
    A0->v = (double *)malloc(sizeof(double) * (size_t)nnz);
    h->w[0] = (double *)malloc(sizeof(double) * (size_t)n);
    if (!A0->rp || !A0->ci || !A0->v || !h->w[0]) { oracle_free(h); return OR_E_OOM; }
    memcpy(A0->rp, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(A0->ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(A0->v, v, sizeof(double) * (size_t)nnz);
    for (int i = 0; i < n; ++i) h->w[0][i] = 1.0;         /* R2 */

    if (smooth_p && agg_steps > 1) {                         /* R15 with R12 */
        st = build_smoothed_composed(h, agg_steps, max_coarse, max_levels, max_dense, min_ratio, match_all);
        if (st) { oracle_free(h); return st; }
        h->smoothed = 1;
        int L = h->nlev - 1;
        if (h->A[L].n > max_dense) { oracle_free(h); return OR_E_STALLED; }
        st = dense_cholesky(&h->A[L], &h->chol);
        if (st) { oracle_free(h); return st; }
        *out = h;
        return OR_OK;
    }

    int l = 0;
    for (;;) {
        or_csr *A = &h->A[l];
        h->dinv[l] = (double *)malloc(sizeof(double) * (size_t)A->n);
        if (!h->dinv[l]) { oracle_free(h); return OR_E_OOM; }
        st = l1_inverse(A, h->dinv[l]);
        if (st) { oracle_free(h); return st; }
        if (A->n <= max_coarse || l + 1 >= max_levels) break;
        int *mate = (int *)malloc(sizeof(int) * (size_t)A->n);
        if (!mate) { oracle_free(h); return OR_E_OOM; }
        long pairs = greedy_matching(A, h->w[l], match_all, mate);
        if (pairs < 0) { free(mate); oracle_free(h); return OR_E_OOM; }
        if (pairs == 0) { free(mate); break; }               /* stall: this level is coarsest */
        if (A->n <= max_dense && (double)A->n < min_ratio * (double)(A->n - pairs)) {
            free(mate);                                       /* R11: too little reduction */
            break;
        }
        h->n_pairs[l] = (int)pairs;
        h->agg[l] = (int *)malloc(sizeof(int) * (size_t)A->n);
        h->p[l] = (double *)malloc(sizeof(double) * (size_t)A->n);
        h->w[l + 1] = (double *)malloc(sizeof(double) * (size_t)A->n);
        if (!h->agg[l] || !h->p[l] || !h->w[l + 1]) { free(mate); oracle_free(h); return OR_E_OOM; }
        int nc = build_aggregates(A->n, mate, h->w[l], h->agg[l], h->p[l], h->w[l + 1]);
        free(mate);
        if (smooth_p) {                                          /* R15 */
            st = smoothed_prolongator(A, h->agg[l], h->p[l], &h->P[l], &h->omega_p[l]);
            if (!st) st = galerkin_smoothed(A, &h->P[l], nc, &h->A[l + 1]);
        } else {
            st = galerkin(A, h->agg[l], h->p[l], nc, &h->A[l + 1]);
        }
        if (st) { oracle_free(h); return st; }
        ++l;
    }
    h->nlev = l + 1;
    h->smoothed = smooth_p ? 1 : 0;
    if (h->A[l].n > max_dense) { oracle_free(h); return OR_E_STALLED; }
    st = keep_pairwise_chain(h);
    if (st) { oracle_free(h); return st; }
    if (agg_steps > 1) {
        st = compose_levels(h, agg_steps);
        if (st) { oracle_free(h); return st; }
        l = h->nlev - 1;
    }
    st = dense_cholesky(&h->A[l], &h->chol);
    if (st) { oracle_free(h); return st; }
    *out = h;
    return OR_OK;
}

/* R13: the hierarchy of h rebuilt for new values v of A_0 (the pattern of
 * h's A_0).  The pairwise chain is re-run with its stored aggregates and
 * prolongators; the kept levels take their matrices from it. */
static double *dup_doubles(const double *a, size_t n) {
    double *b = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (b && n) memcpy(b, a, sizeof(double) * n);
    return b;
}

static int *dup_ints(const int *a, size_t n) {
    int *b = (int *)malloc(sizeof(int) * (n ? n : 1));
    if (b && n) memcpy(b, a, sizeof(int) * n);
    return b;
}

int oracle_update(const or_hier *h, const double *v, or_hier **out) {
    *out = NULL;
    const or_csr *A0 = &h->A[0];
    if (!v || h->pw_nlev < 1 || h->smoothed) return OR_E_INVALID;   /* R15: P depends on A */
    int st = validate(A0->n, A0->rp, A0->ci, v);
    if (st) return st;
    or_hier *g = (or_hier *)calloc(1, sizeof(or_hier));
    if (!g) return OR_E_OOM;
    or_csr chain[OR_MAX_LEVELS];
    memset(chain, 0, sizeof(chain));
    chain[0].n = A0->n;
    chain[0].nnz = A0->nnz;
    chain[0].rp = dup_ints(A0->rp, (size_t)A0->n + 1);
    chain[0].ci = dup_ints(A0->ci, (size_t)A0->nnz);
    chain[0].v = dup_doubles(v, (size_t)A0->nnz);
    if (!chain[0].rp || !chain[0].ci || !chain[0].v) st = OR_E_OOM;
    for (int m = 0; !st && m + 1 < h->pw_nlev; ++m)
        st = galerkin(&chain[m], h->pw_agg[m], h->pw_p[m], h->pw_n[m + 1], &chain[m + 1]);
    g->nlev = h->nlev;
    for (int j = 0; !st && j < h->nlev; ++j) {
        const int m = h->kept[j], n = chain[m].n;
        g->A[j] = chain[m];
        memset(&chain[m], 0, sizeof(or_csr));
        g->dinv[j] = (double *)malloc(sizeof(double) * (size_t)n);
        g->w[j] = dup_doubles(h->w[j], (size_t)n);
        if (!g->dinv[j] || !g->w[j]) { st = OR_E_OOM; break; }
        st = l1_inverse(&g->A[j], g->dinv[j]);
        if (st) break;
        if (j + 1 < h->nlev) {
            g->agg[j] = dup_ints(h->agg[j], (size_t)n);
            g->p[j] = dup_doubles(h->p[j], (size_t)n);
            if (!g->agg[j] || !g->p[j]) { st = OR_E_OOM; break; }
            g->n_pairs[j] = h->n_pairs[j];
        }
    }
    g->smoother = h->smoother; g->gs_nu = h->gs_nu; g->gs_nb = h->gs_nb; g->gs_omega = h->gs_omega;
    g->pw_nlev = h->pw_nlev;
    for (int m = 0; !st && m < h->pw_nlev; ++m) {
        g->pw_n[m] = h->pw_n[m];
        g->kept[m] = h->kept[m];
        if (m + 1 == h->pw_nlev) break;
        g->pw_agg[m] = dup_ints(h->pw_agg[m], (size_t)h->pw_n[m]);
        g->pw_p[m] = dup_doubles(h->pw_p[m], (size_t)h->pw_n[m]);
        if (!g->pw_agg[m] || !g->pw_p[m]) st = OR_E_OOM;
    }
    for (int m = 0; m < OR_MAX_LEVELS; ++m) csr_free(&chain[m]);
    if (!st) st = dense_cholesky(&g->A[g->nlev - 1], &g->chol);
    if (st) { oracle_free(g); return st; }
    *out = g;
    return OR_OK;
}

/* Copy of a hierarchy with A_l, dinv_l, p_l and the Cholesky factor rounded to
 * binary32 (stored as binary64).  Aggregates are those of the FP64 build. */
int oracle_round_f32(const or_hier *h, or_hier **out) {
    *out = NULL;
    or_hier *g = (or_hier *)calloc(1, sizeof(or_hier));
    if (!g) return OR_E_OOM;
    g->nlev = h->nlev;
    g->smoother = h->smoother; g->gs_nu = h->gs_nu; g->gs_nb = h->gs_nb; g->gs_omega = h->gs_omega;
    for (int l = 0; l < h->nlev; ++l) {
        const or_csr *a = &h->A[l];
        or_csr *b = &g->A[l];
        b->n = a->n; b->nnz = a->nnz;
        b->rp = (int *)malloc(sizeof(int) * ((size_t)a->n + 1));
        b->ci = (int *)malloc(sizeof(int) * (size_t)a->nnz);
        b->v = (double *)malloc(sizeof(double) * (size_t)a->nnz);
        g->dinv[l] = (double *)malloc(sizeof(double) * (size_t)a->n);
        g->w[l] = (double *)malloc(sizeof(double) * (size_t)a->n);
        if (!b->rp || !b->ci || !b->v || !g->dinv[l] || !g->w[l]) { oracle_free(g); return OR_E_OOM; }
        memcpy(b->rp, a->rp, sizeof(int) * ((size_t)a->n + 1));
        memcpy(b->ci, a->ci, sizeof(int) * (size_t)a->nnz);
        for (long k = 0; k < a->nnz; ++k) b->v[k] = (double)(float)a->v[k];
        for (int i = 0; i < a->n; ++i) {
            g->dinv[l][i] = (double)(float)h->dinv[l][i];
            g->w[l][i] = h->w[l][i];
        }
        if (l + 1 < h->nlev) {
            g->agg[l] = (int *)malloc(sizeof(int) * (size_t)a->n);
            g->p[l] = (double *)malloc(sizeof(double) * (size_t)a->n);
            if (!g->agg[l] || !g->p[l]) { oracle_free(g); return OR_E_OOM; }
            memcpy(g->agg[l], h->agg[l], sizeof(int) * (size_t)a->n);
            for (int i = 0; i < a->n; ++i) g->p[l][i] = (double)(float)h->p[l][i];
            g->n_pairs[l] = h->n_pairs[l];
            if (h->smoothed) {
                const or_csr *P = &h->P[l];
                or_csr *Q = &g->P[l];
                Q->n = P->n; Q->nnz = P->nnz;
                Q->rp = (int *)malloc(sizeof(int) * ((size_t)P->n + 1));
                Q->ci = (int *)malloc(sizeof(int) * (size_t)(P->nnz > 0 ? P->nnz : 1));
                Q->v = (double *)malloc(sizeof(double) * (size_t)(P->nnz > 0 ? P->nnz : 1));
                if (!Q->rp || !Q->ci || !Q->v) { oracle_free(g); return OR_E_OOM; }
                memcpy(Q->rp, P->rp, sizeof(int) * ((size_t)P->n + 1));
                memcpy(Q->ci, P->ci, sizeof(int) * (size_t)P->nnz);
                for (long k = 0; k < P->nnz; ++k) Q->v[k] = (double)(float)P->v[k];
            }
        }
    }
    g->smoothed = h->smoothed;
    int nL = h->A[h->nlev - 1].n;
    g->chol = (double *)malloc(sizeof(double) * (size_t)nL * (size_t)nL);
    if (!g->chol) { oracle_free(g); return OR_E_OOM; }
    for (size_t k = 0; k < (size_t)nL * (size_t)nL; ++k) g->chol[k] = (double)(float)h->chol[k];
    *out = g;
    return OR_OK;
}

/* ------------------------------------------------------- accessors */

int oracle_nlevels(const or_hier *h) { return h->nlev; }
int oracle_level_n(const or_hier *h, int l) { return h->A[l].n; }
long oracle_level_nnz(const or_hier *h, int l) { return h->A[l].nnz; }
int oracle_level_pairs(const or_hier *h, int l) { return h->n_pairs[l]; }

void oracle_get_level(const or_hier *h, int l, int *rp, int *ci, double *v) {
    const or_csr *a = &h->A[l];
    memcpy(rp, a->rp, sizeof(int) * ((size_t)a->n + 1));
    memcpy(ci, a->ci, sizeof(int) * (size_t)a->nnz);
    memcpy(v, a->v, sizeof(double) * (size_t)a->nnz);
}
void oracle_get_agg(const or_hier *h, int l, int *agg) { memcpy(agg, h->agg[l], sizeof(int) * (size_t)h->A[l].n); }
void oracle_get_p(const or_hier *h, int l, double *p) { memcpy(p, h->p[l], sizeof(double) * (size_t)h->A[l].n); }
void oracle_get_w(const or_hier *h, int l, double *w) { memcpy(w, h->w[l], sizeof(double) * (size_t)h->A[l].n); }
long oracle_prolongator_nnz(const or_hier *h, int l) { return h->smoothed ? h->P[l].nnz : 0; }
double oracle_prolongator_omega(const or_hier *h, int l) { return h->omega_p[l]; }
void oracle_get_prolongator(const or_hier *h, int l, int *rp, int *ci, double *v) {
    const or_csr *P = &h->P[l];
    memcpy(rp, P->rp, sizeof(int) * ((size_t)P->n + 1));
    memcpy(ci, P->ci, sizeof(int) * (size_t)P->nnz);
    memcpy(v, P->v, sizeof(double) * (size_t)P->nnz);
}
void oracle_get_dinv(const or_hier *h, int l, double *d) { memcpy(d, h->dinv[l], sizeof(double) * (size_t)h->A[l].n); }
void oracle_get_chol(const or_hier *h, double *L) {
    int n = h->A[h->nlev - 1].n;
    memcpy(L, h->chol, sizeof(double) * (size_t)n * (size_t)n);
}

/* ------------------------------------------------ operators (Sec. 3.1) */

void oracle_spmv(const or_hier *h, int l, const double *x, double *y) { csr_mv(&h->A[l], x, y); }

/* r_c = P_l^T t: members of each aggregate added in ascending fine index */
void oracle_restrict(const or_hier *h, int l, const double *t, double *rc) {
    int nc = h->A[l + 1].n;
    for (int I = 0; I < nc; ++I) rc[I] = 0.0;
    if (h->smoothed) {                                           /* P^T t, ascending i (R15) */
        const or_csr *P = &h->P[l];
        for (int i = 0; i < P->n; ++i)
            for (int u = P->rp[i]; u < P->rp[i + 1]; ++u) rc[P->ci[u]] += P->v[u] * t[i];
        return;
    }
    for (int i = 0; i < h->A[l].n; ++i) rc[h->agg[l][i]] += h->p[l][i] * t[i];
}

/* z += P_l e */
void oracle_prolong_add(const or_hier *h, int l, const double *e, double *z) {
    if (h->smoothed) {                                           /* z += P e (R15) */
        const or_csr *P = &h->P[l];
        for (int i = 0; i < P->n; ++i) {
            double s = 0.0;
            for (int u = P->rp[i]; u < P->rp[i + 1]; ++u) s += P->v[u] * e[P->ci[u]];
            z[i] += s;
        }
        return;
    }
    OR_PARALLEL_FOR
    for (int i = 0; i < h->A[l].n; ++i) z[i] += h->p[l][i] * e[h->agg[l][i]];
}

/* z = A_L^{-1} r by forward then backward substitution with the dense factor */
void oracle_coarse_solve(const or_hier *h, const double *r, double *z) {
    int n = h->A[h->nlev - 1].n;
    const double *L = h->chol;
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * z[k];
        z[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * z[k];
        z[i] = s / L[(size_t)i * n + i];
    }
}

/* ------------------------------------- hybrid Gauss-Seidel smoother (R14) */

int oracle_set_smoother(or_hier *h, int kind, int nu, int nb, double omega) {
    if (kind == 0) { h->smoother = 0; return OR_OK; }
    if (kind != 1 || nu < 1 || nb < 1 || !(omega > 0.0)) return OR_E_INVALID;
    h->smoother = 1; h->gs_nu = nu; h->gs_nb = nb; h->gs_omega = omega;
    return OR_OK;
}

/* order[q] = the level-l unknown at nested position q (R14) */
void oracle_nested_order(const or_hier *h, int l, int *order) {
    int L = h->nlev - 1;
    for (int q = 0; q < h->A[L].n; ++q) order[q] = q;
    for (int m = L - 1; m >= l; --m) {
        int nf = h->A[m].n, nc = h->A[m + 1].n;
        int *size = (int *)calloc((size_t)nc, sizeof(int));
        int *first = (int *)malloc(sizeof(int) * (size_t)nc);
        int *finer = (int *)malloc(sizeof(int) * (size_t)nf);
        for (int i = 0; i < nf; ++i) size[h->agg[m][i]]++;
        /* coarse unknowns in their nested order, each followed by its members */
        int acc = 0;
        for (int q = 0; q < nc; ++q) { first[order[q]] = acc; acc += size[order[q]]; }
        for (int i = 0; i < nf; ++i) finer[first[h->agg[m][i]]++] = i;   /* ascending i */
        memcpy(order, finer, sizeof(int) * (size_t)nf);
        free(size); free(first); free(finer);
    }
}

/* one sweep x_new = x_old + M^-1 (r - A x_old), M = blockdiag(omega (L+D))
   (forward) or its transpose (backward) over nested-order blocks: within a
   block the correction d solves (L_pp + D_pp) d = (r - A x_old)_p by
   substitution in nested order, and x_new = x_old + d / omega */
static void hgs_sweep(const or_hier *h, int l, const int *order, const int *pos, int backward,
                      const double *r, const double *x_old, double *x_new, double *d) {
    const or_csr *a = &h->A[l];
    int n = a->n, nb = h->gs_nb;
    for (int b0 = 0; b0 < n; b0 += nb) {
        int b1 = b0 + nb < n ? b0 + nb : n;
        for (int s = 0; s < b1 - b0; ++s) {
            int q = backward ? b1 - 1 - s : b0 + s;
            int i = order[q];
            double old = 0.0, fresh = 0.0, aii = 0.0;
            for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
                int j = a->ci[k], qj = pos[j];
                old += a->v[k] * x_old[j];
                if (qj >= b0 && qj < b1 && (backward ? qj > q : qj < q)) fresh += a->v[k] * d[j];
                if (j == i) aii = a->v[k];
            }
            d[i] = ((r[i] - old) - fresh) / aii;
        }
        for (int q = b0; q < b1; ++q) {
            int i = order[q];
            x_new[i] = x_old[i] + d[i] / h->gs_omega;
        }
    }
}

/* x <- nu sweeps (forward from x = 0 if zero_start, else backward from x) */
void oracle_hgs_smooth(const or_hier *h, int l, int backward, int zero_start, const double *r, double *x) {
    int n = h->A[l].n;
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_nested_order(h, l, order);
    for (int q = 0; q < n; ++q) pos[order[q]] = q;
    if (zero_start)
        for (int i = 0; i < n; ++i) x[i] = 0.0;
    for (int s = 0; s < h->gs_nu; ++s) {
        hgs_sweep(h, l, order, pos, backward, r, x, y, d);
        memcpy(x, y, sizeof(double) * (size_t)n);
    }
    free(order); free(pos); free(y); free(d);
}

/* z = V(l, r): eq. (multiplicative_composition); smoother R1 (nu = 1,
   M = diag(l1)) or R14 (nu hybrid Gauss-Seidel sweeps) */
void oracle_vcycle(const or_hier *h, int l, const double *r, double *z) {
    int L = h->nlev - 1;
    if (l == L) { oracle_coarse_solve(h, r, z); return; }
    if (h->smoother == 1) {
        int n = h->A[l].n, nc = h->A[l + 1].n;
        double *t = (double *)malloc(sizeof(double) * (size_t)n);
        double *rc = (double *)malloc(sizeof(double) * (size_t)nc);
        double *e = (double *)malloc(sizeof(double) * (size_t)nc);
        oracle_hgs_smooth(h, l, 0, 1, r, z);                    /* pre-smooth: forward from zero */
        csr_mv(&h->A[l], z, t);
        for (int i = 0; i < n; ++i) t[i] = r[i] - t[i];         /* residual */
        oracle_restrict(h, l, t, rc);
        oracle_vcycle(h, l + 1, rc, e);
        oracle_prolong_add(h, l, e, z);
        oracle_hgs_smooth(h, l, 1, 0, r, z);                    /* post-smooth: backward */
        free(t); free(rc); free(e);
        return;
    }
    int n = h->A[l].n, nc = h->A[l + 1].n;
    const double *dinv = h->dinv[l];
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *rc = (double *)malloc(sizeof(double) * (size_t)nc);
    double *e = (double *)malloc(sizeof(double) * (size_t)nc);
    OR_PARALLEL_FOR
    for (int i = 0; i < n; ++i) z[i] = dinv[i] * r[i];          /* pre-smooth from zero */
    csr_mv(&h->A[l], z, t);
    OR_PARALLEL_FOR
    for (int i = 0; i < n; ++i) t[i] = r[i] - t[i];             /* residual */
    oracle_restrict(h, l, t, rc);                               /* restriction */
    oracle_vcycle(h, l + 1, rc, e);                             /* coarse correction */
    oracle_prolong_add(h, l, e, z);                             /* prolongation */
    csr_mv(&h->A[l], z, t);
    OR_PARALLEL_FOR
    for (int i = 0; i < n; ++i) z[i] += dinv[i] * (r[i] - t[i]); /* post-smooth */
    free(t); free(rc); free(e);
}

/* ---------------------------------------------------- Krylov (Sec. 5, R10) */

/*
 * krylov: 0 = PCG, 1 = FCG(1).  use_x0: x holds the initial guess on entry.
 * fixed_iters > 0: run exactly that many iterations and ignore tol.
 * true_res: at convergence recompute b - A x; if it exceeds tol*||b||, restart
 * the recurrence from it (at most 10 restarts).
 * Outputs: x, *iters, *relres (recurrence residual / ||b||).
 */
int oracle_solve(const or_hier *h, const double *b, double *x, double tol, int maxit,
                 int krylov, int use_x0, int fixed_iters, int true_res,
                 int *iters, double *relres) {
    int n = h->A[0].n;
    const or_csr *A = &h->A[0];
    *iters = 0; *relres = 0.0;
    double nb = sqrt(dot(n, b, b));
    if (!use_x0) for (int i = 0; i < n; ++i) x[i] = 0.0;
    if (nb == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        return OR_OK;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return OR_E_OOM; }
    int status = OR_NOT_CONVERGED;
    int it = 0, restarts = 0;
    double rn = 0.0;
restart:
    csr_mv(A, x, q);
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    rn = sqrt(dot(n, r, r));
    if (fixed_iters <= 0 && rn <= tol * nb) { status = OR_OK; goto done; }
    {
        double rho_old = 0.0, delta_old = 0.0;
        for (int k = 0; ; ++k) {
            if (fixed_iters > 0 ? it >= fixed_iters : it >= maxit) { status = fixed_iters > 0 ? OR_OK : OR_NOT_CONVERGED; break; }
            oracle_vcycle(h, 0, r, z);
            double alpha_num;
            if (krylov == 0) {
                double rho = dot(n, r, z);
                if (k == 0) for (int i = 0; i < n; ++i) p[i] = z[i];
                else { double beta = rho / rho_old; for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i]; }
                rho_old = rho;
                alpha_num = rho;
            } else {
                if (k == 0) for (int i = 0; i < n; ++i) p[i] = z[i];
                else {
                    double beta = -dot(n, z, q) / delta_old;      /* q holds q_old here */
                    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
                }
                alpha_num = 0.0;                                  /* set after q */
            }
            csr_mv(A, p, q);
            double delta = dot(n, p, q);
            if (!(delta > 0.0)) { status = OR_E_NOT_SPD; goto done; }
            if (krylov != 0) alpha_num = dot(n, p, r);
            double alpha = alpha_num / delta;
            OR_PARALLEL_FOR
            for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            delta_old = delta;
            ++it;
            rn = sqrt(dot(n, r, r));
            if (!(rn == rn)) { status = OR_E_NUMERIC; goto done; }
            if (fixed_iters <= 0 && rn <= tol * nb) { status = OR_OK; break; }
        }
    }
    if (status == OR_OK && true_res && fixed_iters <= 0) {
        csr_mv(A, x, q);
        double tr = 0.0;
        for (int i = 0; i < n; ++i) { double d = b[i] - q[i]; tr += d * d; }
        if (sqrt(tr) > tol * nb && restarts < 10 && it < maxit) { ++restarts; status = OR_NOT_CONVERGED; goto restart; }
    }
done:
    *iters = it;
    *relres = rn / nb;
    free(r); free(z); free(p); free(q);
    return status;
}

/* y = A x for a caller-held CSR (no hierarchy): the plain definition, rows
 * summed in ascending column order. */
void oracle_csr_mv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y) {
    or_csr a;
    a.n = n; a.nnz = rp[n];
    a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    csr_mv(&a, x, y);
}
