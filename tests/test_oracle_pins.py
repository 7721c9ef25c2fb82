"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, library routines (numpy / scipy / networkx), brute force on tiny
inputs, invariants the paper states, and the V-cycle error-propagation
formula (Sec. 3.1, eq. multiplicative_composition).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import CSR, lap7, varcoef7, q1_stretched, q1_rhs, uniform_rhs

ULP = np.finfo(np.float64).eps


def csr_from_scipy(M) -> CSR:
    M = sp.csr_matrix(M)
    M.sort_indices()
    return CSR(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def prolongator(H, l):
    n, nc = H.n(l), H.n(l + 1)
    return sp.csr_matrix((H.p(l), (np.arange(n), H.agg(l))), shape=(n, nc))


# --------------------------------------------------------------------------- closed forms

def test_lap7_eigenpairs_through_oracle_spmv():
    # A u = lambda u for u = sin(p pi x) sin(q pi y) sin(r pi z) at the nodes,
    # lambda = (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2) + sin^2(r pi h/2)).
    n = 32
    h = 1.0 / (n + 1)
    H = oracle.Hierarchy(lap7(n))
    x = (np.arange(n) + 1) * h
    for (p, q, r) in [(1, 1, 1), (32, 32, 32), (3, 7, 20), (1, 32, 5)]:
        u = (np.sin(p * np.pi * x)[None, None, :] * np.sin(q * np.pi * x)[None, :, None]
             * np.sin(r * np.pi * x)[:, None, None]).reshape(-1)     # idx = i + n j + n^2 k
        lam = 4.0 / h ** 2 * (np.sin(p * np.pi * h / 2) ** 2 + np.sin(q * np.pi * h / 2) ** 2
                              + np.sin(r * np.pi * h / 2) ** 2)
        Au = H.spmv(0, u)
        assert np.linalg.norm(Au - lam * u) <= 1e-12 * lam * np.linalg.norm(u)
    lmin = 12.0 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    lmax = 12.0 / h ** 2 * np.sin(32 * np.pi * h / 2) ** 2
    assert lmax / lmin == pytest.approx(1.0 / np.tan(np.pi / 66) ** 2, rel=1e-12)


def test_l1_diagonal_closed_form():
    # D_ii = sum_j |a_ij|: 12/h^2 interior, 11/h^2 next to one face, 10 next to an
    # edge, 9 next to a corner (7-point stencil with Dirichlet boundary).
    n = 8
    H = oracle.Hierarchy(lap7(n), max_coarse=10 ** 9)
    inv_h2 = float((n + 1) ** 2)
    d = 1.0 / H.dinv(0)
    i = np.arange(n)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    bnd = (I == 0).astype(int) + (I == n - 1) + (J == 0) + (J == n - 1) + (K == 0) + (K == n - 1)
    expect = ((12 - bnd) * inv_h2).transpose(2, 1, 0).reshape(-1)
    assert np.array_equal(H.dinv(0), 1.0 / expect)
    assert np.allclose(d, expect, rtol=4 * ULP)


def _stencil7(nx, ny, nz, diag, cx, cy, cz):
    """Dense-free 7-point operator on an nx*ny*nz grid (x fastest)."""
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [np.full(N, diag)]
    for (a, b, c) in [(idx[:, :, :-1], idx[:, :, 1:], cx), (idx[:, :-1, :], idx[:, 1:, :], cy),
                      (idx[:-1, :, :], idx[1:, :, :], cz)]:
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [np.full(a.size, c), np.full(a.size, c)]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def test_lap7_32_first_levels_closed_form():
    # Hand derivation for the 32^3 Laplacian with w = 1:
    #  level 0: every weight equals 7/6, so the (lo, hi) tie-break pairs (i, i+1) along x;
    #  A_1 = h^-2 [5; x -1/2, y -1, z -1] on 16x32x32, weights 1.1 (x) and 1.2 (y, z) -> y pairs;
    #  A_2 = h^-2 [4; x -1/2, y -1/2, z -1] on 16x16x32, weights 1.125, 1.125, 1.25 -> z pairs;
    #  A_3 = h^-2 [3; -1/2 x 6] on 16^3 (half the 16^3 Laplacian).  No singletons.
    n = 32
    inv_h2 = 33.0 ** 2
    H = oracle.Hierarchy(lap7(n))
    assert [H.n(l) for l in range(4)] == [32768, 16384, 8192, 4096]
    assert [H.pairs(l) for l in range(3)] == [16384, 8192, 4096]
    i = np.arange(32768)
    assert np.array_equal(H.agg(0), i // 2)
    # level 1 grid 16 x 32 x 32: y pairs (j = 2m, 2m+1)
    i1 = np.arange(16384)
    x1, y1, z1 = i1 % 16, (i1 // 16) % 32, i1 // 512
    assert np.array_equal(H.agg(1), x1 + 16 * (y1 // 2) + 256 * z1)
    i2 = np.arange(8192)
    x2, y2, z2 = i2 % 16, (i2 // 16) % 16, i2 // 256
    assert np.array_equal(H.agg(2), x2 + 16 * y2 + 256 * (z2 // 2))
    expected = {1: (16, 32, 32, 5.0, -0.5, -1.0, -1.0), 2: (16, 16, 32, 4.0, -0.5, -0.5, -1.0),
                3: (16, 16, 16, 3.0, -0.5, -0.5, -0.5)}
    for l, (nx, ny, nz, d, cx, cy, cz) in expected.items():
        E = _stencil7(nx, ny, nz, d * inv_h2, cx * inv_h2, cy * inv_h2, cz * inv_h2)
        A = H.level_scipy(l)
        assert np.array_equal(A.indptr, E.indptr) and np.array_equal(A.indices, E.indices)
        assert np.allclose(A.data, E.data, rtol=8 * ULP, atol=0)
    # all the way down: 9 levels, coarsest 128 unknowns (pairs every level)
    assert H.nlevels == 9 and H.n(8) == 128


def test_1d_galerkin_halves_the_operator():
    # tridiag(-1, 2, -1) of even size: all weights 3/2 tie, pairs (2k, 2k+1),
    # p = 1/sqrt(2) and A_1 = 1/2 tridiag(-1, 2, -1).
    n = 64
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    H = oracle.Hierarchy(csr_from_scipy(T), max_coarse=32)
    assert H.nlevels == 2
    assert np.array_equal(H.agg(0), np.arange(n) // 2)
    A1 = H.level_scipy(1).toarray()
    E = 0.5 * sp.diags([-np.ones(31), 2 * np.ones(32), -np.ones(31)], [-1, 0, 1]).toarray()
    assert np.allclose(A1, E, rtol=4 * ULP, atol=4 * ULP)
    assert np.allclose(H.p(0), 1 / math.sqrt(2), rtol=ULP)


# --------------------------------------------------------------------------- matching

def test_1d_odd_size_tie_break():
    # tridiag(-1, 2, -1) of size 9: every weight ties at 3/2, so the order (lo, hi)
    # ascending decides: pairs (0,1), (2,3), (4,5), (6,7) and the singleton 8.
    n = 9
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    H = oracle.Hierarchy(csr_from_scipy(T), max_coarse=1, max_levels=2)
    assert np.array_equal(H.agg(0), [0, 0, 1, 1, 2, 2, 3, 3, 4])
    assert H.p(0)[8] == 1.0 and H.w(1)[4] == 1.0


def _random_spd(n, density, seed, discrete=False):
    rng = np.random.default_rng(seed)
    if discrete:   # few distinct values: many exact weight ties
        rvs = lambda k: rng.choice([-1.0, -0.5, -0.25, 0.25], k)
    else:
        rvs = lambda k: rng.uniform(-1, 0.3, k)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=rvs)
    M = sp.triu(M, 1)
    M = M + M.T
    d = np.asarray(abs(M).sum(axis=1)).ravel() + (0.5 if discrete else rng.uniform(0.1, 1.0, n))
    M = M + sp.diags(d)
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M


def _edge_weight(a, aii, ajj, wi, wj):
    return 1.0 - 2.0 * a * wi * wj / (aii * wi * wi + ajj * wj * wj)


def _weights_eq(a, aii, ajj, wi, wj):
    """eq. (weights) evaluated in the oracle's stated operation order (R4), so that
    ties compare exactly; numpy float64 arithmetic, one rounding per operation."""
    num = ((2.0 * a) * wi) * wj
    den = (aii * wi) * wi + (ajj * wj) * wj
    return 1.0 - num / den


def _check_matching_level(H, l, check_half_approx=True):
    """Greedy characterisation + half-approximation for level l of H."""
    import networkx as nx
    A = H.level_scipy(l)
    agg = H.agg(l)
    w = H.w(l)
    D = A.diagonal()
    Au = sp.triu(A, 1).tocoo()
    edges = {}
    for i, j, a in zip(Au.row, Au.col, Au.data):
        c = _weights_eq(a, D[i], D[j], w[i], w[j])
        if c > 1.0:
            edges[(int(i), int(j))] = c
    order = np.argsort(agg, kind="stable")
    sa = agg[order]
    M = set()
    starts = np.flatnonzero(np.r_[True, sa[1:] != sa[:-1]])
    sizes = np.diff(np.r_[starts, len(sa)])
    assert sizes.min() >= 1 and sizes.max() <= 2
    for s0, sz in zip(starts, sizes):
        if sz == 2:
            M.add((int(order[s0]), int(order[s0 + 1])))
    assert all(e in edges for e in M), "matched an ineligible edge"
    key = lambda e: (-edges[e], e[0], e[1])   # weight descending, then lo, then hi
    at = {}
    for e in M:
        at[e[0]] = e
        at[e[1]] = e
    for e in edges:
        if e in M:
            continue
        dom = [f for f in (at.get(e[0]), at.get(e[1])) if f is not None and key(f) < key(e)]
        assert dom, f"level {l}: edge {e} not dominated, so the matching is not the greedy one"
    if check_half_approx:
        G = nx.Graph()
        for (i, j), c in edges.items():
            G.add_edge(i, j, weight=math.log(c))
        opt = nx.max_weight_matching(G)
        wopt = sum(math.log(edges[(min(a, b), max(a, b))]) for a, b in opt)
        wg = sum(math.log(edges[e]) for e in M)
        assert wg >= 0.5 * wopt - 1e-12


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("discrete", [False, True])
def test_matching_greedy_characterisation_and_half_approx(seed, discrete):
    # The greedy matching under a strict total order is the unique matching M in
    # which every eligible edge outside M touches a heavier edge of M; its weight
    # is at least half the optimum (the bound the paper quotes for its matching).
    # Weight of an edge = log c (maximum product), eligible iff c > 1.
    A = _random_spd(60, 0.12, seed, discrete=discrete)
    H = oracle.Hierarchy(csr_from_scipy(A), max_coarse=1, max_levels=2)
    _check_matching_level(H, 0)


@pytest.mark.parametrize("case", ["varcoef_12", "q1_7"])
def test_matching_characterisation_on_every_level(case):
    # coarse levels carry a non-uniform w (singletons keep |w_s|, pairs get the norm)
    A = {"varcoef_12": lambda: varcoef7(12, seed=4), "q1_7": lambda: q1_stretched(7, 1.05)}[case]()
    H = oracle.Hierarchy(A, max_coarse=10)
    assert any(len(np.unique(H.w(l))) > 2 for l in range(1, H.nlevels))
    for l in range(H.nlevels - 1):
        _check_matching_level(H, l, check_half_approx=H.n(l) <= 400)


# --------------------------------------------------------------------------- invariants

CASES = {
    "lap7_10": lambda: lap7(10),
    "varcoef_9": lambda: varcoef7(9, seed=5),
    "q1_6": lambda: q1_stretched(6, 1.05),
    "q1_8_uniform": lambda: q1_stretched(8, 1.0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_aggregation_invariants(case):
    A = CASES[case]()
    H = oracle.Hierarchy(A, max_coarse=20)
    assert H.nlevels >= 2
    for l in range(H.nlevels - 1):
        n, nc = H.n(l), H.n(l + 1)
        agg = H.agg(l)
        counts = np.bincount(agg, minlength=nc)
        # a partition of {0..n-1} into aggregates of size 1 or 2; n_c = n_M + n_S >= n/2
        assert agg.min() == 0 and agg.max() == nc - 1
        assert counts.min() >= 1 and counts.max() <= 2
        assert H.pairs(l) == int((counts == 2).sum()) and nc == n - H.pairs(l)
        assert 2 * nc >= n
        # coarse numbering by smallest member ascending
        first = np.full(nc, n)
        np.minimum.at(first, agg, np.arange(n))
        assert np.all(np.diff(first) > 0)
        P = prolongator(H, l)
        # orthonormal columns and w in range(P): P^T P = I, P w_c = w
        PtP = (P.T @ P).toarray()
        assert np.allclose(PtP, np.eye(nc), rtol=0, atol=2 * ULP)
        assert np.allclose(P @ H.w(l + 1), H.w(l), rtol=2 * ULP, atol=0)
        # Galerkin product (Sec. 3.1) against scipy's triple product
        Al = H.level_scipy(l)
        Ac = H.level_scipy(l + 1)
        G = (P.T @ Al @ P).tocsr()
        assert np.allclose(Ac.toarray(), G.toarray(), rtol=1e-14, atol=1e-14 * abs(Al).max())
        # bitwise symmetric, SPD
        Ad = Ac.toarray()
        assert np.array_equal(Ad.view(np.uint64), Ad.T.view(np.uint64))
        np.linalg.cholesky(Ad)
        # A_c w_c = P^T A w
        lhs = Ac @ H.w(l + 1)
        rhs = P.T @ (Al @ H.w(l))
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(Al).max() * np.abs(H.w(l)).max())
        # pairs are eligible edges (c > 1)
        D = Al.diagonal()
        w = H.w(l)
        for I in np.nonzero(counts == 2)[0][:200]:
            i, j = np.nonzero(agg == I)[0]
            assert _edge_weight(Al[i, j], D[i], D[j], w[i], w[j]) > 1.0
    # coarsest factor against numpy's Cholesky
    L = H.chol()
    AL = H.level_scipy(H.nlevels - 1).toarray()
    assert np.allclose(L, np.linalg.cholesky(AL), rtol=1e-12, atol=1e-12 * np.sqrt(abs(AL).max()))


def test_l1_diagonal_definition_general():
    A = varcoef7(7, seed=3)
    H = oracle.Hierarchy(A, max_coarse=10)
    for l in range(H.nlevels):
        M = H.level_scipy(l)
        d = np.asarray(abs(M).sum(axis=1)).ravel()
        assert np.allclose(1.0 / H.dinv(l), d, rtol=8 * ULP)


# --------------------------------------------------------------------------- V-cycle

def _dense_B(H, l):
    """B_l from eq. (multiplicative_composition) with nu = 1, M_l = diag(l1):
    I - B_l A_l = (I - D^-1 A)(I - P B_{l+1} P^T A)(I - D^-1 A), B_L = A_L^-1."""
    A = H.level_scipy(l).toarray()
    if l == H.nlevels - 1:
        return np.linalg.inv(A)
    n = A.shape[0]
    P = prolongator(H, l).toarray()
    S = np.eye(n) - np.diag(H.dinv(l)) @ A
    C = np.eye(n) - P @ _dense_B(H, l + 1) @ P.T @ A
    E = S @ C @ S
    return (np.eye(n) - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("case", ["lap7_6", "q1_4", "varcoef_6", "lap7_8_composed"])
def test_vcycle_matches_multiplicative_composition(case):
    A = {"lap7_6": lambda: lap7(6), "q1_4": lambda: q1_stretched(4, 1.05),
         "varcoef_6": lambda: varcoef7(6, seed=8), "lap7_8_composed": lambda: lap7(8)}[case]()
    H = oracle.Hierarchy(A, max_coarse=12, agg_steps=2 if case.endswith("composed") else 1)
    assert H.nlevels >= 3
    n = H.n(0)
    Bcols = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    Bf = _dense_B(H, 0)
    assert np.allclose(Bcols, Bf, rtol=1e-10, atol=1e-10 * abs(Bf).max())
    # symmetric positive definite preconditioner
    assert np.allclose(Bcols, Bcols.T, rtol=1e-12, atol=1e-12 * abs(Bcols).max())
    assert np.linalg.eigvalsh(0.5 * (Bcols + Bcols.T)).min() > 0


def test_single_level_is_exact_inverse():
    A = lap7(5)
    H = oracle.Hierarchy(A, max_coarse=10 ** 6)
    assert H.nlevels == 1
    b = uniform_rhs(A.n, 4)
    x, it, rr, st = H.solve(b, 1e-10, krylov="cg")
    assert st == 0 and it == 1
    xs = np.linalg.solve(A.to_scipy().toarray(), b)
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)
    z = H.coarse_solve(b)
    import scipy.linalg as sl
    assert np.allclose(z, sl.cho_solve(sl.cho_factor(A.to_scipy().toarray(), lower=True), b), rtol=1e-13)


# --------------------------------------------------------------------------- Krylov

@pytest.mark.parametrize("krylov", ["cg", "fcg"])
def test_krylov_matches_dense_solve(krylov):
    for A in (lap7(8), q1_stretched(5, 1.05), varcoef7(8, seed=2)):
        H = oracle.Hierarchy(A, max_coarse=30)
        b = uniform_rhs(A.n, 9)
        Ad = A.to_scipy().toarray()
        xs = np.linalg.solve(Ad, b)
        x, it, rr, st = H.solve(b, 1e-13, krylov=krylov)
        assert st == 0 and rr <= 1e-13
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)
        # recurrence residual matches the true one
        assert np.linalg.norm(b - Ad @ x) <= 2e-13 * np.linalg.norm(b)


def test_manufactured_solution():
    # b = A u for u = sin(pi x) sin(2 pi y) sin(3 pi z) + x(1-x)y(1-y)z(1-z):
    # ||x - u|| / ||u|| <= kappa * tol.
    n = 24
    A = lap7(n)
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1) * h
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    u = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(3 * np.pi * Z)
         + X * (1 - X) * Y * (1 - Y) * Z * (1 - Z)).reshape(-1)
    b = A.to_scipy() @ u
    H = oracle.Hierarchy(A)
    tol = 1e-8
    kappa = 1.0 / np.tan(np.pi * h / 2) ** 2
    for krylov in ("cg", "fcg"):
        x, it, rr, st = H.solve(b, tol, krylov=krylov)
        assert st == 0
        assert np.linalg.norm(x - u) <= kappa * tol * np.linalg.norm(u)


def test_pcg_and_fcg_agree_for_symmetric_preconditioner():
    A = lap7(16)
    b = uniform_rhs(A.n, 1)
    H = oracle.Hierarchy(A)
    x1, i1, r1, s1 = H.solve(b, 1e-8, krylov="cg")
    x2, i2, r2, s2 = H.solve(b, 1e-8, krylov="fcg")
    assert s1 == s2 == 0 and abs(i1 - i2) <= 1
    assert np.linalg.norm(x1 - x2) <= 1e-7 * np.linalg.norm(x1)


def test_fixed_iterations_and_warm_start():
    A = lap7(10)
    b = uniform_rhs(A.n, 3)
    H = oracle.Hierarchy(A)
    x5, it, rr5, st = H.solve(b, 0.0, fixed_iters=5)
    assert it == 5 and st == 0
    x_all, it_all, _, _ = H.solve(b, 1e-9)
    # warm start from a converged solution returns immediately
    x_w, it_w, _, st_w = H.solve(b, 1e-9, x0=x_all)
    assert it_w == 0 and st_w == 0 and np.array_equal(x_w, x_all)
    # zero right-hand side
    xz, itz, _, stz = H.solve(np.zeros(A.n), 1e-6)
    assert itz == 0 and stz == 0 and not xz.any()


def test_diag_level_count_doubling_claim_of_plain_cg():
    # Without multigrid the iteration count of diagonally preconditioned CG roughly
    # doubles per halving of h; the V-cycle keeps it nearly flat.  (Qualitative,
    # as in the paper's motivation; only the multigrid side runs through the oracle.)
    its = []
    for n in (8, 16, 32):
        A = lap7(n)
        H = oracle.Hierarchy(A)
        _, it, _, st = H.solve(uniform_rhs(A.n, 1), 1e-6, krylov="cg")
        assert st == 0
        its.append(it)
    assert its[-1] <= 2 * its[0] + 4


# --------------------------------------------------------------------------- stalled coarsening

def star_graph(k, hub=None):
    """Hub 0 joined to spokes 1..k (a_0i = -1), diagonally dominant."""
    n = k + 1
    M = sp.lil_matrix((n, n))
    M[0, 0] = float(k + 1) if hub is None else hub
    for i in range(1, n):
        M[0, i] = M[i, 0] = -1.0
        M[i, i] = 2.0
    return csr_from_scipy(M.tocsr())


def pairs_and_isolated(n_pairs, n_iso):
    """n_pairs disjoint edges plus n_iso isolated vertices."""
    n = 2 * n_pairs + n_iso
    M = sp.lil_matrix((n, n))
    for q in range(n_pairs):
        i, j = 2 * q, 2 * q + 1
        M[i, i] = M[j, j] = 2.0
        M[i, j] = M[j, i] = -1.0
    for i in range(2 * n_pairs, n):
        M[i, i] = 1.0
    return csr_from_scipy(M.tocsr())


def test_star_graph_stops_instead_of_shedding_one_pair_per_level():
    # every edge meets the hub: each matching has exactly one pair, so without
    # the stop rule level l has 300 - l rows until max_levels
    A = star_graph(299)
    off = oracle.Hierarchy(A, min_ratio=0.0)
    assert off.nlevels == 50
    assert [off.n(l) for l in range(50)] == [300 - l for l in range(50)]
    assert all(off.pairs(l) == 1 for l in range(49))
    on = oracle.Hierarchy(A)
    assert on.nlevels == 1 and on.n(0) == 300


def test_stop_rule_threshold_is_strict():
    # 100 pairs of 300 rows: 300 == 1.5 * 200, coarsening goes on (to 200 <= max_coarse)
    H = oracle.Hierarchy(pairs_and_isolated(100, 100))
    assert H.nlevels == 2 and H.n(1) == 200 and H.pairs(0) == 100
    # 99 pairs: 300 < 1.5 * 201, level 0 is the coarsest
    H = oracle.Hierarchy(pairs_and_isolated(99, 102))
    assert H.nlevels == 1
    # above the dense limit the rule does not apply: level 1 (201 rows, no
    # edges left) is the coarsest by the no-pair rule
    H = oracle.Hierarchy(pairs_and_isolated(99, 102), max_dense=250)
    assert H.nlevels == 2 and H.n(1) == 201


def test_stop_rule_on_lognormal_coefficients():
    # lognormal cell coefficients leave weakly coupled vertices unmatched on
    # every level; the hierarchy stops where a matching would shrink a level
    # by less than 1.5, and every earlier level shrank by at least that
    A = varcoef7(36, seed=5000)
    on = oracle.Hierarchy(A)
    off = oracle.Hierarchy(A, min_ratio=0.0)
    L = on.nlevels - 1
    assert off.nlevels > on.nlevels
    for l in range(on.nlevels):
        assert on.n(l) == off.n(l)
    for l in range(L):
        assert on.n(l) >= 1.5 * on.n(l + 1)
    assert on.n(L) > 200 and on.n(L) < 1.5 * off.n(L + 1)


# --------------------------------------------------------------------------- aggregate-size composition

@pytest.mark.parametrize("steps", [2, 3])
@pytest.mark.parametrize("case", ["lap7_16", "varcoef_14", "q1_8"])
def test_composed_prolongator_is_product_of_pairwise(case, steps):
    # Sec. 3.1: aggregates larger than pairs come from multiplying successive
    # pairwise prolongators.  The composed hierarchy keeps every steps-th
    # pairwise level; its prolongator equals the (scipy) product of the
    # pairwise ones in between, bitwise, and its coarse matrices are the
    # pairwise Galerkin matrices
    A = {"lap7_16": lambda: lap7(16), "varcoef_14": lambda: varcoef7(14, seed=4),
         "q1_8": lambda: q1_stretched(8, 1.05)}[case]()
    P1 = oracle.Hierarchy(A)
    C = oracle.Hierarchy(A, agg_steps=steps)
    L1 = P1.nlevels - 1
    kept = list(range(0, L1, steps)) + [L1]
    assert C.nlevels == len(kept)
    for j, a in enumerate(kept):
        rp, ci, v = C.level(j)
        orp, oci, ov = P1.level(a)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci) and np.array_equal(v.view(np.uint64), ov.view(np.uint64))
        if j + 1 == len(kept):
            break
        b = kept[j + 1]
        prod = prolongator(P1, a)
        for m in range(a + 1, b):
            prod = (prod @ prolongator(P1, m)).tocsr()
        prod.sort_indices()
        Pc = prolongator(C, j).tocsr()
        Pc.sort_indices()
        assert prod.shape == Pc.shape and np.array_equal(prod.indices, Pc.indices)
        assert np.array_equal(prod.data.view(np.uint64), Pc.data.view(np.uint64))
        # Galerkin identity across the composed step (sums in another order)
        Ac = (Pc.T @ C.level_scipy(j) @ Pc).toarray()
        An = C.level_scipy(j + 1).toarray()
        assert np.abs(Ac - An).max() <= 1e-12 * np.abs(An).max()
        # aggregates of at most 2**(b - a) members
        sizes = np.bincount(C.agg(j), minlength=C.n(j + 1))
        assert sizes.min() >= 1 and sizes.max() <= 2 ** (b - a)


def test_composed_hierarchy_solves():
    A = varcoef7(16, seed=3)
    b = uniform_rhs(A.n, 2)
    for steps in (1, 2, 3):
        H = oracle.Hierarchy(A, agg_steps=steps)
        x, it, rr, st = H.solve(b, 1e-8)
        assert st == 0
        r = b - A.to_scipy() @ x
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)


# --------------------------------------------------------------------------- smoothed prolongator

@pytest.mark.parametrize("case", ["varcoef_9", "q1_8", "lap7_10", "q1_12_composed3", "varcoef_12_composed2"])
def test_smoothed_prolongator_definition(case):
    # Sec. 3.1: P = (I - omega D^-1 A) P^, D = diag(A), omega = 1/||D^-1 A||_inf,
    # against dense numpy on every level; the coarse matrix is P^T A P and is
    # stored bitwise symmetric; P keeps w in range: P w_c = w - omega D^-1 A w
    A = {"varcoef_9": lambda: varcoef7(9, seed=30), "q1_8": lambda: q1_stretched(8, 1.05),
         "lap7_10": lambda: lap7(10), "q1_12_composed3": lambda: q1_stretched(12, 1.05),
         "varcoef_12_composed2": lambda: varcoef7(12, seed=32)}[case]()
    steps = 3 if case.endswith("composed3") else (2 if case.endswith("composed2") else 1)
    H = oracle.Hierarchy(A, smooth_prolongator=True, agg_steps=steps, max_coarse=40)
    assert H.nlevels >= 3
    if steps > 1:
        # the first kept level's composed aggregates come from the pairwise
        # chain of A_0, exactly as without smoothing
        T = oracle.Hierarchy(A, agg_steps=steps, max_coarse=40)
        assert np.array_equal(H.agg(0), T.agg(0)) and np.array_equal(H.p(0).view(np.uint64), T.p(0).view(np.uint64))
        for l in range(H.nlevels - 1):
            sizes = np.bincount(H.agg(l), minlength=H.n(l + 1))
            assert sizes.min() >= 1 and sizes.max() <= 2 ** steps
    for l in range(H.nlevels - 1):
        Al = H.level_scipy(l).toarray()
        d = np.diag(Al)
        om = 1.0 / np.max(np.abs(Al).sum(axis=1) / d)
        assert abs(H.prolongator_omega(l) - om) <= 4 * ULP * om
        Ph = sp.csr_matrix((H.p(l), (np.arange(H.n(l)), H.agg(l))), shape=(H.n(l), H.n(l + 1))).toarray()
        Pd = (np.eye(H.n(l)) - om * (Al / d[:, None])) @ Ph
        P = H.prolongator(l).toarray()
        assert np.abs(P - Pd).max() <= 1e-14 * np.abs(Pd).max(), l
        # pattern: exactly the aggregates of each row's neighbours
        Ps = H.prolongator(l)
        for i in range(0, H.n(l), max(1, H.n(l) // 50)):
            nb = sorted(set(H.agg(l)[H.level_scipy(l).indices[H.level_scipy(l).indptr[i]:H.level_scipy(l).indptr[i + 1]]]))
            assert list(Ps.indices[Ps.indptr[i]:Ps.indptr[i + 1]]) == nb
        w, wc = H.w(l), H.w(l + 1)
        assert np.allclose(P @ wc, w - om * (Al @ w) / d, rtol=1e-13, atol=1e-13 * np.abs(w).max())
        Ac = H.level_scipy(l + 1).toarray()
        assert np.abs(Ac - P.T @ Al @ P).max() <= 1e-12 * np.abs(Ac).max(), l
        assert np.array_equal(Ac.view(np.uint64), Ac.T.view(np.uint64))


def test_smoothed_vcycle_matches_multiplicative_composition():
    A = varcoef7(6, seed=31)
    H = oracle.Hierarchy(A, max_coarse=12, smooth_prolongator=True)
    assert H.nlevels >= 3

    def dense_B(l):
        Al = H.level_scipy(l).toarray()
        if l == H.nlevels - 1:
            return np.linalg.inv(Al)
        n = Al.shape[0]
        P = H.prolongator(l).toarray()
        S = np.eye(n) - np.diag(H.dinv(l)) @ Al
        C = np.eye(n) - P @ dense_B(l + 1) @ P.T @ Al
        return (np.eye(n) - S @ C @ S) @ np.linalg.inv(Al)

    n = H.n(0)
    Bcols = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    Bf = dense_B(0)
    assert np.allclose(Bcols, Bf, rtol=1e-10, atol=1e-10 * abs(Bf).max())
    assert np.allclose(Bcols, Bcols.T, rtol=1e-11, atol=1e-11 * abs(Bcols).max())


def test_smoothed_prolongator_solves_and_options():
    A = q1_stretched(10, 1.05)
    b = q1_rhs(10, 1.05, 2)
    its = {}
    for smooth in (False, True):
        H = oracle.Hierarchy(A, smooth_prolongator=smooth)
        x, it, rr, st = H.solve(b, 1e-8)
        assert st == 0 and np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
        its[smooth] = it
    assert its[True] <= its[False]
    # with aggregates of up to 8 (the paper's configuration) smoothing still
    # pays, at a fraction of the pairwise fill-in
    S3, T3 = oracle.Hierarchy(A, smooth_prolongator=True, agg_steps=3), oracle.Hierarchy(A, agg_steps=3)
    assert S3.solve(b, 1e-8)[1] < T3.solve(b, 1e-8)[1]
    assert sum(S3.nnz(l) for l in range(S3.nlevels)) < 3 * A.nnz
    with pytest.raises(oracle.OracleError):                 # P depends on A: no reuse
        oracle.Hierarchy(A, smooth_prolongator=True).update(A.val)


# --------------------------------------------------------------------------- hybrid Gauss-Seidel smoother

def _nested_order_py(H, l):
    """Nested-aggregate order written out: the coarsest level in its own
    order, then per finer level the members of each coarse unknown (coarse
    unknowns in their nested order), members ascending."""
    L = H.nlevels - 1
    order = list(range(H.n(L)))
    for m in range(L - 1, l - 1, -1):
        agg = H.agg(m)
        members = {}
        for i in range(H.n(m)):
            members.setdefault(int(agg[i]), []).append(i)
        order = [i for I in order for i in members[I]]
    return np.array(order)


def _hgs_M(H, l, nb, omega, backward=False):
    """M = blockdiag(omega (L_pp + D_pp)) (its transpose for backward) in the
    level's own numbering, blocks of nb consecutive nested positions."""
    A = H.level_scipy(l).toarray()
    o = _nested_order_py(H, l)
    Ap = A[np.ix_(o, o)]
    n = A.shape[0]
    Mp = np.zeros_like(Ap)
    for b0 in range(0, n, nb):
        b1 = min(b0 + nb, n)
        blk = Ap[b0:b1, b0:b1]
        Mp[b0:b1, b0:b1] = omega * (np.triu(blk) if backward else np.tril(blk))
    M = np.zeros_like(A)
    M[np.ix_(o, o)] = Mp
    return M


@pytest.mark.parametrize("case", ["varcoef_10", "q1_6_composed2"])
def test_nested_order_definition(case):
    A = varcoef7(10, seed=2) if case == "varcoef_10" else q1_stretched(6, 1.05)
    H = oracle.Hierarchy(A, agg_steps=2 if "composed" in case else 1)
    for l in range(H.nlevels):
        o = H.nested_order(l)
        assert np.array_equal(o, _nested_order_py(H, l)), l
        assert np.array_equal(np.sort(o), np.arange(H.n(l)))


@pytest.mark.parametrize("nb,omega,nu", [(1, 0.8, 2), (10 ** 6, 1.0, 1), (37, 0.9, 1), (64, 1.0, 3)])
def test_hgs_sweeps_are_block_triangular_solves(nb, omega, nu):
    # Sec. 3.1: M = blockdiag(omega (L_pp + D_pp)) over the row blocks; one
    # unknown per block is damped Jacobi with the true diagonal, one block is
    # plain (damped) Gauss-Seidel.  nu forward sweeps from zero, then nu
    # backward sweeps (M^T) from the result, against dense solves with M.
    A = varcoef7(9, seed=3)
    H = oracle.Hierarchy(A).set_smoother("hgs", nu=nu, nb=nb, omega=omega)
    for l in range(H.nlevels - 1):
        Al = H.level_scipy(l).toarray()
        r = uniform_rhs(H.n(l), 10 + l)
        Mf, Mb = _hgs_M(H, l, nb, omega), _hgs_M(H, l, nb, omega, backward=True)
        x = np.zeros(H.n(l))
        for _ in range(nu):
            x = x + np.linalg.solve(Mf, r - Al @ x)
        xo = H.hgs_smooth(l, r)
        assert np.allclose(xo, x, rtol=1e-11, atol=1e-11 * abs(x).max()), l
        y = x.copy()
        for _ in range(nu):
            y = y + np.linalg.solve(Mb, r - Al @ y)
        yo = H.hgs_smooth(l, r, x=xo, backward=True)
        assert np.allclose(yo, y, rtol=1e-10, atol=1e-10 * abs(y).max()), l
    if nb == 1:
        # damped Jacobi: one sweep from zero is r / (omega a_ii)
        d = A.to_scipy().diagonal()
        r = uniform_rhs(A.n, 3)
        H1 = oracle.Hierarchy(A).set_smoother("hgs", nu=1, nb=1, omega=omega)
        assert np.allclose(H1.hgs_smooth(0, r), r / (omega * d), rtol=1e-15, atol=0)


def _dense_B_hgs(H, l, nu, nb, omega):
    """B_l of eq. (multiplicative_composition) with nu forward sweeps of M
    before and nu backward sweeps of M^T after the coarse correction."""
    A = H.level_scipy(l).toarray()
    if l == H.nlevels - 1:
        return np.linalg.inv(A)
    n = A.shape[0]
    P = prolongator(H, l).toarray()
    Mf, Mb = _hgs_M(H, l, nb, omega), _hgs_M(H, l, nb, omega, backward=True)
    Sf = np.linalg.matrix_power(np.eye(n) - np.linalg.solve(Mf, A), nu)
    Sb = np.linalg.matrix_power(np.eye(n) - np.linalg.solve(Mb, A), nu)
    C = np.eye(n) - P @ _dense_B_hgs(H, l + 1, nu, nb, omega) @ P.T @ A
    return (np.eye(n) - Sb @ C @ Sf) @ np.linalg.inv(A)


@pytest.mark.parametrize("case", ["varcoef_6", "q1_4_composed2"])
def test_hgs_vcycle_matches_multiplicative_composition(case):
    A = varcoef7(6, seed=8) if case == "varcoef_6" else q1_stretched(4, 1.05)
    H = oracle.Hierarchy(A, max_coarse=12, agg_steps=2 if "composed" in case else 1)
    H.set_smoother("hgs", nu=2, nb=23, omega=1.0)
    assert H.nlevels >= 3
    n = H.n(0)
    Bcols = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    Bf = _dense_B_hgs(H, 0, 2, 23, 1.0)
    assert np.allclose(Bcols, Bf, rtol=1e-9, atol=1e-9 * abs(Bf).max())
    # forward before, backward after: a symmetric positive definite preconditioner
    assert np.allclose(Bcols, Bcols.T, rtol=1e-10, atol=1e-10 * abs(Bcols).max())
    assert np.linalg.eigvalsh(0.5 * (Bcols + Bcols.T)).min() > 0


def test_hgs_smooths_better_than_l1_jacobi():
    # the paper's reason for Gauss-Seidel: fewer outer iterations
    A = q1_stretched(10, 1.05)
    b = q1_rhs(10, 1.05, 2)
    its = {}
    for kind in ("l1", "hgs"):
        H = oracle.Hierarchy(A).set_smoother(kind, nu=4, nb=256)
        x, it, rr, st = H.solve(b, 1e-8)
        assert st == 0 and np.linalg.norm(b - A.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)
        its[kind] = it
    assert its["hgs"] < its["l1"]


def test_hgs_parameters_validated():
    H = oracle.Hierarchy(lap7(4))
    for bad in [dict(nu=0), dict(nb=0), dict(omega=0.0), dict(omega=float("nan"))]:
        kw = dict(nu=4, nb=8, omega=1.0)
        kw.update(bad)
        with pytest.raises(oracle.OracleError):
            H.set_smoother("hgs", **kw)


# --------------------------------------------------------------------------- coefficient-only reuse

def _same_level(G, H, l):
    for x, y in zip(G.level(l), H.level(l)):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8)), l
    assert np.array_equal(G.dinv(l).view(np.uint64), H.dinv(l).view(np.uint64)), l


@pytest.mark.parametrize("steps", [1, 2])
def test_update_with_power_of_two_scaling_equals_fresh_setup(steps):
    # Sec. 4 reuse: the prolongators are kept and the coarse matrices and
    # smoothers rebuilt.  Scaling A by 4 leaves every edge weight of
    # eq. (weights) bitwise unchanged (numerator and denominator scale
    # exactly), so a fresh setup of 4A matches exactly as A did, and reuse
    # must then give that fresh hierarchy bit for bit: every level, its l1
    # diagonal and the coarsest Cholesky factor.
    A = varcoef7(12, seed=5)
    H = oracle.Hierarchy(A, agg_steps=steps)
    F = oracle.Hierarchy(CSR(A.n, A.row_ptr, A.col, 4.0 * A.val), agg_steps=steps)
    U = H.update(4.0 * A.val)
    assert U.nlevels == F.nlevels == H.nlevels
    for l in range(U.nlevels):
        _same_level(U, F, l)
        if l + 1 < U.nlevels:
            assert np.array_equal(U.agg(l), H.agg(l)) and np.array_equal(U.p(l), H.p(l))
    assert np.array_equal(U.chol().view(np.uint64), F.chol().view(np.uint64))
    # and the same values give back the original hierarchy
    S = U.update(A.val)
    for l in range(S.nlevels):
        _same_level(S, H, l)
    assert np.array_equal(S.chol().view(np.uint64), H.chol().view(np.uint64))


@pytest.mark.parametrize("steps", [1, 3])
def test_update_recomputes_galerkin_and_smoother_from_new_values(steps):
    # new lognormal coefficients on the same pattern: every coarse matrix is
    # P^T A P of the new finer matrix with the ORIGINAL prolongators (scipy
    # products, another summation order), the l1 diagonal is that of the new
    # matrices, and the factor reproduces the new coarsest matrix
    A, B = varcoef7(14, seed=6), varcoef7(14, seed=7)
    assert np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col, B.col)
    H = oracle.Hierarchy(A, agg_steps=steps)
    U = H.update(B.val)
    M = B.to_scipy()
    for l in range(U.nlevels):
        An = U.level_scipy(l)
        assert np.abs((An - M).toarray()).max() <= 1e-12 * np.abs(M).max(), l
        rs = np.asarray(abs(An).sum(axis=1)).ravel()
        assert np.allclose(U.dinv(l), 1.0 / rs, rtol=4 * ULP * 27, atol=0)
        if l + 1 == U.nlevels:
            break
        P = prolongator(H, l)
        assert np.array_equal(U.agg(l), H.agg(l))
        M = (P.T @ An @ P).tocsr()
    Lc = U.chol()
    AL = U.level_scipy(U.nlevels - 1).toarray()
    assert np.abs(Lc @ Lc.T - AL).max() <= 1e-12 * np.abs(AL).max()
    # the old hierarchy's matrices are not the new ones (the update did work)
    assert np.abs(U.level_scipy(1) - H.level_scipy(1)).max() > 1e-3 * np.abs(H.level_scipy(1)).max()
    # and the rebuilt hierarchy preconditions the new matrix
    b = uniform_rhs(B.n, 3)
    x, it, rr, st = U.solve(b, 1e-8)
    assert st == 0 and np.linalg.norm(b - B.to_scipy() @ x) <= 1.01e-8 * np.linalg.norm(b)


def test_update_rejects_bad_values():
    A = varcoef7(6, seed=1)
    H = oracle.Hierarchy(A)
    bad = A.val.copy()
    bad[A.row_ptr[3]:A.row_ptr[4]] *= -1.0          # row 3: negative diagonal
    with pytest.raises(oracle.OracleError) as e:
        H.update(bad)
    assert e.value.code == oracle.E_INVALID
    with pytest.raises(ValueError):
        H.update(A.val[:-1])


# --------------------------------------------------------------------------- failures

def test_invalid_inputs_rejected():
    A = lap7(3)
    bad = CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[5] = A.n + 3
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(bad)
    assert e.value.code == oracle.E_INVALID
    neg = CSR(A.n, A.row_ptr.copy(), A.col.copy(), -A.val.copy())
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(neg)
    assert e.value.code == oracle.E_INVALID


def test_indefinite_matrix_reports_not_spd():
    M = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 1.0]]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(csr_from_scipy(M))
    assert e.value.code == oracle.E_NOT_SPD


# --------------------------------------------------------------------------- FP32 hierarchy (ext. a)

@pytest.mark.parametrize("case", ["q1_6", "varcoef_8", "lap7_8_composed", "q1_6_smoothed"])
def test_round_f32_is_binary32_rounding_of_the_fp64_hierarchy(case):
    """The FP32 hierarchy is the FP64 setup with A_l, the l1 inverse diagonal,
    the prolongator weights and the coarsest Cholesky factor rounded to
    binary32 (numpy's float32 cast is the reference rounding); aggregates and
    the near-null vector w stay as built.  Its V-cycle is the multiplicative
    composition (Sec. 3.1) of those rounded operators with the coarsest solve
    through the rounded factor, B_L = (L32 L32^T)^-1."""
    kw = {"lap7_8_composed": dict(agg_steps=2), "q1_6_smoothed": dict(smooth_prolongator=True, agg_steps=2)}
    A = {"q1_6": lambda: q1_stretched(6, 1.05), "varcoef_8": lambda: varcoef7(8, seed=8),
         "lap7_8_composed": lambda: lap7(8), "q1_6_smoothed": lambda: q1_stretched(6, 1.05)}[case]()
    H = oracle.Hierarchy(A, max_coarse=12, **kw.get(case, {}))
    G = H.round_f32()
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    assert G.nlevels == H.nlevels >= 3
    rounded_any = False
    for l in range(H.nlevels):
        rp, ci, v = H.level(l)
        rq, cq, u = G.level(l)
        assert np.array_equal(rp, rq) and np.array_equal(ci, cq)
        assert np.array_equal(u, f32(v))
        assert np.array_equal(G.dinv(l), f32(H.dinv(l)))
        assert np.array_equal(G.w(l), H.w(l))               # w is not rounded
        rounded_any |= not np.array_equal(u, v) or not np.array_equal(G.dinv(l), H.dinv(l))
        if l + 1 < H.nlevels:
            assert np.array_equal(G.agg(l), H.agg(l))
            assert np.array_equal(G.p(l), f32(H.p(l)))
            PH, PG = H.prolongator(l), G.prolongator(l)
            assert np.array_equal(PH.indptr, PG.indptr) and np.array_equal(PH.indices, PG.indices)
            assert np.array_equal(PG.data, f32(PH.data))
    assert rounded_any
    L64, L32 = H.chol(), G.chol()
    assert np.array_equal(L32, f32(L64))
    assert not np.array_equal(L32, L64)

    def dense_B(l):
        Al = G.level_scipy(l).toarray()
        if l == G.nlevels - 1:
            return np.linalg.inv(L32 @ L32.T)
        n = Al.shape[0]
        P = G.prolongator(l).toarray()
        S = np.eye(n) - np.diag(G.dinv(l)) @ Al
        C = np.eye(n) - P @ dense_B(l + 1) @ P.T @ Al
        return (np.eye(n) - S @ C @ S) @ np.linalg.inv(Al)

    n = G.n(0)
    Bcols = np.stack([G.vcycle(e) for e in np.eye(n)], axis=1)
    Bf = dense_B(0)
    assert np.allclose(Bcols, Bf, rtol=1e-10, atol=1e-10 * abs(Bf).max())
    # and it differs from the FP64 cycle by the binary32 rounding, not less
    B64 = np.stack([H.vcycle(e) for e in np.eye(n)], axis=1)
    d = np.abs(Bcols - B64).max() / np.abs(B64).max()
    assert 1e-10 < d < 1e-4


# --------------------------------------------------------------------------- true-residual restart

def test_true_residual_restart_is_a_warm_restart_from_b_minus_ax():
    """With the true-residual check (ext. a, the stopping test of Sec. 5 taken
    on b - A x), a solve whose recurrence residual meets tol while the true
    residual does not restarts the recurrence from r = b - A x: the result is
    the chain 'solve, then solve again warm-started from x' (each warm start
    recomputes r = b - A x0), and it ends with a true residual within tol."""
    A = lap7(10)
    H = oracle.Hierarchy(A, max_coarse=30)
    b = uniform_rhs(A.n, 9)
    S = A.to_scipy()
    nb = np.linalg.norm(b)
    tol = 5e-16                       # below the recurrence's attainable agreement with b - A x
    x1, it1, rr1, st1 = H.solve(b, tol)
    assert st1 == 0 and rr1 <= tol
    assert np.linalg.norm(b - S @ x1) > tol * nb          # the branch is taken
    x2, it2, rr2, st2 = H.solve(b, tol, true_res=True)
    assert st2 == 0 and it2 > it1
    # the warm-started chain, restarts bounded as in the oracle (10)
    x, total = x1, it1
    for _ in range(10):
        if np.linalg.norm(b - S @ x) <= tol * nb:
            break
        x, itw, _, stw = H.solve(b, tol, maxit=1000 - total, x0=x)
        assert stw == 0
        total += itw
    assert total == it2
    assert np.array_equal(x, x2)
    assert np.linalg.norm(b - S @ x2) <= tol * nb
    # without the request the branch is never taken
    x3, it3, _, _ = H.solve(b, tol, true_res=False)
    assert it3 == it1 and np.array_equal(x3, x1)


def _rounds_matching(A, w):
    """Locally dominant rounds, as the device setup runs them: every vertex's
    eligible neighbours sorted heaviest first (equal weights: smaller index
    first, which for a fixed vertex is the (lo, hi) order); each round an
    unmatched vertex with neighbours left points at its first unmatched one
    (a cursor that only moves forward), mutual pointers are matched, a vertex
    with none left stays single.  Returns mate[] and the number of rounds."""
    n = A.shape[0]
    D = A.diagonal()
    Au = sp.triu(A, 1).tocsr()
    nbrs = [[] for _ in range(n)]
    for i in range(n):
        for k in range(Au.indptr[i], Au.indptr[i + 1]):
            j = int(Au.indices[k])
            c = _weights_eq(Au.data[k], D[i], D[j], w[i], w[j])   # the edge's upper entry, both directions
            if c > 1.0:
                nbrs[i].append((-c, j))
                nbrs[j].append((-c, i))
    for L in nbrs:
        L.sort()
    mate = [-1] * n
    state = [0] * n                 # 0 alive, 1 matched, 2 single
    cur = [0] * n
    rounds = 0
    while any(s == 0 for s in state):
        rounds += 1
        cand = [-1] * n
        for i in range(n):
            if state[i] != 0:
                continue
            while cur[i] < len(nbrs[i]) and mate[nbrs[i][cur[i]][1]] >= 0:
                cur[i] += 1
            if cur[i] < len(nbrs[i]):
                cand[i] = nbrs[i][cur[i]][1]
            else:
                state[i] = 2
        progress = False
        for i in range(n):
            if state[i] == 0 and cand[cand[i]] == i:
                mate[i], state[i], progress = cand[i], 1, True
        assert progress or not any(s == 0 for s in state), "a round with alive vertices matched nothing"
    return np.array(mate), rounds


def _pairs_of(agg):
    order = np.argsort(agg, kind="stable")
    sa = agg[order]
    starts = np.flatnonzero(np.r_[True, sa[1:] != sa[:-1]])
    sizes = np.diff(np.r_[starts, len(sa)])
    return {(int(order[s]), int(order[s + 1])) for s, z in zip(starts, sizes) if z == 2}


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("discrete", [False, True])
def test_locally_dominant_rounds_give_the_greedy_matching(seed, discrete):
    # the device setup's matching (parallel rounds) against the oracle's greedy
    # matching, with many exact weight ties in the discrete case
    A = _random_spd(80, 0.1, 100 + seed, discrete=discrete)
    H = oracle.Hierarchy(csr_from_scipy(A), max_coarse=1, max_levels=2)
    mate, rounds = _rounds_matching(A, np.ones(A.shape[0]))
    got = {(i, int(m)) for i, m in enumerate(mate) if m > i}
    assert got == _pairs_of(H.agg(0))
    assert rounds >= 2


@pytest.mark.parametrize("case", ["varcoef_10", "q1_6"])
def test_locally_dominant_rounds_on_every_level(case):
    # coarse levels (non-uniform w): the rounds give the oracle's pairs on each
    A = {"varcoef_10": lambda: varcoef7(10, seed=8), "q1_6": lambda: q1_stretched(6, 1.05)}[case]()
    H = oracle.Hierarchy(A, max_coarse=10)
    for l in range(H.nlevels - 1):
        mate, _ = _rounds_matching(H.level_scipy(l), H.w(l))
        got = {(i, int(m)) for i, m in enumerate(mate) if m > i}
        assert got == _pairs_of(H.agg(l)), f"level {l}"
