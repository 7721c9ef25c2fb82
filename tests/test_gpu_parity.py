"""GPU parity: every V-cycle operator and the full solve, through the C ABI,
against the CPU FP64 oracle on the same seeded inputs.

Tolerances (derived in the design notes):
  * SpMV-type operators (SPMV, DOWN, UP): normwise
    ||y_gpu - y_or|| <= 1e-13 * || |op| |inputs| ||  (cancellation-safe scale);
  * PROLONG: elementwise, 1e-15 relative to |D^-1 r| + |p e|;
  * COARSE: the GPU applies the explicit inverse A_L^-1, the oracle two
    triangular solves: ||z_gpu - z_or|| <= max(1e-13, 16 cond(A_L) eps) ||z_or||;
  * VCYCLE: composition of the above: ||z_gpu - z_or|| <= 1e-12 ||z_or||;
  * solves: fixed-K iterates ||x_gpu - x_or|| <= 1e-8 ||x_or||; tol runs:
    iterations within +-1 and a true relative residual <= tol;
  * FP32 hierarchy: each operator against the oracle applied to the same
    binary32-rounded hierarchy, normwise 2e-6 of the same scales.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2210_16660_amd as pamg
from workloads import CSR, SplitMix64, lap7, q1_stretched, uniform_rhs, varcoef7, q1_rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS = np.finfo(np.float64).eps


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def arrow_matrix(n3=16, w=0.01):
    """7-point Laplacian plus a row/column coupling unknown 0 to every unknown:
    row 0 holds n^3 entries, more than one tile, exercising the long-row path."""
    A = lap7(n3).to_scipy().tolil()
    N = A.shape[0]
    A = A.tocsr()
    B = sp.lil_matrix((N, N))
    B[0, 1:] = -w
    B[1:, 0] = -w
    B[0, 0] = w * (N - 1) + 1.0
    M = (A + B.tocsr()).tocsr()
    M.sort_indices()
    # bitwise symmetric by construction (same constants mirrored)
    return CSR(N, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


CASES = {
    "lap7_32": lambda: lap7(32),
    "q1_24": lambda: q1_stretched(24, 1.05),
    "varcoef_30": lambda: varcoef7(30, seed=5),
    "arrow_16": lambda: arrow_matrix(16),
    "single_level_lap7_5": lambda: lap7(5),
    # lognormal coefficients: coarsening stalls and stops at 522 rows (the
    # coarsest then runs on many workgroups)
    "stalled_varcoef_48": lambda: varcoef7(48, seed=5000),
    # one level of 2197 rows: the dense factorization over 35 tiles and the
    # multi-workgroup coarse product that writes z
    "single_level_lap7_13": lambda: lap7(13),
    # aggregate-size composition: aggregates of up to 8 unknowns (every third
    # pairwise level kept, prolongators multiplied)
    "q1_24_composed3": lambda: q1_stretched(24, 1.05),
    # the shapes of the large levels: level 0 in 4096-entry tiles with 16-bit
    # column dictionaries (ITEMS 16) and level 1 in 2048-entry dictionary
    # tiles (ITEMS 8) ...
    "q1_64_dict16": lambda: q1_stretched(64, 1.05),
    # ... level 0 in 2048-entry dictionary tiles ...
    "q1_48_dict8": lambda: q1_stretched(48, 1.05),
    # ... and 4096-entry tiles prolongated into by aggregates of up to 8 rows
    # (the fine-row-parallel up-sweep)
    "q1_64_dict16_composed3": lambda: q1_stretched(64, 1.05),
}
KW = {"single_level_lap7_5": {"max_coarse": 1000}, "single_level_lap7_13": {"max_coarse": 4000},
      "q1_24_composed3": {"agg_steps": 3}, "q1_64_dict16_composed3": {"agg_steps": 3}}
# tile capacity (entries per thread) the large-level cases must exercise at levels 0 and 1
TILE_ITEMS = {"q1_64_dict16": (16, 8), "q1_48_dict8": (8, 4), "q1_64_dict16_composed3": (16, None)}


@pytest.fixture(scope="module")
def built():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    cache = {}

    def get(case):
        if case not in cache:
            A = CASES[case]()
            kw = KW.get(case, {})
            O = oracle.Hierarchy(A, **kw)
            H = pamg.Hierarchy(A, build_f32=1, **kw)
            cache[case] = (A, O, H)
        return cache[case]
    return get


def abs_level(O, l):
    M = O.level_scipy(l)
    return abs(M)


def prolong_matrix(O, l):
    return sp.csr_matrix((O.p(l), (np.arange(O.n(l)), O.agg(l))), shape=(O.n(l), O.n(l + 1)))


def rand(n, seed):
    return SplitMix64(seed).uniform(n)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec", [pamg.PREC_F64, pamg.PREC_F32])
def test_operators_every_level(built, case, prec):
    A, O0, H = built(case)
    O = O0 if prec == pamg.PREC_F64 else O0.round_f32()
    tol = 1e-13 if prec == pamg.PREC_F64 else 2e-6
    L = O.nlevels - 1
    assert H.levels == O.nlevels
    if case in TILE_ITEMS:
        info = H.info()
        for l, items in enumerate(TILE_ITEMS[case]):
            assert items is None or info.tile_items[l] == items, (l, info.tile_items[l])
    for l in range(L + 1):
        n = O.n(l)
        x = rand(n, 100 + l)
        r = rand(n, 200 + l)
        absA = abs_level(O, l)
        dinv = O.dinv(l)
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        # SPMV
        H.debug_apply(pamg.OP_SPMV, l, dev(x), out, precision=prec)
        y = O.spmv(l, x)
        scale = np.linalg.norm(absA @ np.abs(x))
        err = np.linalg.norm(host(out) - y)
        assert err <= tol * scale, f"SPMV level {l}: {err / scale:.3e}"
        if l < L:
            nc = O.n(l + 1)
            P = prolong_matrix(O, l)
            # DOWN: P^T (r - A D^-1 r)
            outc = torch.empty(nc, dtype=torch.float64, device="cuda:0")
            H.debug_apply(pamg.OP_DOWN, l, dev(r), outc, precision=prec)
            ref = O.restrict(l, r - O.spmv(l, dinv * r))
            scale = np.linalg.norm(abs(P.T) @ (np.abs(r) + absA @ np.abs(dinv * r)))
            err = np.linalg.norm(host(outc) - ref)
            assert err <= tol * scale, f"DOWN level {l}: {err / scale:.3e}"
            # UP: zp + D^-1 (r - A zp)
            zp = x
            H.debug_apply(pamg.OP_UP, l, dev(r), out, in1=dev(zp), precision=prec)
            ref = zp + dinv * (r - O.spmv(l, zp))
            scale = np.linalg.norm(np.abs(zp) + dinv * (np.abs(r) + absA @ np.abs(zp)))
            err = np.linalg.norm(host(out) - ref)
            assert err <= tol * scale, f"UP level {l}: {err / scale:.3e}"
            # PROLONG: D^-1 r + P e
            e = rand(nc, 300 + l)
            H.debug_apply(pamg.OP_PROLONG, l, dev(r), out, in1=dev(e), precision=prec)
            ref = O.prolong_add(l, e, dinv * r)
            mag = np.abs(dinv * r) + np.abs(P) @ np.abs(e)
            ptol = 1e-15 if prec == pamg.PREC_F64 else 2e-7
            assert np.all(np.abs(host(out) - ref) <= ptol * mag + 1e-300), f"PROLONG level {l}"
    # COARSE
    nL = O.n(L)
    r = rand(nL, 400)
    out = torch.empty(nL, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_COARSE, L, dev(r), out, precision=prec)
    ref = O.coarse_solve(r)
    cond = np.linalg.cond(O.level_scipy(L).toarray())
    ctol = max(1e-13, 16 * cond * EPS) if prec == pamg.PREC_F64 else max(2e-6, 16 * cond * 6e-8)
    err = np.linalg.norm(host(out) - ref) / np.linalg.norm(ref)
    assert err <= ctol, f"COARSE: {err:.3e} (cond {cond:.3g})"
    # VCYCLE
    n0 = O.n(0)
    r = rand(n0, 500)
    out = torch.empty(n0, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_VCYCLE, 0, dev(r), out, precision=prec)
    ref = O.vcycle(r)
    err = np.linalg.norm(host(out) - ref) / np.linalg.norm(ref)
    vtol = max(1e-12, 16 * cond * EPS) if prec == pamg.PREC_F64 else 1e-5
    assert err <= vtol, f"VCYCLE: {err:.3e}"


def _rhs(case, A):
    if case.startswith("q1"):
        N = round((A.n + 1) ** (1 / 3))
        for cand in range(max(2, N - 3), N + 3):
            if (cand + 1) ** 2 * cand - 1 == A.n:
                return q1_rhs(cand, 1.05, 2)
    return uniform_rhs(A.n, 1)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("krylov", ["cg", "fcg"])
def test_solve_fixed_iterations(built, case, krylov):
    A, O, H = built(case)
    b = _rhs(case, A)
    K = 6
    x_or, it_or, _, st = O.solve(b, 0.0, krylov=krylov, fixed_iters=K)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=0.0, krylov=krylov, fixed_iters=K)
    assert info.iterations == it_or == K and info.status == pamg.OK
    err = np.linalg.norm(host(x) - x_or) / np.linalg.norm(x_or)
    assert err <= 1e-8, f"fixed-{K} solution differs by {err:.3e}"


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("krylov", ["cg", "fcg"])
def test_solve_to_tolerance(built, case, krylov):
    A, O, H = built(case)
    b = _rhs(case, A)
    x_or, it_or, rr_or, st = O.solve(b, 1e-6, krylov=krylov)
    assert st == 0
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=1e-6, krylov=krylov)
    assert info.status == pamg.OK
    assert abs(info.iterations - it_or) <= 1, (info.iterations, it_or)
    xs = host(x)
    S = A.to_scipy()
    assert np.linalg.norm(b - S @ xs) <= 1e-6 * np.linalg.norm(b)
    if info.iterations == it_or:
        assert np.linalg.norm(xs - x_or) <= 1e-8 * np.linalg.norm(x_or)


def test_graph_and_eager_paths_agree_bitwise(built):
    A, O, H = built("q1_24")
    b = dev(_rhs("q1_24", A))
    xs = []
    for use_graph, every in [(1, 4), (0, 4), (1, 2), (0, 6), (1, 8)]:
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        info = H.solve(b, x, tol=1e-8, use_graph=use_graph, check_every=every)
        xs.append((host(x), info.iterations))
    for xv, it in xs[1:]:
        assert it == xs[0][1]
        assert np.array_equal(xv.view(np.uint64), xs[0][0].view(np.uint64))


def test_repeated_solves_are_deterministic(built):
    A, O, H = built("varcoef_30")
    b = dev(uniform_rhs(A.n, 7))
    res = []
    for _ in range(3):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        info = H.solve(b, x, tol=1e-9)
        res.append(host(x))
    assert all(np.array_equal(r.view(np.uint64), res[0].view(np.uint64)) for r in res)


def test_warm_start_zero_rhs_and_maxit(built):
    A, O, H = built("lap7_32")
    b = uniform_rhs(A.n, 1)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=1e-9)
    assert info.status == pamg.OK
    # warm start from the converged solution: no iteration needed
    x2 = x.clone()
    info2 = H.solve(dev(b), x2, tol=1e-9, use_x0=1)
    assert info2.iterations == 0 and torch.equal(x2, x)
    # warm start from a partial solution matches the oracle's warm start
    xp, _, _, _ = O.solve(b, 0.0, fixed_iters=2)
    x_or, it_or, _, _ = O.solve(b, 1e-8, x0=xp)
    x3 = dev(xp)
    info3 = H.solve(dev(b), x3, tol=1e-8, use_x0=1)
    assert abs(info3.iterations - it_or) <= 1
    # zero right-hand side: x = 0 without iterating
    xz = dev(np.ones(A.n))
    infoz = H.solve(dev(np.zeros(A.n)), xz, tol=1e-6, use_x0=1)
    assert infoz.iterations == 0 and not host(xz).any()
    # maxit: NOT_CONVERGED with the last iterate
    x4 = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info4 = H.solve(dev(b), x4, tol=1e-14, maxit=3)
    assert info4.status == pamg.NOT_CONVERGED and info4.iterations == 3
    x_or3, _, _, _ = O.solve(b, 0.0, fixed_iters=3)
    assert np.linalg.norm(host(x4) - x_or3) <= 1e-8 * np.linalg.norm(x_or3)


@pytest.mark.parametrize("case", ["lap7_32", "q1_24", "varcoef_30"])
def test_mixed_precision_solve(built, case):
    A, O, H = built(case)
    b = _rhs(case, A)
    x_or, it_or, _, _ = O.solve(b, 1e-6)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=1e-6, precision=pamg.PREC_F32)
    assert info.status == pamg.OK
    xs = host(x)
    S = A.to_scipy()
    true_rel = np.linalg.norm(b - S @ xs) / np.linalg.norm(b)
    assert true_rel <= 1e-6 and abs(info.relres_true - true_rel) <= 1e-9
    assert abs(info.iterations - it_or) <= max(2, it_or // 5)
    err = np.linalg.norm(xs - x_or) / np.linalg.norm(x_or)
    assert err <= 1e-4, f"FP32-preconditioned solution vs FP64 oracle: {err:.3e}"


def test_device_factorization_reports_not_spd():
    M = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 1.0]]))
    A = CSR(3, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)
    with pytest.raises(pamg.PamgError) as e:
        pamg.Hierarchy(A)
    assert e.value.code == pamg.E_NOT_SPD


def test_dense_inverse_at_the_size_limit():
    # 8000 unknowns on one level (125 x 125 tiles): the coarse solve against a
    # sparse direct solve; cond of the 7-point Laplacian in closed form
    import scipy.sparse.linalg as spla
    n3 = 20
    A = lap7(n3)
    H = pamg.Hierarchy(A, build_f32=1, max_coarse=8192)
    assert H.levels == 1
    S = A.to_scipy().tocsc()
    th = np.pi / (n3 + 1)
    cond = (1 - np.cos(n3 * th)) / (1 - np.cos(th))
    r = rand(A.n, 77)
    ref = spla.spsolve(S, r)
    for prec, tol in ((pamg.PREC_F64, max(1e-13, 16 * cond * EPS)), (pamg.PREC_F32, max(2e-6, 16 * cond * 6e-8))):
        out = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
        H.debug_apply(pamg.OP_COARSE, 0, dev(r), out, precision=prec)
        err = np.linalg.norm(host(out) - ref) / np.linalg.norm(ref)
        assert err <= tol, f"precision {prec}: {err:.3e} (cond {cond:.3g})"
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(r), x, tol=1e-10)
    assert info.status == pamg.OK and info.iterations <= 2
    assert np.linalg.norm(host(x) - ref) <= 1e-10 * np.linalg.norm(ref) * cond
