"""Multi-right-hand-side solves (16 columns per pass) through the C ABI.

* every column against the oracle: fixed-K iterates within 1e-8, to-tolerance
  runs within +-1 iteration with a true residual <= tol;
* a column's result is independent of the other columns (bitwise): the same
  right-hand side alone, in a full batch, and at another column position;
* FP32 V-cycle under the FP64 recurrences: true residual <= tol for every
  column, error against the FP64 oracle reported and bounded;
* the coarsest level of the batched cycle runs on the matrix cores
  (FP64 MFMA); the fixed-K parity checks it through the whole cycle.
"""
import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import SplitMix64, lap7, q1_rhs_sequence, q1_stretched, varcoef7

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "lap7_24": (lambda: lap7(24), None),
    "q1_20": (lambda: q1_stretched(20, 1.05), 20),
    "varcoef_22": (lambda: varcoef7(22, seed=6), None),
    "single_level_lap7_5": (lambda: lap7(5), None),
    "stalled_varcoef_48": (lambda: varcoef7(48, seed=5000), None),
    "varcoef_22_composed2": (lambda: varcoef7(22, seed=6), None),
}
KW = {"single_level_lap7_5": {"max_coarse": 1000}, "varcoef_22_composed2": {"agg_steps": 2}}


@pytest.fixture(scope="module")
def built():
    assert torch.cuda.is_available()
    cache = {}

    def get(case):
        if case not in cache:
            make, N = CASES[case]
            A = make()
            kw = KW.get(case, {})
            O = oracle.Hierarchy(A, **kw)
            H = pamg.Hierarchy(A, build_f32=1, **kw)
            if N is not None:
                Bm = q1_rhs_sequence(N, 1.05, 4, 16).T.copy()          # (16, n)
            else:
                Bm = np.stack([SplitMix64(100 + j).uniform(A.n) for j in range(16)])
            cache[case] = (A, O, H, Bm)
        return cache[case]
    return get


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec", [pamg.PREC_F64, pamg.PREC_F32])
def test_batched_coarse_and_vcycle_operators(built, case, prec):
    # each column of the batched coarse solve (FP64: matrix cores) and of the
    # batched V-cycle against the oracle's operators
    A, O0, H, Bm = built(case)
    O = O0 if prec == pamg.PREC_F64 else O0.round_f32()
    L = O.nlevels - 1
    nL = O.n(L)
    R = np.stack([SplitMix64(300 + j).uniform(nL) for j in range(16)])
    out = torch.empty((16, nL), dtype=torch.float64, device="cuda:0")
    H.debug_apply_batch(pamg.OP_COARSE, dev(R), out, precision=prec)
    Z = out.cpu().numpy()
    cond = np.linalg.cond(O.level_scipy(L).toarray())
    ctol = max(1e-13, 16 * cond * np.finfo(np.float64).eps) if prec == pamg.PREC_F64 else max(2e-6, 16 * cond * 6e-8)
    errs = [np.linalg.norm(Z[j] - O.coarse_solve(R[j])) / np.linalg.norm(O.coarse_solve(R[j])) for j in range(16)]
    assert max(errs) <= ctol, f"batched coarse solve errors {['%.1e' % e for e in errs]}"
    n0 = O.n(0)
    out0 = torch.empty((16, n0), dtype=torch.float64, device="cuda:0")
    H.debug_apply_batch(pamg.OP_VCYCLE, dev(Bm), out0, precision=prec)
    Z0 = out0.cpu().numpy()
    vtol = max(1e-12, 16 * cond * np.finfo(np.float64).eps) if prec == pamg.PREC_F64 else 1e-5
    errs = [np.linalg.norm(Z0[j] - O.vcycle(Bm[j])) / np.linalg.norm(O.vcycle(Bm[j])) for j in range(16)]
    assert max(errs) <= vtol, f"batched V-cycle errors {['%.1e' % e for e in errs]}"


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("krylov", ["fcg", "cg"])
def test_batch_fixed_iterations_match_oracle(built, case, krylov):
    A, O, H, Bm = built(case)
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(dev(Bm), X, tol=0.0, fixed_iters=6, krylov=krylov)
    Xh = X.cpu().numpy()
    for j in range(16):
        x_or, it, _, _ = O.solve(Bm[j], 0.0, krylov=krylov, fixed_iters=6)
        assert infos[j].iterations == 6
        err = np.linalg.norm(Xh[j] - x_or) / np.linalg.norm(x_or)
        assert err <= 1e-8, f"column {j}: {err:.3e}"


@pytest.mark.parametrize("case", sorted(CASES))
def test_batch_to_tolerance_match_oracle(built, case):
    A, O, H, Bm = built(case)
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(dev(Bm), X, tol=1e-6)
    Xh = X.cpu().numpy()
    S = A.to_scipy()
    for j in range(16):
        x_or, it_or, _, st = O.solve(Bm[j], 1e-6)
        assert infos[j].status == pamg.OK
        assert abs(infos[j].iterations - it_or) <= 1, (j, infos[j].iterations, it_or)
        assert np.linalg.norm(Bm[j] - S @ Xh[j]) <= 1e-6 * np.linalg.norm(Bm[j])
        if infos[j].iterations == it_or:
            assert np.linalg.norm(Xh[j] - x_or) <= 1e-8 * np.linalg.norm(x_or)


@pytest.mark.parametrize("prec", [pamg.PREC_F64, pamg.PREC_F32])
def test_column_result_independent_of_batch(built, prec):
    A, O, H, Bm = built("varcoef_22")
    full = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    inf_full = H.solve_batch(dev(Bm), full, tol=1e-8, precision=prec)
    j = 5
    alone = torch.zeros((1, A.n), dtype=torch.float64, device="cuda:0")
    inf_alone = H.solve_batch(dev(Bm[j:j + 1]), alone, tol=1e-8, precision=prec)
    assert inf_alone[0].iterations == inf_full[j].iterations
    assert torch.equal(alone[0], full[j]), "column differs when solved alone"
    # the same right-hand side at another position, among different companions
    other = np.stack([Bm[j]] + [SplitMix64(900 + k).uniform(A.n) for k in range(6)])
    mix = torch.zeros(other.shape, dtype=torch.float64, device="cuda:0")
    inf_mix = H.solve_batch(dev(other), mix, tol=1e-8, precision=prec)
    assert inf_mix[0].iterations == inf_full[j].iterations
    assert torch.equal(mix[0], full[j]), "column differs in another batch position"


def test_graph_and_eager_batches_agree_bitwise(built):
    A, O, H, Bm = built("q1_20")
    xs = []
    for use_graph, every in [(1, 4), (0, 4), (1, 6)]:
        X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
        infos = H.solve_batch(dev(Bm), X, tol=1e-8, use_graph=use_graph, check_every=every)
        xs.append((X.cpu().numpy(), [i.iterations for i in infos]))
    for X, its in xs[1:]:
        assert its == xs[0][1]
        assert np.array_equal(X.view(np.uint64), xs[0][0].view(np.uint64))


@pytest.mark.parametrize("case", ["q1_20", "varcoef_22"])
def test_batch_mixed_precision(built, case):
    A, O, H, Bm = built(case)
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(dev(Bm), X, tol=1e-6, precision=pamg.PREC_F32)
    Xh = X.cpu().numpy()
    S = A.to_scipy()
    for j in range(16):
        assert infos[j].status == pamg.OK
        rel = np.linalg.norm(Bm[j] - S @ Xh[j]) / np.linalg.norm(Bm[j])
        assert rel <= 1e-6 and abs(rel - infos[j].relres_true) <= 1e-9
        x_or, it_or, _, _ = O.solve(Bm[j], 1e-6)
        assert np.linalg.norm(Xh[j] - x_or) <= 1e-4 * np.linalg.norm(x_or)


def test_partial_batch_zero_column_and_maxit(built):
    A, O, H, Bm = built("lap7_24")
    B3 = Bm[:3].copy()
    B3[1] = 0.0
    X = torch.ones(B3.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(dev(B3), X, tol=1e-6)
    Xh = X.cpu().numpy()
    assert infos[1].iterations == 0 and infos[1].status == pamg.OK and not Xh[1].any()
    for j in (0, 2):
        x_or, it_or, _, _ = O.solve(B3[j], 1e-6)
        assert abs(infos[j].iterations - it_or) <= 1
    X2 = torch.zeros(B3.shape, dtype=torch.float64, device="cuda:0")
    infos2 = H.solve_batch(dev(B3), X2, tol=1e-14, maxit=3)
    assert infos2[0].status == pamg.NOT_CONVERGED and infos2[0].iterations == 3


def test_batch_argument_errors(built):
    A, O, H, Bm = built("lap7_24")
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pamg.PamgError):
        H.solve_batch(dev(Bm), X, use_x0=1)
    too_many = torch.zeros((17, A.n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(pamg.PamgError):
        H.solve_batch(too_many, too_many.clone())


def test_batch_autotuner_choices(built):
    A, O, H, Bm = built("q1_20")
    cfg = H.batch_config(pamg.PREC_F64)
    assert len(cfg) == H.levels - 1
    for du, dc, uu, uc in cfg:
        assert du in (1, 2, 4, 8, 16) and uu in (1, 2, 4, 8, 16) and dc in (1, 2, 4) and uc in (1, 2, 4)


@pytest.mark.parametrize("case", ["q1_20", "varcoef_22_composed2"])
@pytest.mark.parametrize("prec", [pamg.PREC_F64, pamg.PREC_F32])
def test_every_kernel_variant_gives_the_same_columns(built, case, prec):
    # the autotuner's fifteen (unroll, columns per lane) variants change only
    # scheduling: pin each one on every level in turn, and a mixed assignment,
    # and every column must come out bitwise the same
    A, O, H, Bm = built(case)
    L = H.levels - 1
    tuned = H.batch_config(prec)
    variants = [(u, c) for c in (1, 2, 4) for u in (1, 2, 4, 8, 16)]
    rng = SplitMix64(77)
    picks = rng.integers(2 * L, 0, len(variants) - 1)
    mixed = [variants[int(picks[2 * l])] + variants[int(picks[2 * l + 1])] for l in range(L)]
    configs = [[v + v] * L for v in variants] + [mixed]
    ref = None
    try:
        for cfg in configs:
            H.set_batch_config(cfg, precision=prec)
            assert H.batch_config(prec)[1:] == cfg[1:] and H.batch_config(prec)[0][:2] == cfg[0][:2]
            X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
            infos = H.solve_batch(dev(Bm), X, tol=1e-8, precision=prec)
            got = (X.cpu().numpy(), [i.iterations for i in infos])
            if ref is None:
                ref = got
                continue
            assert got[1] == ref[1], cfg
            assert np.array_equal(got[0].view(np.uint64), ref[0].view(np.uint64)), f"variant {cfg[0]} differs"
    finally:
        H.set_batch_config(tuned, precision=prec)
    assert H.batch_config(prec) == tuned


def test_batch_set_config_rejects_unknown_variants(built):
    A, O, H, Bm = built("lap7_24")
    L = H.levels - 1
    with pytest.raises(pamg.PamgError):
        H.set_batch_config([(3, 1, 4, 1)] * L)
    with pytest.raises(pamg.PamgError):
        H.set_batch_config([(4, 8, 4, 1)] * L)
