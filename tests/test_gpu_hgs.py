"""Hybrid forward/backward Gauss-Seidel smoother (Sec. 3.1) through the C ABI,
against the oracle (R14) on the same seeded inputs.

Tolerances: a sweep sums each row as (r - A x_old) then the in-block part,
like the oracle, but over the device column order and with a multiply by
1/a_ii instead of a divide, so per row the results differ by a few units in
the last place of |A||x|; sweeps are contractions and the V-cycle composes
a fixed number of them, so normwise 1e-11 holds with margin for the smoother
and the V-cycle (a block assignment or direction error is O(1)).  Solves:
iterations within +-1, true residual <= tol, and the oracle's iterate within
1e-8 when the counts agree.
"""
import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import CSR, q1_stretched, uniform_rhs, varcoef7

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = {
    # name: (matrix, agg_steps, sweeps, block, omega, smoothed prolongators)
    "varcoef_30_nb256": (lambda: varcoef7(30, seed=21), 1, 4, 256, 1.0, False),
    "q1_24_nb64_omega12": (lambda: q1_stretched(24, 1.05), 1, 2, 64, 1.2, False),
    "varcoef_26_nb37_ragged": (lambda: varcoef7(26, seed=22), 1, 3, 37, 1.0, False),
    "q1_20_composed2_nb128": (lambda: q1_stretched(20, 1.05), 2, 4, 128, 1.0, False),
    "varcoef_18_nb1_jacobi": (lambda: varcoef7(18, seed=23), 1, 2, 1, 1.5, False),
    # the paper's preconditioner (Sec. 3.1, Table 1): smoothed prolongators
    # over aggregates of up to 8, 4 + 4 hybrid Gauss-Seidel sweeps
    "q1_24_smoothed_composed3_nu4": (lambda: q1_stretched(24, 1.05), 3, 4, 256, 1.5, True),
    "varcoef_22_smoothed_nb64": (lambda: varcoef7(22, seed=24), 1, 2, 64, 1.2, True),
}


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(case):
        if case not in cache:
            mk, steps, nu, nb, om, sm = CASES[case]
            A = mk()
            H = pamg.Hierarchy(A, agg_steps=steps, smoother="hgs", sweeps=nu, gs_block=nb, omega=om, build_f32=1,
                               smooth_prolongator=int(sm))
            O = oracle.Hierarchy(A, agg_steps=steps, smooth_prolongator=sm).set_smoother("hgs", nu=nu, nb=nb, omega=om)
            cache[case] = (A, H, O)
        return cache[case]

    return get


@pytest.mark.parametrize("case", sorted(CASES))
def test_smoother_sweeps_match_oracle(built, case):
    A, H, O = built(case)
    assert H.levels == O.nlevels
    for l in range(O.nlevels - 1):
        n = O.n(l)
        r = uniform_rhs(n, 100 + l)
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        H.debug_apply(pamg.OP_SMOOTH, l, dev(r), out)
        x = host(out)
        xo = O.hgs_smooth(l, r)
        assert np.linalg.norm(x - xo) <= 1e-11 * np.linalg.norm(xo), (l, "forward")
        # backward sweeps from the forward result
        H.debug_apply(pamg.OP_SMOOTH, l, dev(r), out, in1=dev(xo))
        y = host(out)
        yo = O.hgs_smooth(l, r, x=xo, backward=True)
        assert np.linalg.norm(y - yo) <= 1e-11 * np.linalg.norm(yo), (l, "backward")


@pytest.mark.parametrize("case", sorted(CASES))
def test_vcycle_matches_oracle(built, case):
    A, H, O = built(case)
    r = uniform_rhs(A.n, 7)
    out = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_VCYCLE, 0, dev(r), out)
    z = host(out)
    zo = O.vcycle(r)
    assert np.linalg.norm(z - zo) <= 1e-11 * np.linalg.norm(zo)


@pytest.mark.parametrize("case", ["varcoef_30_nb256", "q1_24_nb64_omega12", "q1_20_composed2_nb128",
                                  "q1_24_smoothed_composed3_nu4"])
def test_solve_matches_oracle(built, case):
    A, H, O = built(case)
    b = uniform_rhs(A.n, 9)
    x_or, it_or, _, _ = O.solve(b, 1e-8)
    for prec in (pamg.PREC_F64, pamg.PREC_F32):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        info = H.solve(dev(b), x, tol=1e-8, precision=prec, true_residual=1)
        xs = host(x)
        assert info.status == pamg.OK
        assert np.linalg.norm(b - A.to_scipy() @ xs) <= 1e-8 * np.linalg.norm(b)
        if prec == pamg.PREC_F64:
            assert abs(info.iterations - it_or) <= 1, (info.iterations, it_or)
            if info.iterations == it_or:
                assert np.linalg.norm(xs - x_or) <= 1e-8 * np.linalg.norm(x_or)
        else:
            assert abs(info.iterations - it_or) <= 2, (info.iterations, it_or)


def test_gauss_seidel_needs_fewer_iterations_than_l1_jacobi():
    A = q1_stretched(32, 1.05)
    b = uniform_rhs(A.n, 4)
    its = {}
    for kind in ("l1", "hgs"):
        H = pamg.Hierarchy(A, smoother=kind)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        its[kind] = H.solve(dev(b), x, tol=1e-8).iterations
    assert its["hgs"] < its["l1"]


def test_batched_engine_refuses_gauss_seidel_and_update_keeps_it(built):
    A, H, O = built("varcoef_26_nb37_ragged")
    B = dev(np.stack([uniform_rhs(A.n, 1), uniform_rhs(A.n, 2)]))
    X = torch.zeros_like(B)
    with pytest.raises(pamg.PamgError) as e:
        H.solve_batch(B, X, tol=1e-6)
    assert e.value.code == pamg.E_INVALID
    # coefficient update: 4A gives bitwise the solve of a fresh 4A setup
    mk, steps, nu, nb, om, _ = CASES["varcoef_26_nb37_ragged"]
    A4 = CSR(A.n, A.row_ptr, A.col, 4.0 * A.val)
    G = pamg.Hierarchy(A, agg_steps=steps, smoother="hgs", sweeps=nu, gs_block=nb, omega=om)
    F = pamg.Hierarchy(A4, agg_steps=steps, smoother="hgs", sweeps=nu, gs_block=nb, omega=om)
    G.update_values(A4.val)
    b = uniform_rhs(A.n, 12)
    xs = []
    for K in (G, F):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        K.solve(dev(b), x, tol=1e-8)
        xs.append(host(x))
    assert np.array_equal(xs[0].view(np.uint64), xs[1].view(np.uint64))
