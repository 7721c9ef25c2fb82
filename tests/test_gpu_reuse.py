"""Coefficient-only reuse through the C ABI (pamg_hierarchy_update_values).

* the device update gives, level by level, bitwise the oracle's update
  (Galerkin chain with the kept aggregates, R13), also with aggregate-size
  composition and for values handed over from device memory;
* scaling A by 4 (edge weights unchanged, so the matchings are the same)
  makes the updated hierarchy bitwise a fresh setup of 4A: same levels and the
  same solve, bit for bit, FP64 and FP32 V-cycles, single and batched;
* a solve on the updated hierarchy agrees with the oracle's solve on the
  oracle's updated hierarchy (same tolerances as the other solve parity);
* invalid values are refused before anything changes; updating back to the
  original values restores the original solve bitwise.
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


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))


def check_levels_equal_oracle(H, O):
    assert H.levels == O.nlevels
    for l in range(O.nlevels):
        rp, ci, v = H.level_csr(l)
        orp, oci, ov = O.level(l)
        assert same_bits(rp, orp) and same_bits(ci, oci), l
        assert same_bits(v, ov), f"level {l} values differ"


def solve(H, b, **kw):
    x = torch.zeros(H.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, **kw)
    return host(x), info


@pytest.mark.parametrize("steps", [1, 2])
@pytest.mark.parametrize("on_device", [False, True])
def test_update_matches_oracle_update_bitwise(steps, on_device):
    A, B = varcoef7(22, seed=11), varcoef7(22, seed=12)
    H = pamg.Hierarchy(A, agg_steps=steps)
    O = oracle.Hierarchy(A, agg_steps=steps).update(B.val)
    H.update_values(dev(B.val) if on_device else B.val)
    check_levels_equal_oracle(H, O)
    # the solve on the updated hierarchy against the oracle's
    b = uniform_rhs(A.n, 5)
    x, info = solve(H, b, tol=1e-8)
    x_or, it_or, _, _ = O.solve(b, 1e-8)
    assert info.status == pamg.OK and abs(info.iterations - it_or) <= 1
    assert np.linalg.norm(b - B.to_scipy() @ x) <= 1e-8 * np.linalg.norm(b)
    if info.iterations == it_or:
        assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or)
    # a second update (plans reused) back to A equals the oracle's setup of A
    H.update_values(A.val)
    check_levels_equal_oracle(H, oracle.Hierarchy(A, agg_steps=steps))


@pytest.mark.parametrize("case", ["q1_20", "varcoef_26_composed3"])
def test_scaled_update_is_bitwise_a_fresh_setup(case):
    A = {"q1_20": lambda: q1_stretched(20, 1.05), "varcoef_26_composed3": lambda: varcoef7(26, seed=13)}[case]()
    kw = {"agg_steps": 3} if "composed3" in case else {}
    A4 = CSR(A.n, A.row_ptr, A.col, 4.0 * A.val)
    H = pamg.Hierarchy(A, build_f32=1, **kw)
    F = pamg.Hierarchy(A4, build_f32=1, **kw)
    H.update_values(A4.val)
    for l in range(F.levels):
        assert all(same_bits(x, y) for x, y in zip(H.level_csr(l), F.level_csr(l))), l
    b = uniform_rhs(A.n, 6)
    for prec in (pamg.PREC_F64, pamg.PREC_F32):
        xh, ih = solve(H, b, tol=1e-8, precision=prec)
        xf, if_ = solve(F, b, tol=1e-8, precision=prec)
        assert ih.iterations == if_.iterations and same_bits(xh, xf), prec
    # batched engine of the updated hierarchy: bitwise the fresh one's
    Bm = np.stack([uniform_rhs(A.n, 20 + j) for j in range(3)])
    Xh = torch.zeros((3, A.n), dtype=torch.float64, device="cuda:0")
    Xf = torch.zeros_like(Xh)
    ih = H.solve_batch(dev(Bm), Xh, tol=1e-8)
    if_ = F.solve_batch(dev(Bm), Xf, tol=1e-8)
    assert [i.iterations for i in ih] == [i.iterations for i in if_]
    assert same_bits(host(Xh), host(Xf))


def test_invalid_values_refused_and_hierarchy_unchanged():
    A = varcoef7(16, seed=14)
    H = pamg.Hierarchy(A)
    b = uniform_rhs(A.n, 7)
    x0, _ = solve(H, b, tol=1e-8)
    bad = A.val.copy()
    bad[A.row_ptr[5]:A.row_ptr[6]] *= -1.0       # negative diagonal in row 5
    with pytest.raises(pamg.PamgError) as e:
        H.update_values(bad)
    assert e.value.code == pamg.E_INVALID
    nan = A.val.copy()
    nan[7] = np.nan
    with pytest.raises(pamg.PamgError) as e:
        H.update_values(dev(nan))
    assert e.value.code == pamg.E_INVALID
    with pytest.raises(ValueError):
        H.update_values(A.val[:-1])
    x1, _ = solve(H, b, tol=1e-8)
    assert same_bits(x0, x1)
    # new values, then back: the original solve bit for bit
    H.update_values(varcoef7(16, seed=15).val)
    x2, _ = solve(H, b, tol=1e-8)
    assert not same_bits(x0, x2)
    H.update_values(A.val)
    x3, _ = solve(H, b, tol=1e-8)
    assert same_bits(x0, x3)
