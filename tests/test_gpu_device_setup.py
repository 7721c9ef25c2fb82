"""Device construction of the large levels (pamg_params.device_setup) through
the C ABI.

* aggregates and every level's matrix (row pointers, columns, the values'
  bit patterns) equal the oracle's on grids whose finest levels are built on
  the device, down to small levels, with and without column dictionaries,
  including a stalled coarsening;
* at 128^3 the hierarchy matches the stored digest of the oracle's;
* a device-built hierarchy solves bitwise like the host-built one (FP64 and
  FP32 V-cycles, fixed iterations and to tolerance), so its layout (row
  order, tiles, dictionaries) is equivalent;
* coefficient-only updates work on a device-built hierarchy and give the
  host-built hierarchy's results;
* with aggregate-size composition (agg_steps 2 and 3) the kept levels'
  composed aggregates, matrices and solves are the oracle's / host's too;
* configurations the device construction does not cover (small inputs, an
  unsymmetric pattern, the hybrid Gauss-Seidel smoother) are built on the
  host, with identical results;
* the device checks a large input's rows as the host does: every kind of
  defect is refused with the host build's code and message, and the
  optional bitwise symmetry check too.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import CSR, SplitMix64, lap7, q1_stretched, varcoef7

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


# name: (matrix, pamg params, oracle params, least number of device levels)
CASES = {
    "q1_40": (lambda: q1_stretched(40, 1.05), {"device_min_rows": 1000}, {}, 3),
    "varcoef_48": (lambda: varcoef7(48, seed=21), {"device_min_rows": 1000}, {}, 3),
    "lap7_44": (lambda: lap7(44), {"device_min_rows": 1000}, {}, 3),
    "q1_32_deep": (lambda: q1_stretched(32, 1.05), {"device_min_rows": 64, "max_dense": 256},
                   {"max_dense": 256}, 5),
    "varcoef_36_stalled": (lambda: varcoef7(36, seed=5000), {"device_min_rows": 64, "max_dense": 512},
                           {"max_dense": 512}, 2),
    "lap7_30_small_coarse": (lambda: lap7(30), {"device_min_rows": 64, "max_dense": 64, "max_coarse": 20},
                             {"max_dense": 64, "max_coarse": 20}, 6),
    "q1_40_composed2": (lambda: q1_stretched(40, 1.05), {"device_min_rows": 1000, "agg_steps": 2},
                        {"agg_steps": 2}, 2),
    "varcoef_48_composed3": (lambda: varcoef7(48, seed=21), {"device_min_rows": 1000, "agg_steps": 3},
                             {"agg_steps": 3}, 1),
    "q1_32_deep_composed2": (lambda: q1_stretched(32, 1.05), {"device_min_rows": 64, "max_dense": 256,
                                                             "agg_steps": 2}, {"max_dense": 256, "agg_steps": 2}, 3),
}


def check_against_oracle(H, O):
    assert H.levels == O.nlevels
    for l in range(H.levels - 1):
        assert np.array_equal(H.aggregates(l), O.agg(l)), f"level {l} aggregates differ"
    for l in range(H.levels):
        rp, ci, v = H.level_csr(l)
        orp, oci, ov = O.level(l)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci), f"level {l} pattern differs"
        assert np.array_equal(v.view(np.uint64), ov.view(np.uint64)), f"level {l} values differ"


@pytest.mark.parametrize("case", sorted(CASES))
def test_device_setup_bitexact_with_oracle(case):
    make, kw, okw, least = CASES[case]
    A = make()
    H = pamg.Hierarchy(A, device_setup=1, **kw)
    info = H.info()
    print(case, "device levels", info.device_levels, "of", info.levels, flush=True)
    assert info.device_levels >= least
    O = oracle.Hierarchy(A, max_coarse=okw.get("max_coarse", 200), max_dense=okw.get("max_dense", 8192),
                         agg_steps=okw.get("agg_steps", 1))
    check_against_oracle(H, O)


def test_device_setup_matches_the_oracle_digest_at_128():
    with open(os.path.join(HERE, "golden", "q1_128_setup.json")) as f:
        ref = json.load(f)["levels"]
    A = q1_stretched(128, 1.05)
    H = pamg.Hierarchy(A, device_setup=1)
    info = H.info()
    print("128^3 device levels", info.device_levels, "of", info.levels, f"setup {info.setup_ms:.0f} ms", flush=True)
    assert info.device_levels >= 5 and info.levels == len(ref)

    def digest(a, dtype):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()

    for l, r in enumerate(ref):
        rp, ci, v = H.level_csr(l)
        assert (len(rp) - 1, int(rp[-1])) == (r["n"], r["nnz"])
        assert digest(rp, np.int32) == r["rp"] and digest(ci, np.int32) == r["ci"], f"level {l} pattern"
        assert digest(v, np.float64) == r["v"], f"level {l} values"
        if "agg" in r:
            assert digest(H.aggregates(l), np.int32) == r["agg"], f"level {l} aggregates"


@pytest.mark.parametrize("case", ["q1_40", "varcoef_48", "q1_32_deep", "q1_40_composed2", "varcoef_48_composed3"])
def test_device_built_hierarchy_solves_like_the_host_built_one(case):
    make, kw, _, _ = CASES[case]
    A = make()
    Hd = pamg.Hierarchy(A, device_setup=1, build_f32=1, **kw)
    Hh = pamg.Hierarchy(A, device_setup=0, build_f32=1, **{k: v for k, v in kw.items() if k != "device_min_rows"})
    assert Hd.info().device_levels >= 1 and Hh.info().device_levels == 0
    assert list(Hd.info().tile_items)[:Hd.levels] == list(Hh.info().tile_items)[:Hh.levels]
    b = dev(SplitMix64(77).uniform(A.n))
    for prec in (pamg.PREC_F64, pamg.PREC_F32):
        for kwargs in ({"fixed_iters": 7, "tol": 0.0}, {"tol": 1e-8}):
            xd = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
            xh = torch.zeros_like(xd)
            idd = Hd.solve(b, xd, precision=prec, **kwargs)
            ih = Hh.solve(b, xh, precision=prec, **kwargs)
            assert idd.iterations == ih.iterations
            assert torch.equal(xd, xh), (prec, kwargs)


@pytest.mark.parametrize("case", ["q1_40_nb64", "varcoef_48_nb256_composed2", "q1_32_nb37"])
def test_gauss_seidel_schedule_on_the_device_solves_like_the_host_one(case):
    # the hybrid Gauss-Seidel schedule (depths, in-block entry ranges, 1 / a_ii)
    # built on the device is the host's, so the solves agree bit for bit
    make, kw = {
        "q1_40_nb64": (lambda: q1_stretched(40, 1.05), dict(sweeps=2, gs_block=64, omega=2.0)),
        "varcoef_48_nb256_composed2": (lambda: varcoef7(48, seed=34), dict(agg_steps=2)),
        "q1_32_nb37": (lambda: q1_stretched(32, 1.05), dict(sweeps=3, gs_block=37, omega=1.2)),
    }[case]
    A = make()
    Hd = pamg.Hierarchy(A, device_setup=1, device_min_rows=1000, build_f32=1, smoother="hgs", **kw)
    Hh = pamg.Hierarchy(A, device_setup=0, build_f32=1, smoother="hgs", **kw)
    assert Hd.info().device_levels >= 1 and Hh.info().device_levels == 0
    for l in range(Hh.levels - 1):
        assert np.array_equal(Hd.aggregates(l), Hh.aggregates(l))
    b = dev(SplitMix64(78).uniform(A.n))
    for prec in (pamg.PREC_F64, pamg.PREC_F32):
        for kwargs in ({"fixed_iters": 5, "tol": 0.0}, {"tol": 1e-8}):
            xd = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
            xh = torch.zeros_like(xd)
            idd = Hd.solve(b, xd, precision=prec, **kwargs)
            ih = Hh.solve(b, xh, precision=prec, **kwargs)
            assert idd.iterations == ih.iterations
            assert torch.equal(xd, xh), (prec, kwargs)
    if case == "q1_40_nb64":
        # a coefficient update recomputes 1 / a_ii of every level on the device,
        # on the device-built levels too: still bitwise the host-built hierarchy
        A2 = q1_stretched(40, 1.07)
        assert np.array_equal(A2.col, A.col)
        Hd.update_values(A2.val)
        Hh.update_values(A2.val)
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        xh = torch.zeros_like(xd)
        assert Hd.solve(b, xd, tol=1e-8).iterations == Hh.solve(b, xh, tol=1e-8).iterations
        assert torch.equal(xd, xh)


@pytest.mark.parametrize("steps", [1, 2])
def test_coefficient_update_on_a_device_built_hierarchy(steps):
    A = varcoef7(40, seed=31)
    B = varcoef7(40, seed=32)          # same pattern, new coefficients
    Hd = pamg.Hierarchy(A, device_setup=1, device_min_rows=1000, agg_steps=steps)
    Hh = pamg.Hierarchy(A, device_setup=0, agg_steps=steps)
    assert Hd.info().device_levels >= 1
    Hd.update_values(B.val)
    Hh.update_values(B.val)
    for l in range(Hh.levels):
        assert all(np.array_equal(u, w) for u, w in zip(Hd.level_csr(l), Hh.level_csr(l)))
    b = dev(SplitMix64(5).uniform(A.n))
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    xh = torch.zeros_like(xd)
    assert Hd.solve(b, xd, tol=1e-8).iterations == Hh.solve(b, xh, tol=1e-8).iterations
    assert torch.equal(xd, xh)


def drop_upper_entry(A, row):
    """A copy of A without the first stored entry right of the diagonal in
    `row` (the pattern is then unsymmetric)."""
    rp, ci, v = A.row_ptr.copy(), A.col.copy(), A.val.copy()
    k = next(k for k in range(rp[row], rp[row + 1]) if ci[k] > row)
    keep = np.ones(len(ci), bool)
    keep[k] = False
    rp2 = rp.copy()
    rp2[row + 1:] -= 1
    return CSR(A.n, rp2.astype(np.int32), ci[keep].astype(np.int32), v[keep])


def test_configurations_left_to_the_host():
    cases = [
        (lap7(20), {}),                                     # below the size floor
        (drop_upper_entry(lap7(40), 1234), {"device_min_rows": 1000}),   # unsymmetric pattern
        (lap7(40), {"device_min_rows": 1000, "agg_steps": 2, "smooth_prolongator": 1}),
    ]
    for A, kw in cases:
        Hd = pamg.Hierarchy(A, device_setup=1, **kw)
        Hh = pamg.Hierarchy(A, device_setup=0, **{k: v for k, v in kw.items() if k != "device_min_rows"})
        assert Hd.info().device_levels == 0
        assert Hd.levels == Hh.levels
        for l in range(Hh.levels - 1):
            assert np.array_equal(Hd.aggregates(l), Hh.aggregates(l))


def test_value_asymmetry_uses_the_upper_entry_like_the_host():
    # a structurally symmetric matrix whose lower triangle differs in the last
    # bit: the matching weighs each edge by its upper entry on both paths
    A = varcoef7(40, seed=33)
    v = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    low = A.col < rows
    v[low] = np.nextafter(v[low], 0.0)
    B = CSR(A.n, A.row_ptr, A.col, v)
    Hd = pamg.Hierarchy(B, device_setup=1, device_min_rows=1000)
    Hh = pamg.Hierarchy(B, device_setup=0)
    assert Hd.info().device_levels >= 2
    for l in range(Hh.levels - 1):
        assert np.array_equal(Hd.aggregates(l), Hh.aggregates(l))
    for l in range(Hh.levels):
        assert all(np.array_equal(u, w) for u, w in zip(Hd.level_csr(l), Hh.level_csr(l)))


@pytest.mark.parametrize("what", ["col_range", "unsorted", "neg_diag", "no_diag", "nan", "rowptr",
                                  "rowptr_past_end"])
def test_device_validation_refuses_like_the_host(what):
    # one defect in row 7000 of a matrix the device would build
    A = lap7(42)
    rp, ci, v = A.row_ptr.copy(), A.col.copy(), A.val.copy()
    r = 7000
    b = rp[r]
    d = b + int(np.flatnonzero(ci[b:rp[r + 1]] == r)[0])      # the diagonal entry
    if what == "col_range":
        ci[b] = 10 ** 7
    elif what == "unsorted":
        ci[b], ci[b + 1] = ci[b + 1], ci[b]
    elif what == "neg_diag":
        v[d] = -1.0
    elif what == "no_diag":
        ci[d] = r + 2                                           # between r + 1 and r + 42 in lap7(42)
        ci[b:rp[r + 1]] = np.sort(ci[b:rp[r + 1]])
    elif what == "nan":
        v[b + 1] = np.nan
    elif what == "rowptr":
        rp[r + 1] = rp[r] - 1
    elif what == "rowptr_past_end":
        rp[r + 1] = rp[-1] + 100
    B = CSR(A.n, rp, ci, v)
    msgs = []
    for ds in (1, 0):
        with pytest.raises(pamg.PamgError) as e:
            pamg.Hierarchy(B, device_setup=ds, device_min_rows=1000)
        assert e.value.code == pamg.E_INVALID
        msgs.append(str(e.value))
    assert msgs[0].split(": ", 1)[1] == msgs[1].split(": ", 1)[1], msgs   # the smallest failing row on both
    assert msgs[0].endswith(f"in row {r}"), msgs


def test_device_symmetry_check():
    A = varcoef7(42, seed=3)
    v = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    k = int(np.flatnonzero(A.col > rows)[1234])                  # one upper entry
    v[k] = v[k] * (1.0 + 2 ** -40)
    B = CSR(A.n, A.row_ptr, A.col, v)
    assert pamg.Hierarchy(B, device_setup=1, device_min_rows=1000).info().device_levels >= 1
    with pytest.raises(pamg.PamgError) as e:
        pamg.Hierarchy(B, device_setup=1, device_min_rows=1000, check_symmetry=1)
    assert e.value.code == pamg.E_INVALID and "symmetric" in str(e.value)
