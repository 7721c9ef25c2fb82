"""C-ABI library on the CPU: symbols, argument validation, and the host
setup's bit-exact parity with the oracle (aggregates and coarse matrices)."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import CSR, lap7, q1_stretched, varcoef7

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pamg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pamg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = pamg.lib()
    names = header_functions()
    assert "pamg_setup" in names and "pamg_solve" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/pamg.h but not exported"
    assert set(names) == set(pamg.SIGNATURES), "binding signatures out of sync with the header"


def test_defaults():
    p = pamg.params()
    assert (p.max_coarse, p.max_levels, p.max_dense, p.match_all_edges) == (200, 50, 8192, 0)
    assert p.min_ratio == 1.5
    assert (p.device_setup, p.device_min_rows) == (1, 0)
    o = pamg.solve_opts()
    assert o.tol == 1e-6 and o.maxit == 1000 and o.krylov == pamg.KRYLOV_FCG and o.check_every == 4


def _bad(A, **mut):
    rp, ci, v = A.row_ptr.copy(), A.col.copy(), A.val.copy()
    for k, f in mut.items():
        f(rp, ci, v)
    return CSR(A.n, rp, ci, v)


@pytest.mark.parametrize("what", ["col_range", "unsorted", "neg_diag", "no_diag", "nan", "rowptr", "rowptr_past_end"])
def test_invalid_csr_rejected(what):
    A = lap7(4)
    muts = {
        "col_range": lambda rp, ci, v: ci.__setitem__(3, 10 ** 6),
        "unsorted": lambda rp, ci, v: ci.__setitem__(slice(1, 3), ci[1:3][::-1].copy()),
        "neg_diag": lambda rp, ci, v: v.__setitem__(0, -1.0),
        "no_diag": lambda rp, ci, v: ci.__setitem__(0, 1) if ci[0] == 0 and ci[1] == 1 else None,
        "nan": lambda rp, ci, v: v.__setitem__(5, np.nan),
        "rowptr": lambda rp, ci, v: rp.__setitem__(2, rp[3] + 1),
        # a row ending past nnz (a later row then runs backwards): rejected
        # without reading the row
        "rowptr_past_end": lambda rp, ci, v: rp.__setitem__(1, rp[-1] + 100),
    }
    B = _bad(A, m=muts[what])
    with pytest.raises(pamg.PamgError) as e:
        pamg.Hierarchy(B, host_only=1)
    assert e.value.code == pamg.E_INVALID
    assert pamg.lib().pamg_last_error().decode()


def test_symmetry_check_option():
    A = lap7(4)
    B = CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    B.val[1] *= 1.0 + 2 ** -40          # break bitwise symmetry of one pair
    pamg.Hierarchy(B, host_only=1)       # accepted without the check
    with pytest.raises(pamg.PamgError) as e:
        pamg.Hierarchy(B, host_only=1, check_symmetry=1)
    assert e.value.code == pamg.E_INVALID


def test_host_only_skips_the_coarse_factorization():
    # the coarsest factorization runs on the device: an indefinite coarsest
    # matrix still gives a host-only hierarchy (the device setup reports it)
    import scipy.sparse as sp
    M = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 1.0]]))
    A = CSR(3, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)
    H = pamg.Hierarchy(A, host_only=1)
    assert H.levels == 1


def test_stalled_coarsening_stops_like_the_oracle():
    from test_oracle_pins import pairs_and_isolated, star_graph
    for A, kw in [(star_graph(299), {}), (star_graph(299), {"min_ratio": 0.0}),
                  (pairs_and_isolated(100, 100), {}), (pairs_and_isolated(99, 102), {}),
                  (pairs_and_isolated(99, 102), {"max_dense": 250})]:
        O = oracle.Hierarchy(A, **kw)
        H = pamg.Hierarchy(A, host_only=1, **kw)
        assert H.levels == O.nlevels
        assert [H.info().n[l] for l in range(H.levels)] == [O.n(l) for l in range(O.nlevels)]


def test_stall_reported():
    # a diagonal matrix has no edges: no pair can be formed above max_dense
    n = 300
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    with pytest.raises(pamg.PamgError) as e:
        pamg.Hierarchy(A, host_only=1, max_dense=100)
    assert e.value.code == pamg.E_STALLED
    H = pamg.Hierarchy(A, host_only=1)     # within max_dense: the level is the coarsest
    assert H.levels == 1


def test_bad_params_rejected():
    with pytest.raises(pamg.PamgError):
        pamg.Hierarchy(lap7(3), host_only=1, max_levels=0)
    with pytest.raises(pamg.PamgError):
        pamg.Hierarchy(lap7(3), host_only=1, max_dense=8193)
    with pytest.raises(pamg.PamgError):
        pamg.Hierarchy(lap7(3), host_only=1, min_ratio=float("nan"))
    with pytest.raises(pamg.PamgError):
        pamg.Hierarchy(lap7(3), host_only=1, agg_steps=5)
    # smoother parameters
    for kw in [dict(smooth_prolongator=2),
               dict(smoother=2), dict(sweeps=2), dict(smoother="hgs", sweeps=17),
               dict(smoother="hgs", gs_block=257), dict(smoother="hgs", omega=-1.0),
               dict(smoother="hgs", omega=float("inf")), dict(smoother="hgs", gs_block=-1)]:
        with pytest.raises(pamg.PamgError) as e:
            pamg.Hierarchy(lap7(3), host_only=1, **kw)
        assert e.value.code == pamg.E_INVALID, kw
    # defaults and the paper's nu = 4 are accepted; the Gauss-Seidel schedule
    # is built on the host
    H = pamg.Hierarchy(lap7(8), host_only=1, smoother="hgs")
    assert H.info().levels >= 2
    pamg.Hierarchy(lap7(8), host_only=1, smoother="hgs", sweeps=4, gs_block=1, omega=0.7)
    # the paper's preconditioner: smoothed prolongators over aggregates of up to
    # 8 with the hybrid Gauss-Seidel smoother
    H = pamg.Hierarchy(lap7(10), host_only=1, smoother="hgs", smooth_prolongator=1, agg_steps=3)
    assert H.info().levels >= 2


def test_host_only_hierarchy_refuses_device_calls():
    H = pamg.Hierarchy(lap7(4), host_only=1)
    with pytest.raises(pamg.PamgError) as e:
        H.solve(8, 16, stream=0)
    assert e.value.code in (pamg.E_INVALID,)
    # a coefficient update needs the device hierarchy too (refused before any
    # device call)
    with pytest.raises(pamg.PamgError) as e:
        H.update_values(lap7(4).val, stream=0)
    assert e.value.code == pamg.E_INVALID


CASES = {
    "lap7_24": (lambda: lap7(24), {}),
    "lap7_odd_13": (lambda: lap7(13), {}),
    "varcoef_20": (lambda: varcoef7(20, seed=5), {}),
    "q1_20": (lambda: q1_stretched(20, 1.05), {}),
    "q1_12_uniform": (lambda: q1_stretched(12, 1.0), {}),
    "q1_16_match_all": (lambda: q1_stretched(16, 1.05), {"match_all": True}),
    "lap7_16_small_coarse": (lambda: lap7(16), {"max_coarse": 20}),
    "varcoef_36_stalled": (lambda: varcoef7(36, seed=5000), {}),
    "q1_16_composed3": (lambda: q1_stretched(16, 1.05), {"agg_steps": 3}),
    "varcoef_20_composed2": (lambda: varcoef7(20, seed=5), {"agg_steps": 2}),
    "varcoef_18_smoothed": (lambda: varcoef7(18, seed=6), {"smooth_prolongator": True}),
    "q1_12_smoothed": (lambda: q1_stretched(12, 1.05), {"smooth_prolongator": True}),
    "q1_20_smoothed_composed3": (lambda: q1_stretched(20, 1.05), {"smooth_prolongator": True, "agg_steps": 3}),
    "varcoef_24_smoothed_composed2": (lambda: varcoef7(24, seed=7), {"smooth_prolongator": True, "agg_steps": 2}),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_setup_bitexact_with_oracle(case):
    make, kw = CASES[case]
    A = make()
    sm = bool(kw.get("smooth_prolongator", False))
    O = oracle.Hierarchy(A, max_coarse=kw.get("max_coarse", 200), match_all=kw.get("match_all", False),
                         agg_steps=kw.get("agg_steps", 1), smooth_prolongator=sm)
    H = pamg.Hierarchy(A, host_only=1, max_coarse=kw.get("max_coarse", 200),
                       match_all_edges=int(kw.get("match_all", False)), agg_steps=kw.get("agg_steps", 1),
                       smooth_prolongator=int(sm))
    assert H.levels == O.nlevels
    for l in range(H.levels - 1):
        assert np.array_equal(H.aggregates(l), O.agg(l)), f"level {l} aggregates differ"
    for l in range(H.levels):
        rp, ci, v = H.level_csr(l)
        orp, oci, ov = O.level(l)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert np.array_equal(v.view(np.uint64), ov.view(np.uint64)), f"level {l} values differ"


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_setup_independent_of_thread_count(threads):
    A = varcoef7(18, seed=9)
    ref = pamg.Hierarchy(A, host_only=1, num_threads=1)
    H = pamg.Hierarchy(A, host_only=1, num_threads=threads)
    for l in range(ref.levels - 1):
        assert np.array_equal(H.aggregates(l), ref.aggregates(l))


@pytest.mark.slow
def test_setup_bitexact_q1_128():
    A = q1_stretched(128, 1.05)
    O = oracle.Hierarchy(A)
    H = pamg.Hierarchy(A, host_only=1)
    assert H.levels == O.nlevels == 16
    for l in range(H.levels - 1):
        assert np.array_equal(H.aggregates(l), O.agg(l))
