"""Parity at 256^3 (stretched Q1, 16,908,543 dofs, 452,982,511 nonzeros; the
FP64 against FP32-hierarchy workload), in the launch configuration the
benchmark times.

Expected values are the oracle's, stored by `tests/golden/make_golden.py 256`
(level sizes, FCG iteration count to 1e-6, sampled entries and norms of x, of
the 5-iteration iterate and of z = B b).  FP64: level sizes exact, iterations
within +-1, true residual <= 1e-6, fixed-5 and (equal counts) converged
samples within 1e-8, V-cycle samples within 1e-12.  FP32 hierarchy under the
FP64 FCG: true residual <= 1e-6, error against the oracle's FP64 solution
reported and bounded.  The hierarchy (its large levels built on the device)
matches, level by level and bit for bit, the digest of the oracle's stored by
`tests/golden/make_golden_setup.py 256` (aggregates, row pointers, columns,
values).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_2210_16660_amd as pamg
from workloads import q1_rhs, q1_stretched

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "q1_256_fcg.json")))


@pytest.fixture(scope="module")
def c3():
    assert torch.cuda.is_available()
    w = GOLD["workload"]
    log = lambda m: print(f"[fullsize 256] {m}", flush=True)
    A = q1_stretched(w["q1_elements"], w["ratio"], progress=log)
    b = q1_rhs(w["q1_elements"], w["ratio"], w["rhs_seed"], progress=log)
    assert A.n == w["n"] and A.nnz == w["nnz"]
    log(f"n={A.n} nnz={A.nnz}; setup")
    H = pamg.Hierarchy(A, build_f32=1)
    log("setup done")
    return A, b, H, np.array(GOLD["sample_index"])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


def test_hierarchy_sizes_256(c3):
    A, b, H, idx = c3
    sizes, _ = H.level_sizes()
    assert sizes == GOLD["level_n"]
    assert H.info().tile_items[0] == 16


def test_solve_to_tolerance_256(c3):
    A, b, H, idx = c3
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=GOLD["fcg_tol"], krylov="fcg")
    assert info.status == pamg.OK
    assert abs(info.iterations - GOLD["fcg_iterations"]) <= 1
    xs = x.cpu().numpy()
    rel = np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b)
    assert rel <= GOLD["fcg_tol"]
    g = np.array(GOLD["x_sample"])
    err = np.linalg.norm(xs[idx] - g) / np.linalg.norm(g)
    print(f"[fullsize 256] FP64: {info.iterations} iterations (oracle {GOLD['fcg_iterations']}), "
          f"true relres {rel:.3e}, sampled error {err:.2e}", flush=True)
    if info.iterations == GOLD["fcg_iterations"]:
        assert err <= 1e-8
        assert abs(np.linalg.norm(xs) - GOLD["x_norm"]) <= 1e-8 * GOLD["x_norm"]


def test_fixed_iterations_256(c3):
    A, b, H, idx = c3
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=0.0, fixed_iters=5)
    assert info.iterations == 5
    xs = x.cpu().numpy()
    g = np.array(GOLD["x5_sample"])
    assert np.linalg.norm(xs[idx] - g) <= 1e-8 * np.linalg.norm(g)
    assert abs(np.linalg.norm(xs) - GOLD["x5_norm"]) <= 1e-8 * GOLD["x5_norm"]


def test_vcycle_sample_256(c3):
    A, b, H, idx = c3
    z = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_VCYCLE, 0, dev(b), z)
    zs = z.cpu().numpy()
    g = np.array(GOLD["z_sample"])
    assert np.linalg.norm(zs[idx] - g) <= 1e-12 * np.linalg.norm(g)
    assert abs(np.linalg.norm(zs) - GOLD["z_norm"]) <= 1e-12 * GOLD["z_norm"]


def test_mixed_precision_256(c3):
    A, b, H, idx = c3
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=GOLD["fcg_tol"], precision=pamg.PREC_F32)
    assert info.status == pamg.OK
    xs = x.cpu().numpy()
    rel = np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b)
    assert rel <= GOLD["fcg_tol"] and abs(rel - info.relres_true) <= 1e-9
    g = np.array(GOLD["x_sample"])
    err = np.linalg.norm(xs[idx] - g) / np.linalg.norm(g)
    print(f"[fullsize 256] FP32 hierarchy: {info.iterations} iterations (FP64 oracle {GOLD['fcg_iterations']}), "
          f"{info.restarts} restarts, true relres {rel:.3e}, sampled error vs the FP64 oracle {err:.2e}", flush=True)
    assert abs(info.iterations - GOLD["fcg_iterations"]) <= max(2, GOLD["fcg_iterations"] // 5)
    assert err <= 1e-4


def test_hierarchy_matches_the_oracle_digest_256(c3):
    path = os.path.join(os.path.dirname(__file__), "golden", "q1_256_setup.json")
    ref = json.load(open(path))["levels"]
    A, b, H, idx = c3
    info = H.info()
    assert info.device_levels >= 5 and info.levels == len(ref)

    def digest(a, dtype):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()

    for l, r in enumerate(ref):
        rp, ci, v = H.level_csr(l)
        assert (len(rp) - 1, int(rp[-1])) == (r["n"], r["nnz"]), l
        assert digest(rp, np.int32) == r["rp"] and digest(ci, np.int32) == r["ci"], f"level {l} pattern"
        assert digest(v, np.float64) == r["v"], f"level {l} values"
        if "agg" in r:
            assert digest(H.aggregates(l), np.int32) == r["agg"], f"level {l} aggregates"
        del rp, ci, v
