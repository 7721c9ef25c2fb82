"""Parity at the benchmark's full size (128^3 stretched Q1, 2,130,047 dofs,
56.6M nonzeros), in the launch configuration the benchmark times.

Expected values are the oracle's, stored by tests/golden/make_golden.py
(iteration count, recurrence residual and sampled entries of x, of the
5-iteration iterate and of z = B b); the level-0 SpMV is checked in full
against the oracle's plain CSR product.
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import SplitMix64, q1_rhs, q1_stretched

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "q1_128_fcg.json")))


@pytest.fixture(scope="module")
def c2():
    assert torch.cuda.is_available()
    w = GOLD["workload"]
    A = q1_stretched(w["q1_elements"], w["ratio"])
    b = q1_rhs(w["q1_elements"], w["ratio"], w["rhs_seed"])
    assert A.n == w["n"] and A.nnz == w["nnz"]
    print(f"[fullsize] n={A.n} nnz={A.nnz}", flush=True)
    H = pamg.Hierarchy(A, build_f32=1)
    return A, b, H, np.array(GOLD["sample_index"])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


def test_hierarchy_sizes(c2):
    A, b, H, idx = c2
    sizes, _ = H.level_sizes()
    assert sizes == GOLD["level_n"]


def test_solve_to_tolerance(c2):
    A, b, H, idx = c2
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=GOLD["fcg_tol"], krylov="fcg")
    assert info.status == pamg.OK
    assert abs(info.iterations - GOLD["fcg_iterations"]) <= 1
    xs = x.cpu().numpy()
    S = A.to_scipy()
    assert np.linalg.norm(b - S @ xs) <= GOLD["fcg_tol"] * np.linalg.norm(b)
    if info.iterations == GOLD["fcg_iterations"]:
        g = np.array(GOLD["x_sample"])
        assert np.linalg.norm(xs[idx] - g) <= 1e-8 * np.linalg.norm(g)
        assert abs(np.linalg.norm(xs) - GOLD["x_norm"]) <= 1e-8 * GOLD["x_norm"]


def test_fixed_iterations(c2):
    A, b, H, idx = c2
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=0.0, fixed_iters=5)
    assert info.iterations == 5
    xs = x.cpu().numpy()
    g = np.array(GOLD["x5_sample"])
    assert np.linalg.norm(xs[idx] - g) <= 1e-8 * np.linalg.norm(g)
    assert abs(np.linalg.norm(xs) - GOLD["x5_norm"]) <= 1e-8 * GOLD["x5_norm"]


def test_vcycle_sample(c2):
    A, b, H, idx = c2
    z = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_VCYCLE, 0, dev(b), z)
    zs = z.cpu().numpy()
    g = np.array(GOLD["z_sample"])
    assert np.linalg.norm(zs[idx] - g) <= 1e-12 * np.linalg.norm(g)
    assert abs(np.linalg.norm(zs) - GOLD["z_norm"]) <= 1e-12 * GOLD["z_norm"]


def test_level0_spmv_full(c2):
    A, b, H, idx = c2
    x = SplitMix64(5).uniform(A.n)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_SPMV, 0, dev(x), y)
    ref = oracle.csr_mv(A, x)
    absA = A.to_scipy()
    absA.data = np.abs(absA.data)
    scale = np.linalg.norm(absA @ np.abs(x))
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-13 * scale


def test_mixed_precision_full(c2):
    A, b, H, idx = c2
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    info = H.solve(dev(b), x, tol=1e-6, precision=pamg.PREC_F32)
    assert info.status == pamg.OK
    xs = x.cpu().numpy()
    S = A.to_scipy()
    rel = np.linalg.norm(b - S @ xs) / np.linalg.norm(b)
    assert rel <= 1e-6
    g = np.array(GOLD["x_sample"])
    err = np.linalg.norm(xs[idx] - g) / np.linalg.norm(g)
    print(f"[fullsize] FP32 V-cycle: {info.iterations} iterations (FP64 oracle {GOLD['fcg_iterations']}), "
          f"true relres {rel:.2e}, sampled error vs oracle {err:.2e}", flush=True)
    assert err <= 1e-4
