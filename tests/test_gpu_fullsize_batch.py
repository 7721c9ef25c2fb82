"""Parity of the 16-right-hand-side engine at full size: the 128^3
stretched-mesh Q1 operator (2,130,047 dofs) with the 16 right-hand sides of
consecutive time steps (base divergence field, seed 4, plus 15 successive 5 %
perturbations), in the configuration the benchmark times (autotuned
variants, graph-replayed blocks).

Expected values are the oracle's, stored by tests/golden/make_golden_batch.py:
per column the FCG iteration count to 1e-6 and sampled entries of x and of
the 6-iteration iterate.  FP64 V-cycle: fixed-6 samples within 1e-8,
iterations within +-1, x samples within 1e-8 when the counts agree, true
residual <= 1e-6.  FP32 V-cycle under the FP64 recurrences: true residual
<= 1e-6 and the error against the oracle's FP64 solution reported and
bounded (1e-4 on the samples).
"""
import json
import os

import numpy as np
import pytest

import paper_2210_16660_amd as pamg
from workloads import q1_rhs_sequence, q1_stretched

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "q1_128_batch16.json")))


@pytest.fixture(scope="module")
def c4():
    assert torch.cuda.is_available()
    w = GOLD["workload"]
    A = q1_stretched(w["q1_elements"], w["ratio"])
    assert A.n == w["n"] and A.nnz == w["nnz"]
    Bm = q1_rhs_sequence(w["q1_elements"], w["ratio"], w["rhs_seed"], w["columns"]).T.copy()   # (16, n)
    print(f"[fullsize batch] n={A.n} nnz={A.nnz}", flush=True)
    H = pamg.Hierarchy(A, build_f32=1)
    return A, Bm, H, np.array(GOLD["sample_index"])


def test_batch_fixed_iterations_full_size(c4):
    A, Bm, H, idx = c4
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(torch.from_numpy(Bm).cuda(), X, tol=0.0, fixed_iters=GOLD["fixed_iters"])
    Xh = X.cpu().numpy()
    for j, col in enumerate(GOLD["columns"]):
        assert infos[j].iterations == GOLD["fixed_iters"]
        g = np.array(col["xk_sample"])
        assert np.linalg.norm(Xh[j][idx] - g) <= 1e-8 * np.linalg.norm(g), j
        assert abs(np.linalg.norm(Xh[j]) - col["xk_norm"]) <= 1e-8 * col["xk_norm"], j


@pytest.mark.parametrize("prec", [pamg.PREC_F64, pamg.PREC_F32])
def test_batch_to_tolerance_full_size(c4, prec):
    A, Bm, H, idx = c4
    X = torch.zeros(Bm.shape, dtype=torch.float64, device="cuda:0")
    infos = H.solve_batch(torch.from_numpy(Bm).cuda(), X, tol=GOLD["fcg_tol"], precision=prec)
    Xh = X.cpu().numpy()
    S = A.to_scipy()
    errs, its = [], []
    for j, col in enumerate(GOLD["columns"]):
        assert infos[j].status == pamg.OK, j
        rel = np.linalg.norm(Bm[j] - S @ Xh[j]) / np.linalg.norm(Bm[j])
        assert rel <= GOLD["fcg_tol"], (j, rel)
        g = np.array(col["x_sample"])
        err = np.linalg.norm(Xh[j][idx] - g) / np.linalg.norm(g)
        errs.append(err)
        its.append((infos[j].iterations, col["fcg_iterations"]))
        if prec == pamg.PREC_F64:
            assert abs(infos[j].iterations - col["fcg_iterations"]) <= 1, j
            if infos[j].iterations == col["fcg_iterations"]:
                assert err <= 1e-8, (j, err)
        else:
            assert err <= 1e-4, (j, err)
    print(f"[fullsize batch] precision {prec}: iterations (gpu, oracle) {its}; "
          f"largest sampled error vs the FP64 oracle {max(errs):.2e}", flush=True)
