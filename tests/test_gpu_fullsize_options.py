"""Parity of the optional configurations at the benchmark's full size (128^3
stretched Q1, 2,130,047 dofs): aggregate-size composition, coefficient-only
reuse, the hybrid Gauss-Seidel smoother, smoothed prolongators, and both
together (the paper's preconditioner).

Expected values are the oracle's, stored by tests/golden/make_golden_options.py
(level sizes, FCG iterations to 1e-6, sampled entries of z = B b).  Bars as
for the default configuration: hierarchy sizes exact, V-cycle samples within
1e-11 of the oracle's (1e-12 for the tentative cycle's fused kernels; the
Gauss-Seidel and smoothed cycles sum rows in another order over more
operators), iterations within +-1 and the true residual at tolerance.
"""
import json
import os

import numpy as np
import pytest

import paper_2210_16660_amd as pamg
from workloads import q1_rhs, q1_stretched

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD_PATH = os.path.join(os.path.dirname(__file__), "golden", "q1_128_options.json")
GOLD = json.load(open(GOLD_PATH))

CONFIGS = {
    "agg_steps_2": (dict(agg_steps=2), None, 1e-12),
    "reuse_updated_to_1.06": (dict(), "reuse", 1e-12),
    "hybrid_gs_nu4_nb256_omega1.5": (dict(smoother="hgs", sweeps=4, gs_block=256, omega=1.5), None, 1e-11),
    "smoothed_agg_steps_3": (dict(agg_steps=3, smooth_prolongator=1), None, 1e-11),
    # the paper's preconditioner: smoothed prolongators over aggregates of up
    # to 8 with the hybrid Gauss-Seidel smoother
    "smoothed_agg_steps_3_hgs_nu2_nb64_omega2": (dict(agg_steps=3, smooth_prolongator=1, smoother="hgs", sweeps=2,
                                                      gs_block=64, omega=2.0), None, 1e-11),
}


@pytest.fixture(scope="module")
def problem():
    w = GOLD["workload"]
    A = q1_stretched(w["q1_elements"], w["ratio"])
    b = q1_rhs(w["q1_elements"], w["ratio"], w["rhs_seed"])
    assert A.n == w["n"] and A.nnz == w["nnz"]
    return A, b, np.array(GOLD["sample_index"])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_option_at_full_size(problem, name):
    A, b, idx = problem
    kw, mode, ztol = CONFIGS[name]
    g = GOLD[name]
    print(f"[fullsize-options] {name}", flush=True)
    H = pamg.Hierarchy(A, **kw)
    M = A
    if mode == "reuse":
        M = q1_stretched(GOLD["workload"]["q1_elements"], GOLD["reuse_ratio"])
        H.update_values(dev(M.val))
    info = H.info()
    assert [info.n[l] for l in range(info.levels)] == g["level_n"]
    z = torch.empty(A.n, dtype=torch.float64, device="cuda:0")
    H.debug_apply(pamg.OP_VCYCLE, 0, dev(b), z)
    zs = z.cpu().numpy()
    gz = np.array(g["z_sample"])
    assert np.linalg.norm(zs[idx] - gz) <= ztol * np.linalg.norm(gz)
    assert abs(np.linalg.norm(zs) - g["z_norm"]) <= ztol * g["z_norm"]
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
    res = H.solve(dev(b), x, tol=1e-6, true_residual=1)
    assert res.status == pamg.OK and abs(res.iterations - g["fcg_iterations"]) <= 1, (res.iterations, g)
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - M.to_scipy() @ xs) <= 1e-6 * np.linalg.norm(b)
