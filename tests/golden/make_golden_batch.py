"""Write the stored expected values of the full-size 16-right-hand-side test.

Calls only the CPU oracle (and the seeded input generators): the 128^3
stretched-mesh Q1 operator with 16 right-hand sides from consecutive time
steps (a base divergence field from seed 4 plus 15 successive smooth
perturbations of 5 % amplitude, seeds 5..19); for every column the FCG
solve to 1e-6 (iteration count, recurrence residual, sampled entries and
norm of x) and the 6-iteration iterate (sampled entries and norm).

    python tests/golden/make_golden_batch.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import SplitMix64, q1_rhs_sequence, q1_stretched  # noqa: E402


def main():
    N, ratio, seed, K = 128, 1.05, 4, 6
    A = q1_stretched(N, ratio)
    B = q1_rhs_sequence(N, ratio, seed, 16)                # (n, 16)
    O = oracle.Hierarchy(A)
    idx = np.unique(SplitMix64(98).integers(600, 0, A.n - 1))[:512]
    cols = []
    for j in range(16):
        b = np.ascontiguousarray(B[:, j])
        x, it, rr, st = O.solve(b, 1e-6, krylov="fcg")
        assert st == 0
        xk, _, _, _ = O.solve(b, 0.0, krylov="fcg", fixed_iters=K)
        cols.append({"fcg_iterations": it, "fcg_relres": rr, "x_norm": float(np.linalg.norm(x)),
                     "x_sample": [float(v) for v in x[idx]], "xk_norm": float(np.linalg.norm(xk)),
                     "xk_sample": [float(v) for v in xk[idx]]})
        print(f"column {j}: {it} iterations, relres {rr:.3e}", flush=True)
    out = {
        "source": "oracle/oracle.c via tests/golden/make_golden_batch.py",
        "workload": {"q1_elements": N, "ratio": ratio, "rhs_seed": seed, "columns": 16, "n": A.n, "nnz": A.nnz},
        "fcg_tol": 1e-6,
        "fixed_iters": K,
        "sample_index": idx.tolist(),
        "columns": cols,
    }
    with open(os.path.join(HERE, f"q1_{N}_batch16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
