"""Write the stored expected values of the full-size parity test.

Calls only the CPU oracle (and the seeded input generators): the 128^3
stretched-mesh Q1 system with its divergence right-hand side (seed 2),
solved by FCG + the V-cycle to 1e-6; stores the iteration count, the
recurrence residual and sampled entries of the solution, of the 5-iteration
iterate and of one V-cycle application z = B b.

    python tests/golden/make_golden.py [N]     (N = 128 by default; 256 for the large case)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import SplitMix64, q1_rhs, q1_stretched  # noqa: E402


def main():
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 128
    ratio, seed = 1.05, {128: 2, 256: 3}.get(N, 2)
    A = q1_stretched(N, ratio)
    b = q1_rhs(N, ratio, seed)
    O = oracle.Hierarchy(A)
    idx = np.unique(SplitMix64(99).integers(600, 0, A.n - 1))[:512]
    x, it, rr, st = O.solve(b, 1e-6, krylov="fcg")
    assert st == 0
    x5, _, _, _ = O.solve(b, 0.0, krylov="fcg", fixed_iters=5)
    z = O.vcycle(b)
    nlev, level_n = O.nlevels, [O.n(l) for l in range(O.nlevels)]
    del O
    out = {
        "source": "oracle/oracle.c via tests/golden/make_golden.py",
        "workload": {"q1_elements": N, "ratio": ratio, "rhs_seed": seed, "n": A.n, "nnz": A.nnz},
        "levels": nlev,
        "level_n": level_n,
        "fcg_tol": 1e-6,
        "fcg_iterations": it,
        "fcg_relres": rr,
        "x_norm": float(np.linalg.norm(x)),
        "x5_norm": float(np.linalg.norm(x5)),
        "z_norm": float(np.linalg.norm(z)),
        "sample_index": idx.tolist(),
        "x_sample": [float(v) for v in x[idx]],
        "x5_sample": [float(v) for v in x5[idx]],
        "z_sample": [float(v) for v in z[idx]],
    }
    with open(os.path.join(HERE, f"q1_{N}_fcg.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"levels {nlev}, iterations {it}, relres {rr:.3e}")


if __name__ == "__main__":
    main()
