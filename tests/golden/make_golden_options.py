"""Write the stored expected values of the full-size parity tests of the
optional configurations (aggregate-size composition, hybrid Gauss-Seidel
smoother, smoothed prolongators, both together, coefficient-only reuse).

Calls only the CPU oracle (and the seeded input generators) on the 128^3
stretched-mesh Q1 system with its divergence right-hand side (seed 2); for
each configuration it stores the hierarchy's level sizes, sampled entries of
one V-cycle application z = B b and the FCG iteration count to 1e-6.

    python tests/golden/make_golden_options.py            # every configuration
    python tests/golden/make_golden_options.py NAME ...   # only those, into the existing file
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import SplitMix64, q1_rhs, q1_stretched  # noqa: E402

N, RATIO, SEED = 128, 1.05, 2


def record(name, O, b, idx, out):
    t = time.time()
    z = O.vcycle(b)
    x, it, rr, st = O.solve(b, 1e-6, krylov="fcg")
    assert st == 0, (name, st)
    out[name] = {
        "levels": O.nlevels,
        "level_n": [O.n(l) for l in range(O.nlevels)],
        "fcg_iterations": it,
        "fcg_relres": rr,
        "z_norm": float(np.linalg.norm(z)),
        "z_sample": [float(v) for v in z[idx]],
    }
    print(f"{name}: levels {O.nlevels}, iterations {it}, {time.time() - t:.0f}s", flush=True)


def main(names):
    A = q1_stretched(N, RATIO)
    b = q1_rhs(N, RATIO, SEED)
    idx = np.unique(SplitMix64(99).integers(600, 0, A.n - 1))[:512]
    path = os.path.join(HERE, f"q1_{N}_options.json")
    out = {"source": "oracle/oracle.c via tests/golden/make_golden_options.py",
           "workload": {"q1_elements": N, "ratio": RATIO, "rhs_seed": SEED, "n": A.n, "nnz": A.nnz},
           "sample_index": idx.tolist()}
    if names:
        out = json.load(open(path))
        assert out["sample_index"] == idx.tolist()

    def want(name):
        return not names or name in names

    if want("agg_steps_2"):
        record("agg_steps_2", oracle.Hierarchy(A, agg_steps=2), b, idx, out)
    if want("reuse_updated_to_1.06") or want("hybrid_gs_nu4_nb256_omega1.5"):
        O = oracle.Hierarchy(A)
        if want("reuse_updated_to_1.06"):
            out["reuse_ratio"] = RATIO + 0.01
            record("reuse_updated_to_1.06", O.update(q1_stretched(N, RATIO + 0.01).val), b, idx, out)
        if want("hybrid_gs_nu4_nb256_omega1.5"):
            record("hybrid_gs_nu4_nb256_omega1.5", O.set_smoother("hgs", nu=4, nb=256, omega=1.5), b, idx, out)
        del O
    if want("smoothed_agg_steps_3"):
        record("smoothed_agg_steps_3", oracle.Hierarchy(A, agg_steps=3, smooth_prolongator=True), b, idx, out)
    if want("smoothed_agg_steps_3_hgs_nu2_nb64_omega2"):
        # the paper's preconditioner (Sec. 3.1): smoothed prolongators over
        # aggregates of up to 8 with the hybrid Gauss-Seidel smoother
        O = oracle.Hierarchy(A, agg_steps=3, smooth_prolongator=True).set_smoother("hgs", nu=2, nb=64, omega=2.0)
        record("smoothed_agg_steps_3_hgs_nu2_nb64_omega2", O, b, idx, out)
        del O
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
