"""Write the stored digest of the hierarchy the oracle builds at 128^3 (or N^3).

Calls only the CPU oracle (and the seeded input generator): the N^3
stretched-mesh Q1 operator (ratio 1.05), pairwise aggregation with the
default stopping rules (Sec. 3.1).  For every level: its size, number of
stored entries, and SHA-256 digests of the canonical CSR arrays (row
pointer, columns, the values' binary64 bit patterns) and of the aggregate
numbering, so that a hierarchy built elsewhere can be checked bit for bit
without running the oracle.

    python tests/golden/make_golden_setup.py [N]     (default 128; writes q1_<N>_setup.json)
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import q1_stretched  # noqa: E402


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def main():
    N, ratio = (int(sys.argv[1]) if len(sys.argv) > 1 else 128), 1.05
    A = q1_stretched(N, ratio)
    O = oracle.Hierarchy(A)
    levels = []
    for l in range(O.nlevels):
        rp, ci, v = O.level(l)
        rec = {"n": int(len(rp) - 1), "nnz": int(rp[-1]), "rp": digest(rp, np.int32), "ci": digest(ci, np.int32),
               "v": digest(v, np.float64)}
        if l + 1 < O.nlevels:
            rec["agg"] = digest(O.agg(l), np.int32)
        levels.append(rec)
        print(f"level {l}: n {rec['n']} nnz {rec['nnz']}", flush=True)
    out = {"source": f"oracle.Hierarchy(q1_stretched({N}, 1.05)), default parameters",
           "digest": "sha256 of the little-endian int32 / binary64 arrays", "levels": levels}
    with open(os.path.join(HERE, f"q1_{N}_setup.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
