"""The oracle's all-cores timing build (the CPU baseline's second figure)
computes bitwise what the plain single-threaded build computes: its row and
element loops are split over threads, every reduction stays serial."""
import os
import subprocess
import sys

import numpy as np

import oracle
from workloads import q1_rhs, q1_stretched

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, hashlib
import numpy as np
sys.path.insert(0, {root!r})
import oracle
if {omp}:
    oracle.use_openmp_build()
from workloads import q1_rhs, q1_stretched
A = q1_stretched(10, 1.05)
b = q1_rhs(10, 1.05, 2)
H = oracle.Hierarchy(A)
x, it, rr, st = H.solve(b, 1e-8)
x6, _, _, _ = H.solve(b, 0.0, fixed_iters=6, krylov="cg")
print(it, hashlib.sha256(x.tobytes() + x6.tobytes()).hexdigest())
"""


def run(omp):
    env = dict(os.environ, OMP_NUM_THREADS="4")
    env.pop("ORACLE_LIB_OVERRIDE", None)
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, omp=omp)], env=env, capture_output=True,
                       text=True, timeout=300, check=True)
    return r.stdout.split()


def test_openmp_build_is_bitwise_the_plain_build():
    oracle.build()
    plain, omp = run(False), run(True)
    assert plain == omp
    assert int(plain[0]) > 0
