"""Build libpamg.so in-tree for gfx950.

* csrc/setup.cpp (host hierarchy construction) is compiled with g++ and
  -ffp-contract=off so that every weight, prolongator entry and Galerkin sum
  is one IEEE operation per written operation.
* csrc/device.hip (single right-hand side kernels, driver, C ABI),
  csrc/batch.hip (16 right-hand sides), csrc/serve.hip (server),
  csrc/dense.hip (coarsest-level factorization), csrc/reuse.hip
  (coefficient-only updates), csrc/context.hip (allocation) and
  csrc/dsetup.hip (device construction of the large levels, with
  -ffp-contract=off like setup.cpp) are compiled with hipcc for
  gfx950 (in parallel).  Packed-FP32 instructions are disabled for all device
  code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpamg.so")
ARCH = os.environ.get("PAMG_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    setup_o = os.path.join(BUILD, "setup.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-pthread",
          "-I", INC, "-I", CSRC, "-c", os.path.join(CSRC, "setup.cpp"), "-o", setup_o])
    objs = []
    procs = []
    for name in ("device", "batch", "serve", "dense", "reuse", "context", "dsetup"):
        o = os.path.join(BUILD, f"{name}.o")
        # the device setup reproduces the host's floating-point operations one by one
        exact = ["-ffp-contract=off"] if name == "dsetup" else []
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", *NO_PACKED_FP32, *exact,
               "-I", INC, "-I", CSRC, "-c", os.path.join(CSRC, f"{name}.hip"), "-o", o]
        print(" ".join(cmd), flush=True)
        procs.append((name, subprocess.Popen(cmd)))
        objs.append(o)
    failed = [name for name, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed for {', '.join(failed)}")
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, setup_o, "-o", tmp, "-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
