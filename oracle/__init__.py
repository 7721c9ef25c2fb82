"""ctypes binding of the CPU FP64 oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a test may point the binding at a deliberately mutated build of the oracle
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOT_SPD, E_NUMERIC, E_OOM, E_STALLED = -1, -2, -3, -4, -6

BUILD_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             _SRC, "-o", _LIB, "-lm"]


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build() -> str:
    """Compile the oracle (gcc, no FMA contraction), and its all-cores timing
    build (the same source with -fopenmp: the solve phase's row and element
    loops split over threads, results bitwise those of the plain build)."""
    for lib_path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        tmp = lib_path + ".tmp"
        cmd = BUILD_CMD[:-3] + extra + ["-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return _LIB


_lib = None


def use_openmp_build() -> None:
    """Load the all-cores timing build instead of the plain one (must be called
    before the first use of the oracle in this process)."""
    global _LIB_OVERRIDE
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
        build()
    _LIB_OVERRIDE = _LIB_OMP


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.oracle_setup.argtypes = [C.c_int, ip, ip, dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                   C.c_int, C.c_int, C.POINTER(vp)]
        L.oracle_prolongator_nnz.argtypes = [vp, C.c_int]
        L.oracle_prolongator_nnz.restype = C.c_long
        L.oracle_prolongator_omega.argtypes = [vp, C.c_int]
        L.oracle_prolongator_omega.restype = C.c_double
        L.oracle_get_prolongator.argtypes = [vp, C.c_int, ip, ip, dp]
        L.oracle_setup.restype = C.c_int
        L.oracle_round_f32.argtypes = [vp, C.POINTER(vp)]
        L.oracle_round_f32.restype = C.c_int
        L.oracle_update.argtypes = [vp, dp, C.POINTER(vp)]
        L.oracle_update.restype = C.c_int
        L.oracle_set_smoother.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double]
        L.oracle_set_smoother.restype = C.c_int
        L.oracle_nested_order.argtypes = [vp, C.c_int, ip]
        L.oracle_hgs_smooth.argtypes = [vp, C.c_int, C.c_int, C.c_int, dp, dp]
        L.oracle_free.argtypes = [vp]
        for name in ("oracle_nlevels",):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = C.c_int
        L.oracle_level_n.argtypes = [vp, C.c_int]
        L.oracle_level_n.restype = C.c_int
        L.oracle_level_pairs.argtypes = [vp, C.c_int]
        L.oracle_level_pairs.restype = C.c_int
        L.oracle_level_nnz.argtypes = [vp, C.c_int]
        L.oracle_level_nnz.restype = C.c_long
        L.oracle_get_level.argtypes = [vp, C.c_int, ip, ip, dp]
        L.oracle_get_agg.argtypes = [vp, C.c_int, ip]
        for name in ("oracle_get_p", "oracle_get_w", "oracle_get_dinv"):
            getattr(L, name).argtypes = [vp, C.c_int, dp]
        L.oracle_get_chol.argtypes = [vp, dp]
        L.oracle_spmv.argtypes = [vp, C.c_int, dp, dp]
        L.oracle_restrict.argtypes = [vp, C.c_int, dp, dp]
        L.oracle_prolong_add.argtypes = [vp, C.c_int, dp, dp]
        L.oracle_coarse_solve.argtypes = [vp, dp, dp]
        L.oracle_vcycle.argtypes = [vp, C.c_int, dp, dp]
        L.oracle_solve.argtypes = [vp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, ip, dp]
        L.oracle_solve.restype = C.c_int
        L.oracle_csr_mv.argtypes = [C.c_int, ip, ip, dp, dp, dp]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def csr_mv(A, x):
    """y = A x with the oracle's plain row loop (no hierarchy needed)."""
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    ci = np.ascontiguousarray(A.col, np.int32)
    v = np.ascontiguousarray(A.val, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(A.n)
    lib().oracle_csr_mv(int(A.n), _p(rp, C.c_int), _p(ci, C.c_int), _p(v, C.c_double), _p(x, C.c_double),
                        _p(y, C.c_double))
    return y


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code}")
        self.code = code


class Hierarchy:
    """The oracle's AMG hierarchy in canonical (setup) numbering."""

    def __init__(self, A, max_coarse=200, max_levels=50, max_dense=8192, min_ratio=1.5, match_all=False,
                 agg_steps=1, smooth_prolongator=False, _handle=None):
        L = lib()
        if _handle is not None:
            self._h = _handle
            return
        self._keep = (np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                      np.ascontiguousarray(A.val, np.float64))
        h = C.c_void_p()
        rc = L.oracle_setup(int(A.n), _p(self._keep[0], C.c_int), _p(self._keep[1], C.c_int),
                            _p(self._keep[2], C.c_double), max_coarse, max_levels, max_dense,
                            float(min_ratio), 1 if match_all else 0, int(agg_steps),
                            1 if smooth_prolongator else 0, C.byref(h))
        if rc != 0:
            raise OracleError(rc, "oracle_setup")
        self._h = h
        del self._keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_free(h)
            self._h = None

    def round_f32(self) -> "Hierarchy":
        h = C.c_void_p()
        rc = lib().oracle_round_f32(self._h, C.byref(h))
        if rc != 0:
            raise OracleError(rc, "oracle_round_f32")
        return Hierarchy(None, _handle=h)

    def update(self, val) -> "Hierarchy":
        """The hierarchy rebuilt for new values of A_0 (same pattern), keeping
        every aggregate and prolongator (coefficient-only reuse)."""
        v = np.ascontiguousarray(val, np.float64)
        if v.shape != (self.nnz(0),):
            raise ValueError("update values must have the pattern's nnz entries")
        h = C.c_void_p()
        rc = lib().oracle_update(self._h, _p(v, C.c_double), C.byref(h))
        if rc != 0:
            raise OracleError(rc, "oracle_update")
        return Hierarchy(None, _handle=h)

    def set_smoother(self, kind: str = "l1", nu: int = 4, nb: int = 256, omega: float = 1.5):
        """'l1' (l1-Jacobi, one pre- and one post-sweep) or 'hgs' (hybrid
        forward/backward Gauss-Seidel: nu sweeps over nested-order blocks of nb)."""
        k = {"l1": 0, "hgs": 1}[kind]
        rc = lib().oracle_set_smoother(self._h, k, int(nu), int(nb), float(omega))
        if rc != 0:
            raise OracleError(rc, "oracle_set_smoother")
        return self

    def prolongator(self, l: int):
        """P_l as scipy CSR: the smoothed prolongator (R15), or the tentative
        one built from agg and p."""
        import scipy.sparse as sp
        n, nc = self.n(l), self.n(l + 1)
        nnz = lib().oracle_prolongator_nnz(self._h, l)
        if nnz == 0:
            return sp.csr_matrix((self.p(l), (np.arange(n), self.agg(l))), shape=(n, nc))
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lib().oracle_get_prolongator(self._h, l, _p(rp, C.c_int), _p(ci, C.c_int), _p(v, C.c_double))
        return sp.csr_matrix((v, ci, rp), shape=(n, nc))

    def prolongator_omega(self, l: int) -> float:
        return lib().oracle_prolongator_omega(self._h, l)

    def nested_order(self, l: int) -> np.ndarray:
        o = np.empty(self.n(l), np.int32)
        lib().oracle_nested_order(self._h, l, _p(o, C.c_int))
        return o

    def hgs_smooth(self, l, r, x=None, backward=False):
        """nu hybrid Gauss-Seidel sweeps on A_l x = r: forward from zero
        (x None), or backward from x."""
        r = np.ascontiguousarray(r, np.float64)
        if x is None:
            out = np.zeros(self.n(l))
            lib().oracle_hgs_smooth(self._h, l, 1 if backward else 0, 1, _p(r, C.c_double), _p(out, C.c_double))
        else:
            out = np.array(x, np.float64, copy=True)
            lib().oracle_hgs_smooth(self._h, l, 1 if backward else 0, 0, _p(r, C.c_double), _p(out, C.c_double))
        return out

    @property
    def nlevels(self) -> int:
        return lib().oracle_nlevels(self._h)

    def n(self, l: int) -> int:
        return lib().oracle_level_n(self._h, l)

    def nnz(self, l: int) -> int:
        return lib().oracle_level_nnz(self._h, l)

    def pairs(self, l: int) -> int:
        return lib().oracle_level_pairs(self._h, l)

    def level(self, l: int):
        n, nnz = self.n(l), self.nnz(l)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        lib().oracle_get_level(self._h, l, _p(rp, C.c_int), _p(ci, C.c_int), _p(v, C.c_double))
        return rp, ci, v

    def level_scipy(self, l: int):
        import scipy.sparse as sp
        rp, ci, v = self.level(l)
        return sp.csr_matrix((v, ci, rp), shape=(self.n(l), self.n(l)))

    def agg(self, l: int) -> np.ndarray:
        a = np.empty(self.n(l), np.int32)
        lib().oracle_get_agg(self._h, l, _p(a, C.c_int))
        return a

    def _vec(self, fn, l):
        a = np.empty(self.n(l), np.float64)
        fn(self._h, l, _p(a, C.c_double))
        return a

    def p(self, l):
        return self._vec(lib().oracle_get_p, l)

    def w(self, l):
        return self._vec(lib().oracle_get_w, l)

    def dinv(self, l):
        return self._vec(lib().oracle_get_dinv, l)

    def chol(self) -> np.ndarray:
        nL = self.n(self.nlevels - 1)
        L = np.empty((nL, nL), np.float64)
        lib().oracle_get_chol(self._h, _p(L, C.c_double))
        return L

    # ---- operators
    def spmv(self, l, x):
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty(self.n(l))
        lib().oracle_spmv(self._h, l, _p(x, C.c_double), _p(y, C.c_double))
        return y

    def restrict(self, l, t):
        t = np.ascontiguousarray(t, np.float64)
        rc = np.empty(self.n(l + 1))
        lib().oracle_restrict(self._h, l, _p(t, C.c_double), _p(rc, C.c_double))
        return rc

    def prolong_add(self, l, e, z):
        e = np.ascontiguousarray(e, np.float64)
        z = np.array(z, np.float64, copy=True)
        lib().oracle_prolong_add(self._h, l, _p(e, C.c_double), _p(z, C.c_double))
        return z

    def coarse_solve(self, r):
        r = np.ascontiguousarray(r, np.float64)
        z = np.empty(self.n(self.nlevels - 1))
        lib().oracle_coarse_solve(self._h, _p(r, C.c_double), _p(z, C.c_double))
        return z

    def vcycle(self, r, l=0):
        r = np.ascontiguousarray(r, np.float64)
        z = np.empty(self.n(l))
        lib().oracle_vcycle(self._h, l, _p(r, C.c_double), _p(z, C.c_double))
        return z

    def solve(self, b, tol=1e-6, maxit=1000, krylov="fcg", x0=None, fixed_iters=0, true_res=False):
        """Returns (x, iterations, relres, status)."""
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros(self.n(0)) if x0 is None else np.array(x0, np.float64, copy=True)
        it = C.c_int()
        rr = C.c_double()
        k = {"cg": 0, "pcg": 0, "fcg": 1}[krylov]
        st = lib().oracle_solve(self._h, _p(b, C.c_double), _p(x, C.c_double), tol, maxit, k,
                                0 if x0 is None else 1, fixed_iters, 1 if true_res else 0,
                                C.byref(it), C.byref(rr))
        return x, it.value, rr.value, st
