"""Python binding of libpamg (include/pamg.h): argument marshalling only.

Every step of setup and solve runs in the C++/HIP library; this module only
converts arguments.  Device vectors are passed as torch tensors (their data
pointers) or raw integers, and the stream defaults to torch's current stream.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpamg.so")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOT_SPD, E_NUMERIC, E_OOM, E_DEVICE, E_STALLED, E_BUSY = -1, -2, -3, -4, -5, -6, -7
PREC_F64, PREC_F32 = 0, 1
KRYLOV_CG, KRYLOV_FCG = 0, 1
OP_SPMV, OP_DOWN, OP_UP, OP_PROLONG, OP_COARSE, OP_VCYCLE, OP_KRYLOV, OP_SMOOTH = 0, 1, 2, 3, 4, 5, 6, 7
SMOOTHER_L1_JACOBI, SMOOTHER_HYBRID_GS = 0, 1
MAX_LEVELS = 64


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class pamg_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class pamg_context_stats(C.Structure):
    _fields_ = [("allocs", C.c_uint64), ("frees", C.c_uint64), ("failed", C.c_uint64), ("live_bytes", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("device", C.c_int32), ("users", C.c_int32)]


class pamg_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.POINTER(C.c_int32)),
                ("col_idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class pamg_params(C.Structure):
    _fields_ = [("max_coarse", C.c_int32), ("max_levels", C.c_int32), ("max_dense", C.c_int32),
                ("match_all_edges", C.c_int32), ("build_f32", C.c_int32), ("num_threads", C.c_int32),
                ("check_symmetry", C.c_int32), ("host_only", C.c_int32), ("min_ratio", C.c_double),
                ("agg_steps", C.c_int32), ("smoother", C.c_int32), ("sweeps", C.c_int32),
                ("gs_block", C.c_int32), ("omega", C.c_double), ("smooth_prolongator", C.c_int32),
                ("device_setup", C.c_int32), ("device_min_rows", C.c_int32), ("reserved", C.c_int32 * 2)]


class pamg_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("use_x0", C.c_int32), ("krylov", C.c_int32),
                ("precision", C.c_int32), ("check_every", C.c_int32), ("fixed_iters", C.c_int32),
                ("use_graph", C.c_int32), ("true_residual", C.c_int32), ("reserved", C.c_int32 * 8)]


class pamg_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
                ("relres", C.c_double), ("relres_true", C.c_double), ("solve_ms", C.c_double)]


class pamg_hier_info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int32 * MAX_LEVELS), ("nnz", C.c_int64 * MAX_LEVELS),
                ("pairs", C.c_int32 * MAX_LEVELS), ("setup_ms", C.c_double), ("operator_complexity", C.c_double),
                ("device_bytes", C.c_uint64), ("vcycle_bytes_f64", C.c_uint64), ("vcycle_bytes_f32", C.c_uint64),
                ("spmv_bytes", C.c_uint64), ("tile_items", C.c_int32 * MAX_LEVELS),
                ("csr_vcycle_bytes_f64", C.c_uint64), ("csr_vcycle_bytes_f32", C.c_uint64),
                ("device_levels", C.c_int32), ("reserved0", C.c_int32)]


class pamg_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("block_iters", C.c_int32), ("precision", C.c_int32),
                ("use_graph", C.c_int32), ("single_path", C.c_int32), ("batch_from", C.c_int32),
                ("setup_workers", C.c_int32), ("device_setup", C.c_int32), ("reserved", C.c_int32 * 3)]


class pamg_request(C.Structure):
    _fields_ = [("op_key", C.c_uint64), ("A", C.POINTER(pamg_csr)), ("b_dev", C.c_void_p), ("x_dev", C.c_void_p),
                ("tol", C.c_double), ("maxit", C.c_int32), ("reserved", C.c_int32), ("tag", C.c_uint64)]


class pamg_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("iterations", C.c_int32), ("relres", C.c_double),
                ("relres_true", C.c_double), ("queue_ms", C.c_double), ("latency_ms", C.c_double)]


class pamg_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("bytes_in_use", C.c_uint64), ("hbm_budget_bytes", C.c_uint64), ("cached_operators", C.c_int32),
                ("active_columns", C.c_int32), ("pending", C.c_int32), ("pad", C.c_int32), ("setups", C.c_uint64),
                ("evictions", C.c_uint64), ("blocks", C.c_uint64), ("busy_ms", C.c_double),
                ("algorithmic_bytes", C.c_uint64), ("host_setup_ms", C.c_double),
                ("device_setup_ms", C.c_double), ("engines_built", C.c_uint64), ("engines_freed", C.c_uint64)]


# every entry point declared in include/pamg.h: name -> (restype, argtypes)
_VP = C.c_void_p
SIGNATURES = {
    "pamg_params_default": (C.c_int, [C.POINTER(pamg_params)]),
    "pamg_solve_opts_default": (C.c_int, [C.POINTER(pamg_solve_opts)]),
    "pamg_context_create": (C.c_int, [C.c_int32, C.POINTER(pamg_allocator), C.POINTER(_VP)]),
    "pamg_context_destroy": (C.c_int, [_VP]),
    "pamg_context_stats_get": (C.c_int, [_VP, C.POINTER(pamg_context_stats)]),
    "pamg_setup": (C.c_int, [_VP, C.POINTER(pamg_csr), C.POINTER(pamg_params), _VP, C.POINTER(_VP)]),
    "pamg_hierarchy_destroy": (C.c_int, [_VP]),
    "pamg_hierarchy_info": (C.c_int, [_VP, C.POINTER(pamg_hier_info)]),
    "pamg_hierarchy_aggregates": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32)]),
    "pamg_hierarchy_level_csr": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double)]),
    "pamg_hierarchy_update_values": (C.c_int, [_VP, _VP, C.c_int32, _VP]),
    "pamg_solve": (C.c_int, [_VP, _VP, _VP, C.POINTER(pamg_solve_opts), _VP, C.POINTER(pamg_solve_info)]),
    "pamg_solve_noalloc": (C.c_int, [_VP, _VP, _VP, C.POINTER(pamg_solve_opts), _VP, C.POINTER(pamg_solve_info)]),
    "pamg_solve_batch": (C.c_int, [_VP, C.c_int32, _VP, C.c_int64, _VP, C.c_int64, C.POINTER(pamg_solve_opts), _VP,
                                   C.POINTER(pamg_solve_info)]),
    "pamg_batch_config": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32)]),
    "pamg_batch_set_config": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32)]),
    "pamg_debug_apply_batch": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _VP, _VP]),
    "pamg_debug_apply": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, _VP, _VP, _VP, _VP]),
    "pamg_time_kernels": (C.c_int, [_VP, C.c_int32, _VP, C.c_int32, _VP, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "pamg_time_op": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _VP, C.POINTER(C.c_double),
                               C.POINTER(C.c_uint64)]),
    "pamg_server_opts_default": (C.c_int, [C.POINTER(pamg_server_opts)]),
    "pamg_server_estimate_bytes": (C.c_int, [C.POINTER(pamg_csr), C.c_int32, C.POINTER(C.c_uint64)]),
    "pamg_server_create": (C.c_int, [_VP, C.POINTER(pamg_server_opts), C.POINTER(_VP)]),
    "pamg_server_submit": (C.c_int, [_VP, C.POINTER(pamg_request)]),
    "pamg_server_poll": (C.c_int, [_VP, C.POINTER(pamg_completion), C.c_int32, C.POINTER(C.c_int32)]),
    "pamg_server_stats_get": (C.c_int, [_VP, C.POINTER(pamg_server_stats)]),
    "pamg_server_destroy": (C.c_int, [_VP]),
    "pamg_last_error": (C.c_char_p, []),
}

_lib = None


class PamgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pamg error {code}: {msg}")
        self.code = code


def lib():
    """Load libpamg.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python paper_2210_16660_amd/build.py`")
        # PyTorch first: the library then binds to the HIP runtime PyTorch
        # loaded (one runtime per process, so that device pointers, streams
        # and the caching allocator are shared)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str, allow=(OK,)):
    if rc not in allow:
        raise PamgError(rc, f"{what}: {lib().pamg_last_error().decode()}")
    return rc


def _ptr(x):
    """Device pointer of a torch tensor (or an int)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def params(**kw) -> pamg_params:
    p = pamg_params()
    _check(lib().pamg_params_default(C.byref(p)), "pamg_params_default")
    for k, v in kw.items():
        if k == "smoother" and isinstance(v, str):
            v = {"l1": SMOOTHER_L1_JACOBI, "l1_jacobi": SMOOTHER_L1_JACOBI, "hgs": SMOOTHER_HYBRID_GS}[v]
        setattr(p, k, float(v) if k in ("min_ratio", "omega") else int(v))
    return p


def solve_opts(**kw) -> pamg_solve_opts:
    o = pamg_solve_opts()
    _check(lib().pamg_solve_opts_default(C.byref(o)), "pamg_solve_opts_default")
    for k, v in kw.items():
        if k == "krylov" and isinstance(v, str):
            v = {"cg": KRYLOV_CG, "pcg": KRYLOV_CG, "fcg": KRYLOV_FCG}[v]
        if k == "precision" and isinstance(v, str):
            v = {"f64": PREC_F64, "fp64": PREC_F64, "f32": PREC_F32, "fp32": PREC_F32}[v]
        setattr(o, k, v if k == "tol" else int(v))
    return o


class Context:
    """A pamg_context: the device and the allocator of every device buffer of
    the hierarchies and servers made with it.

    allocator="torch" (default): PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc/delete on the stream the library
    names); "hip": hipMalloc/hipFree; or a pair of Python callables
    (alloc(nbytes, stream) -> device pointer or 0, free(ptr, stream)).  Keep
    the context alive while its hierarchies and servers exist (they hold a
    reference)."""

    def __init__(self, device=None, allocator="torch"):
        if device is None:
            import torch
            device = torch.cuda.current_device()
        self.device = int(device)
        self._cb = None
        if allocator == "hip":
            a = None
        else:
            if allocator == "torch":
                alloc_py, free_py = _torch_allocator(self.device)
            else:
                alloc_py, free_py = allocator

            def _alloc(nbytes, stream, user):
                try:
                    return int(alloc_py(int(nbytes), int(stream or 0))) or None
                except Exception:          # an allocator failure is reported as PAMG_E_OOM
                    return None

            def _free(ptr, stream, user):
                try:
                    free_py(int(ptr), int(stream or 0))
                except Exception:
                    pass

            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            a = pamg_allocator(self._cb[0], self._cb[1], None)
        h = C.c_void_p()
        _check(lib().pamg_context_create(self.device, C.byref(a) if a is not None else None, C.byref(h)),
               "pamg_context_create")
        self._h = h

    def stats(self) -> pamg_context_stats:
        st = pamg_context_stats()
        _check(lib().pamg_context_stats_get(self._h, C.byref(st)), "pamg_context_stats_get")
        return st

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _check(_lib.pamg_context_destroy(self._h), "pamg_context_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except PamgError:
            pass


def _torch_allocator(device):
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, device, stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


_default_contexts = {}


def default_context(device=None) -> Context:
    """The binding's context per device: PyTorch's caching allocator."""
    import torch
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default_contexts:
        _default_contexts[d] = Context(d, "torch")
    return _default_contexts[d]


class Hierarchy:
    """An AMG hierarchy built by pamg_setup (owned by the library).  Its device
    buffers come from `context` (default: the binding's PyTorch-allocator
    context of the current device)."""

    def __init__(self, A, stream=None, context=None, **kw):
        rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.col, dtype=np.int32)
        v = np.ascontiguousarray(A.val, dtype=np.float64)
        csr = pamg_csr(int(A.n), int(rp[-1]), rp.ctypes.data_as(C.POINTER(C.c_int32)),
                       ci.ctypes.data_as(C.POINTER(C.c_int32)), v.ctypes.data_as(C.POINTER(C.c_double)))
        self.params = params(**kw)
        h = C.c_void_p()
        if self.params.host_only:
            s, self.context = None, context
        else:
            s, self.context = _stream(stream), context if context is not None else default_context()
        _check(lib().pamg_setup(self.context._h if self.context is not None else None, C.byref(csr),
                                C.byref(self.params), s, C.byref(h)), "pamg_setup")
        self._h = h
        self.n = int(A.n)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.pamg_hierarchy_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def info(self) -> pamg_hier_info:
        i = pamg_hier_info()
        _check(lib().pamg_hierarchy_info(self._h, C.byref(i)), "pamg_hierarchy_info")
        return i

    @property
    def levels(self) -> int:
        return self.info().levels

    def level_sizes(self):
        i = self.info()
        return [i.n[l] for l in range(i.levels)], [i.nnz[l] for l in range(i.levels)]

    def aggregates(self, level: int) -> np.ndarray:
        n = self.info().n[level]
        a = np.empty(n, np.int32)
        _check(lib().pamg_hierarchy_aggregates(self._h, level, a.ctypes.data_as(C.POINTER(C.c_int32))),
               "pamg_hierarchy_aggregates")
        return a

    def level_csr(self, level: int):
        i = self.info()
        n, nnz = i.n[level], i.nnz[level]
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        _check(lib().pamg_hierarchy_level_csr(self._h, level, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                              ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                              v.ctypes.data_as(C.POINTER(C.c_double))), "pamg_hierarchy_level_csr")
        return rp, ci, v

    def update_values(self, val, stream=None):
        """Coefficient-only reuse: new values of the setup matrix (same pattern,
        its CSR order), a numpy array or a float64 device tensor of nnz entries.
        Aggregates and prolongators are kept; everything else is recomputed."""
        nnz = self.info().nnz[0]
        if isinstance(val, np.ndarray):
            v = np.ascontiguousarray(val, dtype=np.float64)
            if v.shape != (nnz,):
                raise ValueError(f"expected {nnz} values")
            _check(lib().pamg_hierarchy_update_values(self._h, v.ctypes.data, 0, _stream(stream)),
                   "pamg_hierarchy_update_values")
        else:
            if tuple(val.shape) != (nnz,) or not val.is_contiguous() or str(val.dtype) != "torch.float64":
                raise ValueError(f"expected a contiguous float64 tensor of {nnz} values")
            _check(lib().pamg_hierarchy_update_values(self._h, _ptr(val), 1, _stream(stream)),
                   "pamg_hierarchy_update_values")

    def solve(self, b, x, stream=None, **kw) -> pamg_solve_info:
        """Solve A x = b for device tensors b, x (float64, n).  x is the initial
        guess when use_x0=1.  Returns the info struct; raises on errors."""
        o = solve_opts(**kw)
        info = pamg_solve_info()
        _check(lib().pamg_solve(self._h, _ptr(b), _ptr(x), C.byref(o), _stream(stream), C.byref(info)),
               "pamg_solve", allow=(OK, NOT_CONVERGED))
        return info

    def solve_noalloc(self, b, x, stream=None, **kw):
        """pamg_solve_noalloc: as solve(), with no allocation of any kind (the
        solve state and partials in the library's static per-GPU scratch,
        direct launches).  Calls on one GPU must not overlap."""
        o = solve_opts(**kw)
        info = pamg_solve_info()
        _check(lib().pamg_solve_noalloc(self._h, _ptr(b), _ptr(x), C.byref(o), _stream(stream), C.byref(info)),
               "pamg_solve_noalloc", allow=(OK, NOT_CONVERGED))
        return info

    def solve_batch(self, B, X, stream=None, **kw):
        """Solve A X = B for a (nrhs, n) float64 device tensor B (row j = right-hand
        side j, i.e. column-major n x nrhs with ld = n); X has the same shape.
        Returns the list of per-column info structs."""
        nrhs = int(B.shape[0])
        ld = int(B.shape[1])
        o = solve_opts(**kw)
        infos = (pamg_solve_info * nrhs)()
        _check(lib().pamg_solve_batch(self._h, nrhs, _ptr(B), ld, _ptr(X), int(X.shape[1]), C.byref(o),
                                      _stream(stream), infos), "pamg_solve_batch", allow=(OK, NOT_CONVERGED))
        return list(infos)

    def debug_apply_batch(self, op: int, in16, out16, precision: int = PREC_F64, stream=None):
        """Batched COARSE or VCYCLE on a (16, n_level) device tensor."""
        _check(lib().pamg_debug_apply_batch(self._h, op, precision, _ptr(in16), _ptr(out16), _stream(stream)),
               "pamg_debug_apply_batch")

    def batch_config(self, precision: int = PREC_F64):
        """Autotuned (down unroll, down cols/lane, up unroll, up cols/lane) per level."""
        L = self.levels - 1
        cfg = (C.c_int32 * (4 * max(L, 1)))()
        _check(lib().pamg_batch_config(self._h, precision, cfg), "pamg_batch_config")
        return [tuple(cfg[4 * l:4 * l + 4]) for l in range(L)]

    def set_batch_config(self, cfg, precision: int = PREC_F64):
        """Pin the multi-RHS kernel variants: cfg[l] = (down unroll, down cols/lane,
        up unroll, up cols/lane) for l = 0 .. levels-2 (level 0's up entries ignored)."""
        L = self.levels - 1
        if len(cfg) != L:
            raise ValueError(f"expected {L} levels of variants")
        arr = (C.c_int32 * (4 * max(L, 1)))(*[int(v) for t in cfg for v in t])
        _check(lib().pamg_batch_set_config(self._h, precision, arr), "pamg_batch_set_config")

    def debug_apply(self, op: int, level: int, in0, out, in1=None, precision: int = PREC_F64, stream=None):
        _check(lib().pamg_debug_apply(self._h, op, level, precision, _ptr(in0), _ptr(in1), _ptr(out),
                                      _stream(stream)), "pamg_debug_apply")

    def time_kernels(self, r, reps: int = 20, precision: int = PREC_F64, stream=None):
        vms, sms = C.c_double(), C.c_double()
        _check(lib().pamg_time_kernels(self._h, precision, _ptr(r), reps, _stream(stream), C.byref(vms),
                                       C.byref(sms)), "pamg_time_kernels")
        return vms.value, sms.value


    def time_op(self, op: int, level: int = 0, reps: int = 20, precision: int = PREC_F64, stream=None):
        """(ms per launch, algorithmic bytes per launch) of one solve kernel."""
        ms, nb = C.c_double(), C.c_uint64()
        _check(lib().pamg_time_op(self._h, op, level, precision, reps, _stream(stream), C.byref(ms), C.byref(nb)),
               "pamg_time_op")
        return ms.value, nb.value


def setup(A, **kw) -> Hierarchy:
    return Hierarchy(A, **kw)


class _HostCSR:
    """A CSR kept alive (and its pamg_csr view) while a server may read it."""

    def __init__(self, A):
        self.rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
        self.ci = np.ascontiguousarray(A.col, dtype=np.int32)
        self.v = np.ascontiguousarray(A.val, dtype=np.float64)
        self.csr = pamg_csr(int(A.n), int(self.rp[-1]), self.rp.ctypes.data_as(C.POINTER(C.c_int32)),
                            self.ci.ctypes.data_as(C.POINTER(C.c_int32)),
                            self.v.ctypes.data_as(C.POINTER(C.c_double)))


def server_estimate_bytes(A, precision: int = PREC_F32) -> int:
    """Admission charge of an uncached operator (host CSR A)."""
    hc = _HostCSR(A)
    out = C.c_uint64()
    _check(lib().pamg_server_estimate_bytes(C.byref(hc.csr), int(precision), C.byref(out)),
           "pamg_server_estimate_bytes")
    return out.value


class Server:
    """Continuous-batching solve server (pamg_server_*).  Keeps the operator
    CSRs and the device vectors of outstanding requests alive until their
    completions are polled."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, block_iters: int = 4, precision: int = PREC_F32,
                 use_graph: int = 0, single_path: int = 0, batch_from: int = 4, setup_workers: int = 1,
                 device_setup: int = 1, context=None):
        o = pamg_server_opts()
        _check(lib().pamg_server_opts_default(C.byref(o)), "pamg_server_opts_default")
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.block_iters = int(block_iters)
        o.precision = int(precision)
        o.use_graph = int(use_graph)
        o.single_path = int(single_path)
        o.batch_from = int(batch_from)
        o.setup_workers = int(setup_workers)
        o.device_setup = int(device_setup)
        h = C.c_void_p()
        self.context = context if context is not None else default_context()
        _check(lib().pamg_server_create(self.context._h, C.byref(o), C.byref(h)), "pamg_server_create")
        self._h = h
        self._ops = {}
        self._live = {}

    def submit(self, op_key: int, A, b, x, tol: float = 1e-6, tag: int = 0, maxit: int = 1000):
        """Queue a solve of A x = b (device tensors b, x).  A (a CSR) is needed the
        first time op_key is used; later requests may pass None."""
        if A is not None and op_key not in self._ops:
            self._ops[op_key] = _HostCSR(A)
        hc = self._ops.get(op_key)
        req = pamg_request(int(op_key), C.pointer(hc.csr) if hc is not None else None, _ptr(b), _ptr(x), float(tol),
                           int(maxit), 0, int(tag))
        self._live[int(tag)] = (b, x)
        _check(lib().pamg_server_submit(self._h, C.byref(req)), "pamg_server_submit")

    def poll(self, max_n: int = 256):
        out = (pamg_completion * max_n)()
        n = C.c_int32()
        _check(lib().pamg_server_poll(self._h, out, max_n, C.byref(n)), "pamg_server_poll")
        res = [out[i] for i in range(n.value)]
        for c in res:
            self._live.pop(int(c.tag), None)
        return res

    def stats(self) -> pamg_server_stats:
        s = pamg_server_stats()
        _check(lib().pamg_server_stats_get(self._h, C.byref(s)), "pamg_server_stats_get")
        return s

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.pamg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
