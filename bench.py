"""Benchmark: FCG + AMG V-cycle solve of the stretched-mesh Q1 pressure system
(256^3 elements, 16.9M dofs, 453M nonzeros, by default) to a true relative
residual of 1e-6 on one MI355X.

A step is one complete solve from x0 = 0 (every outer iteration: V-cycle
down-sweeps, coarse solve, up-sweeps, Krylov SpMV, dot products, axpys,
convergence test, and the final true-residual check), with the hierarchy and
all vectors resident in HBM.  The value is the plain FP64 form; the same line
carries the FP32-hierarchy form (its time, iterations, true residual and
error against the oracle's stored FP64 solution), the V-cycle's and the
level-0 kernels' HBM rates, and the CPU oracle's time per iteration on the
same system.  The hierarchy setup is timed separately.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]
                    [--no-cpu-baseline] [--cpu-iters I] [--cpu-deadline S]
    python bench.py --mode kernels [--reps R] [--n N] [--precision f64|f32]
                    (level-0 kernels and a plain copy only, for hardware-counter
                    runs under rocprofv3)
    python bench.py --mode batch --n 128 [--steps K]  (16 right-hand sides from
                    consecutive time steps: one batched solve vs 16 single
                    solves, FP64 and FP32 V-cycles; prints its own JSON line)
    python bench.py --mode reuse --n 128 [--steps K]  (coefficient-only update of
                    the hierarchy for a second stretching ratio on the same
                    mesh, against a fresh setup; prints its own JSON line)
    python bench.py --mode setup --n 256 [--steps K]  (hierarchy setup: the
                    device construction of the large levels, K runs, against
                    the host construction; prints its own JSON line)
    python bench.py --mode serve [--requests R] [--serve-load F]
                    [--budget-gib G] [--single-path 0|1] [--batch-from B]
                    [--setup-workers W]
                    (serving stream: variable-coefficient 7-point operators
                    from a pool of 64, a closed loop for the capacity, then
                    Poisson arrivals at F (default 0.7) x that capacity under
                    an HBM budget of G GiB (default 64); p50/p99 latency and
                    solves/s; prints its own JSON line)

Byte model of the roofline figures: plain CSR (int32 column indices and row
pointers, 8-byte values) with each owned vector entry counted once, as the
algorithmic bytes of the method; the library's own tile format moves fewer
matrix bytes (16-bit dictionary positions), reported beside it.  The
roofline "traffic" figure comes from profiles/traffic_q1_<n>.json (HBM bytes
per launch from FETCH_SIZE/WRITE_SIZE counter runs, calibrated on a plain
copy); it is reported only for the workload, precision and kernel source it
was measured on (SHA-256 of csrc/kernels.hpp), else null.

The CPU baseline runs the oracle in a child process started at once: its
hierarchy setup (minutes at 256^3) overlaps the GPU work, and its solve
phase is timed after the GPU timing, single-threaded on one pinned core and
on all cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNELS_SRC = os.path.join(ROOT, "paper_2210_16660_amd", "csrc", "kernels.hpp")


def kernels_hash() -> str:
    return hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()


def traffic_for(kernel: str, n: int, precision: str, agg_steps: int):
    """Counter-measured HBM bytes per launch of `kernel`, if measured on this
    kernel source, for this workload size, precision and aggregate size."""
    path = os.path.join(ROOT, "profiles", f"traffic_q1_{n}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    cfg = rec.get("config", {})
    if (rec.get("kernels_hpp_sha256") != kernels_hash() or cfg.get("n_elements") != n
            or cfg.get("precision") != precision or cfg.get("agg_steps") != agg_steps):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes")


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """Plain device-to-device copy (torch), GB/s counting read + write."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def csr_bytes(nnz, n, s):
    """Bytes of one pass over a CSR matrix: int32 columns, s-byte values,
    int32 row pointers (the survey's M_l)."""
    return nnz * (4 + s) + 4 * (n + 1)


def level0_csr_bytes(info, name, s=8):
    """Algorithmic bytes of one launch of a level-0 kernel, plain-CSR model:
    Krylov pass M_0 + 6 n_0 8 (z, p_old, q_old, r in; p, q out); down-sweep
    M_0 + (4 n_0 + n_1) s; up-sweep M_0 + (6 n_0 + n_1) s; SpMV M_0 + 2 n_0 8."""
    n0, n1, nnz0 = info.n[0], info.n[1] if info.levels > 1 else 0, info.nnz[0]
    if name == "krylov_spmv_l0":
        return csr_bytes(nnz0, n0, 8) + 6 * n0 * 8
    if name == "vcycle_down_l0":
        return csr_bytes(nnz0, n0, s) + (4 * n0 + n1) * s
    if name == "vcycle_up_l0":
        return csr_bytes(nnz0, n0, s) + (6 * n0 + n1) * s
    if name == "spmv_l0":
        return csr_bytes(nnz0, n0, 8) + 2 * n0 * 8
    raise KeyError(name)


def rhs_seed(n):
    """Right-hand-side seeds of the stored oracle values: 128^3 seed 2, 256^3 seed 3."""
    return {256: 3}.get(n, 2)


def load_golden(n, ratio, seed, A):
    path = os.path.join(ROOT, "tests", "golden", f"q1_{n}_fcg.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    w = g["workload"]
    if w["rhs_seed"] != seed or w["n"] != A.n or w["ratio"] != ratio:
        return None
    return g


def load_workload(args, seed, write=True):
    """The Q1 operator and its divergence right-hand side; with --cache DIR the
    generated arrays are kept there (.npy) for later runs on the same machine
    (several profiler passes in one session)."""
    import numpy as np
    from workloads import CSR, q1_rhs, q1_stretched
    if args.cache:
        stem = os.path.join(args.cache, f"q1_{args.n}_{args.ratio!r}_seed{seed}")
        names = [stem + s for s in ("_rp.npy", "_ci.npy", "_v.npy", "_b.npy")]
        if all(os.path.exists(f) for f in names):
            rp, ci, v, b = (np.load(f) for f in names)
            return CSR(len(rp) - 1, rp, ci, v), b
    A = q1_stretched(args.n, args.ratio)
    b = q1_rhs(args.n, args.ratio, seed)
    if args.cache and write:
        os.makedirs(args.cache, exist_ok=True)
        for f, arr in zip(names, (A.row_ptr, A.col, A.val, b)):
            np.save(f + ".tmp.npy", arr)
            os.replace(f + ".tmp.npy", f)
    return A, b


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline_worker(args) -> int:
    """The CPU baseline leg (a child process of the benchmark): the oracle's
    hierarchy for the same workload is built first (its setup is reported, not
    counted), then, when the parent says so on stdin (after its GPU timing),
    `cpu_iters` FCG iterations of the oracle's solve are timed three times
    single-threaded on one pinned core and three times on all cores of this
    process's affinity mask (the oracle's OpenMP timing build, bitwise the
    plain build); medians reported per iteration."""
    import ctypes

    import numpy as np

    import oracle
    oracle.use_openmp_build()
    gomp = ctypes.CDLL("libgomp.so.1")
    t0 = time.perf_counter()
    A, b = load_workload(args, rhs_seed(args.n), write=False)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    O = oracle.Hierarchy(A, agg_steps=args.agg_steps)
    t_setup = time.perf_counter() - t0
    del A
    print(json.dumps({"ready": True, "gen_s": round(t_gen, 1), "setup_s": round(t_setup, 1)}), flush=True)
    if sys.stdin.readline().strip() != "go":
        return 0
    cpus = sorted(os.sched_getaffinity(0))

    def timed(threads):
        gomp.omp_set_num_threads(threads)
        runs = []
        for _ in range(3):
            t = time.perf_counter()
            _, it, _, _ = O.solve(b, 0.0, krylov="fcg", fixed_iters=args.cpu_iters)
            runs.append(1e3 * (time.perf_counter() - t) / it)
        return sorted(runs)[1], runs

    os.sched_setaffinity(0, {cpus[0]})
    one, one_runs = timed(1)
    os.sched_setaffinity(0, set(cpus))
    # the host share of one GPU can be smaller than the mask: OMP_NUM_THREADS caps it
    threads = max(1, min(len(cpus), int(os.environ.get("OMP_NUM_THREADS", len(cpus)))))
    allc, all_runs = timed(threads)
    print(json.dumps({"single_ms_per_iter": one, "single_runs": one_runs, "all_ms_per_iter": allc,
                      "iters": args.cpu_iters,
                      "all_runs": all_runs, "threads": threads, "setup_s": round(t_setup, 1),
                      "gen_s": round(t_gen, 1), **cpu_info()}), flush=True)
    return 0


class CpuBaseline:
    """Starts the CPU baseline worker at once (its oracle setup overlaps the
    GPU work) and collects it after the GPU timing."""

    def __init__(self, args, log):
        import subprocess
        self.log = log
        self.t0 = time.perf_counter()
        cmd = [sys.executable, "-u", os.path.abspath(__file__), "--cpu-baseline-worker", "--n", str(args.n),
               "--ratio", repr(args.ratio), "--agg-steps", str(args.agg_steps), "--cpu-iters", str(args.cpu_iters)]
        if args.cache:
            cmd += ["--cache", args.cache]
        self.p = subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
        self.deadline = args.cpu_deadline

    def _readline(self, until):
        import select
        while True:
            left = until - time.perf_counter()
            if left <= 0:
                return None
            r, _, _ = select.select([self.p.stdout], [], [], min(left, 30.0))
            if r:
                return self.p.stdout.readline()
            self.log(f"waiting for the CPU baseline worker ({time.perf_counter() - self.t0:.0f} s)")

    def collect(self, gpu_iters, gpu_ms_per_iter):
        until = self.t0 + self.deadline
        line = self._readline(until)
        if not line:
            self.p.kill()
            self.p.wait()
            self.log("CPU baseline worker did not finish its setup within the time budget")
            return None
        ready = json.loads(line)
        self.log(f"oracle setup {ready['setup_s']} s; timing the oracle's solve")
        self.p.stdin.write("go\n")
        self.p.stdin.flush()
        line = self._readline(time.perf_counter() + 600)
        self.p.wait()
        if not line:
            return None
        r = json.loads(line)
        return {
            "value": round(r["single_ms_per_iter"], 1),
            "unit": "ms per FCG iteration",
            "cores": 1,
            "kind": "oracle",
            "sample": f"3 timed runs of the oracle's FCG solve phase, {r['iters']} iterations each, on the "
                      f"same operator and right-hand side (median per "
                      f"iteration; its hierarchy setup of {r['setup_s']} s is not counted), single-threaded and "
                      f"pinned to one core",
            "all_cores": {"value": round(r["all_ms_per_iter"], 1), "unit": "ms per FCG iteration",
                          "threads": r["threads"], "build": "the oracle's OpenMP timing build (row and element loops "
                                                            "over threads, reductions serial; bitwise the plain build)"},
            "runs_ms_per_iter": {"single": [round(v, 1) for v in r["single_runs"]],
                                 "all_cores": [round(v, 1) for v in r["all_runs"]]},
            "gpu_ms_per_iter": round(gpu_ms_per_iter, 3),
            "single_vs_gpu": round(r["single_ms_per_iter"] / gpu_ms_per_iter, 1),
            "oracle_setup_s": r["setup_s"],
            "per_solve_ms_scaled": round(r["single_ms_per_iter"] * gpu_iters, 1),
            "per_solve_note": f"per-iteration median x the {gpu_iters} iterations of the GPU solve (an estimate, "
                              f"not a timed full solve)",
            "nproc": r["nproc"], "affinity_cpus": r["affinity_cpus"], "cpu_model": r["cpu_model"],
        }



def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="Q1 mesh elements per direction")
    ap.add_argument("--ratio", type=float, default=1.05)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"],
                    help="batch/reuse modes: V-cycle precision (the solve mode times both)")
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations per timed CPU baseline run")
    ap.add_argument("--cpu-deadline", type=float, default=420.0,
                    help="seconds from the start by which the CPU baseline's oracle setup must be done")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--mode", default="solve", choices=["solve", "kernels", "batch", "serve", "reuse", "setup"])
    ap.add_argument("--device-setup", type=int, default=1, choices=[0, 1],
                    help="build the large levels of the hierarchy on the device (bitwise the host build)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="serving: open-loop arrival rate as a fraction of the closed-loop capacity")
    ap.add_argument("--single-path", type=int, default=1, choices=[0, 1],
                    help="serving: a request alone on its operator runs on the single-right-hand-side solver")
    ap.add_argument("--batch-from", type=int, default=4,
                    help="serving: waiting requests of one operator from which they are batched")
    ap.add_argument("--setup-workers", type=int, default=4,
                    help="serving: host phases of new operators built at once")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--cache", default="", help="directory that keeps the generated workload between runs")
    ap.add_argument("--agg-steps", type=int, default=1,
                    help="aggregate-size composition: keep every n-th pairwise level (aggregates up to 2^n)")
    ap.add_argument("--smoother", default="l1", choices=["l1", "hgs"],
                    help="l1-Jacobi 1+1, or hybrid forward/backward Gauss-Seidel")
    ap.add_argument("--sweeps", type=int, default=0, help="hybrid GS sweeps per side (0: 4)")
    ap.add_argument("--gs-block", type=int, default=0, help="hybrid GS block size (0: 256)")
    ap.add_argument("--omega", type=float, default=0.0, help="hybrid GS damping (0: 1.5)")
    ap.add_argument("--smooth-prolongator", action="store_true",
                    help="smoothed prolongators P = (I - w D^-1 A) P^ (moderate sizes: coarse levels fill in)")
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        return cpu_baseline_worker(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not supported "
                                   "(the row-block sharding design is described in DESIGN.md)",
                          "n_gpus": args.gpus}))
        return 2

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    cpu = None
    if args.mode == "solve" and not args.no_cpu_baseline:
        cpu = CpuBaseline(args, log)

    import numpy as np
    import torch

    import paper_2210_16660_amd as pamg

    if args.mode == "serve":
        return bench_serve(args, torch, np, pamg, log)
    t0 = time.perf_counter()
    seed = rhs_seed(args.n)
    A, b = load_workload(args, seed)
    log(f"generated Q1 {args.n}^3: n={A.n} nnz={A.nnz}, right-hand side seed {seed}, "
        f"in {time.perf_counter() - t0:.1f}s")
    if args.mode == "batch":
        return bench_batch(args, A, torch, np, pamg, log)
    if args.mode == "reuse":
        return bench_reuse(args, A, b, torch, np, pamg, log)
    if args.mode == "setup":
        return bench_setup(args, A, torch, pamg, log)
    dev = torch.device("cuda:0")

    t0 = time.perf_counter()
    smooth_kw = {} if args.smoother == "l1" else dict(smoother="hgs", sweeps=args.sweeps, gs_block=args.gs_block,
                                                      omega=args.omega)
    if args.smooth_prolongator:
        smooth_kw["smooth_prolongator"] = 1
    H = pamg.Hierarchy(A, build_f32=1, agg_steps=args.agg_steps, device_setup=args.device_setup, **smooth_kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = H.info()
    log(f"setup {setup_s:.2f}s ({info.device_levels} levels built on the device), {info.levels} levels, "
        f"operator complexity {info.operator_complexity:.3f}")

    b_d = torch.from_numpy(b).to(dev)
    x_d = torch.zeros(A.n, dtype=torch.float64, device=dev)

    if args.mode == "kernels":
        # one warm solve fills every work vector with real data, then each
        # level-0 kernel and a plain copy are launched back to back
        prec = pamg.PREC_F32 if args.precision == "f32" else pamg.PREC_F64
        H.solve(b_d, x_d, tol=args.tol, precision=prec)
        out = {}
        for name, op in (("vcycle_down_l0", pamg.OP_DOWN), ("vcycle_up_l0", pamg.OP_UP),
                         ("krylov_spmv_l0", pamg.OP_KRYLOV)):
            ms, nb = H.time_op(op, 0, reps=args.reps, precision=pamg.PREC_F64 if op == pamg.OP_KRYLOV else prec)
            out[name] = {"ms": ms, "bytes": nb, "GBps": nb / (ms * 1e-3) / 1e9}
        gbs, cms = copy_bandwidth(torch, reps=args.reps)
        out["copy_2GiB"] = {"ms": cms, "bytes": 2 * (1 << 31), "GBps": gbs}
        print(json.dumps(out), flush=True)
        return 0

    golden = load_golden(args.n, args.ratio, seed, A) if args.agg_steps == 1 and args.smoother == "l1" \
        and not args.smooth_prolongator else None
    S = A.to_scipy()
    bn = float(np.linalg.norm(b))
    res = {}
    for name, prec, steps, warm in (("f64", pamg.PREC_F64, args.steps, args.warmup),
                                    ("f32", pamg.PREC_F32, max(1, args.steps // 2), max(1, args.warmup // 2))):
        opts = dict(tol=args.tol, krylov="fcg", precision=prec, true_residual=1)
        for k in range(warm):
            x_d.zero_()
            t1 = time.perf_counter()
            inf = H.solve(b_d, x_d, **opts)
            log(f"{name} warm-up solve {k}: {1e3 * (time.perf_counter() - t1):.1f} ms, {inf.iterations} iterations")
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            x_d.zero_()
            inf = H.solve(b_d, x_d, **opts)
            if inf.status != pamg.OK:
                log(f"{name} solve status {inf.status}")
                return 1
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t_start) / steps
        x = x_d.cpu().numpy()
        rel = float(np.linalg.norm(b - S @ x) / bn)
        entry = {"ms_per_solve": round(ms, 4), "steps": steps, "iterations": inf.iterations,
                 "restarts": inf.restarts, "relres_true": rel}
        if golden is not None:
            idx = np.array(golden["sample_index"])
            xo = np.array(golden["x_sample"])
            entry["err_vs_oracle_sample"] = float(np.linalg.norm(x[idx] - xo) / np.linalg.norm(xo))
            entry["oracle_iterations"] = golden["fcg_iterations"]
        res[name] = entry
        res[name + "_x"] = x
        log(f"{name}: {ms:.2f} ms/solve, {inf.iterations} iterations, true relres {rel:.3e}"
            + (f", sampled error vs oracle {entry['err_vs_oracle_sample']:.2e}" if golden is not None else ""))
        if rel > args.tol:
            print(json.dumps({"error": f"{name} solve did not reach the tolerance", **entry}), flush=True)
            return 1
    err32 = float(np.linalg.norm(res["f32_x"] - res["f64_x"]) / np.linalg.norm(res["f64_x"]))
    ms_per_step = res["f64"]["ms_per_solve"]
    iters = res["f64"]["iterations"]

    # V-cycle and SpMV throughput (back-to-back, HIP events on this stream)
    r_d = b_d.clone()
    plain = args.smoother == "l1" and not args.smooth_prolongator
    vc = {}
    for name, prec in (("f64", pamg.PREC_F64), ("f32", pamg.PREC_F32)):
        v_ms, s_ms = H.time_kernels(r_d, reps=20, precision=prec)
        csr_b = info.csr_vcycle_bytes_f64 if prec == pamg.PREC_F64 else info.csr_vcycle_bytes_f32
        tile_b = info.vcycle_bytes_f64 if prec == pamg.PREC_F64 else info.vcycle_bytes_f32
        vc[name] = {"ms": v_ms, "GBps": csr_b / (v_ms * 1e-3) / 1e9 if plain else float("nan"),
                    "GBps_tile_format": tile_b / (v_ms * 1e-3) / 1e9 if plain else float("nan"), "spmv_ms": s_ms}
    s_ms = vc["f64"]["spmv_ms"]
    s_gbs = level0_csr_bytes(info, "spmv_l0") / (s_ms * 1e-3) / 1e9

    # the kernels that stream the level-0 matrix, each timed live with HIP events
    kern = {}
    if args.smooth_prolongator:
        level0_ops = (("krylov_spmv_l0", pamg.OP_KRYLOV),)
    else:
        level0_ops = ((("vcycle_down_l0", pamg.OP_DOWN), ("vcycle_up_l0", pamg.OP_UP)) if args.smoother == "l1"
                      else (("hgs_sweep_l0", pamg.OP_SMOOTH),)) + (("krylov_spmv_l0", pamg.OP_KRYLOV),)
    for name, op in level0_ops:
        ms, nb = H.time_op(op, 0, reps=20, precision=pamg.PREC_F64)
        k = {"ms": ms, "bytes_tile_format": nb, "GBps_tile_format": nb / (ms * 1e-3) / 1e9}
        if name != "hgs_sweep_l0":
            k["bytes"] = level0_csr_bytes(info, name)
            k["GBps"] = k["bytes"] / (ms * 1e-3) / 1e9
        kern[name] = k
    dom = max(kern, key=lambda k: kern[k]["ms"])
    dk = kern[dom]
    copy_gbs, _ = copy_bandwidth(torch)
    traffic = traffic_for(dom, args.n, "f64", args.agg_steps) if plain else None
    log(f"V-cycle {vc['f64']['ms']:.3f} ms ({vc['f64']['GBps']:.0f} GB/s), FP32 V-cycle {vc['f32']['ms']:.3f} ms; "
        f"SpMV {s_ms:.3f} ms ({s_gbs:.0f} GB/s); "
        + ", ".join(f"{k} {v['ms']:.4f} ms {v.get('GBps', float('nan')):.0f} GB/s" for k, v in kern.items()))
    achieved = dk.get("GBps", dk["GBps_tile_format"])

    def r1(v):
        return round(v, 1) if v == v else None

    result = {
        "metric": "PCG-AMG solve time to 1e-6 rel. residual + V-cycle HBM GB/s (% of peak)",
        "value": round(ms_per_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"Q1 hexahedral FE Laplacian, {args.n}^3 elements, vertical stretching {args.ratio}, "
                        f"divergence right-hand side seed {seed}; FCG + AMG V-cycle (pairwise matching aggregation"
                        + (f", aggregates of up to {2 ** args.agg_steps}" if args.agg_steps > 1 else "")
                        + (", smoothed prolongators, " if args.smooth_prolongator else ", ")
                        + ("l1-Jacobi 1+1" if args.smoother == "l1" else
                           f"hybrid forward/backward Gauss-Seidel {H.params.sweeps or 4}+{H.params.sweeps or 4} "
                           f"(blocks of {H.params.gs_block or 256}, omega {H.params.omega or 1.5:g})")
                        + f", dense coarse solve) to a true relative residual of {args.tol:g}; value: the plain "
                          f"FP64 form; the FP32-hierarchy form in 'mixed_precision'",
            "n": A.n, "nnz": A.nnz, "levels": info.levels,
            "operator_complexity": round(info.operator_complexity, 4),
            "aggregate_steps": args.agg_steps,
            "smoother": args.smoother,
            "smoothed_prolongator": bool(args.smooth_prolongator),
        },
        "iterations": iters,
        "relres_true": res["f64"]["relres_true"],
        "err_vs_oracle_sample": res["f64"].get("err_vs_oracle_sample"),
        "oracle_iterations": res["f64"].get("oracle_iterations"),
        "mixed_precision": {**res["f32"], "speedup_vs_f64": round(ms_per_step / res["f32"]["ms_per_solve"], 3),
                            "solution_relerr_vs_f64": err32, "vcycle_ms": round(vc["f32"]["ms"], 4),
                            "vcycle_GBps": r1(vc["f32"]["GBps"])},
        "setup_s": round(setup_s, 3),
        "setup_device_levels": info.device_levels,
        "vcycle_ms": round(vc["f64"]["ms"], 4),
        "vcycle_GBps": r1(vc["f64"]["GBps"]),
        "vcycle_pct_peak": round(100 * vc["f64"]["GBps"] / HBM_PEAK_GBS, 2) if plain else None,
        "vcycle_GBps_tile_format": r1(vc["f64"]["GBps_tile_format"]),
        "spmv_ms": round(s_ms, 4),
        "spmv_GBps": round(s_gbs, 1),
        "spmv_pct_peak": round(100 * s_gbs / HBM_PEAK_GBS, 2),
        "byte_model": "plain CSR (int32 columns and row pointers, 8-byte values) with each owned vector entry "
                      "counted once; *_tile_format: the library's tile format (16-bit dictionary positions)",
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "copy_GBps": round(copy_gbs, 1),
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
    }
    if cpu is not None:
        cb = cpu.collect(iters, ms_per_step / iters)
        result["cpu_baseline"] = cb if cb is not None else {
            "value": None, "unit": "ms per FCG iteration", "cores": 1, "kind": "oracle",
            "sample": f"not measured: the oracle's setup did not finish within {args.cpu_deadline:g} s"}
    print(json.dumps(result), flush=True)
    return 0


def bench_batch(args, A, torch, np, pamg, log) -> int:
    """16 right-hand sides (a base divergence field plus successive 5%
    perturbations, seed 4) solved as one batch versus one at a time."""
    from workloads import q1_rhs_sequence
    t0 = time.perf_counter()
    Bm = q1_rhs_sequence(args.n, args.ratio, 4, 16).T.copy()        # (16, n)
    log(f"16 right-hand sides in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    H = pamg.Hierarchy(A, build_f32=1, device_setup=args.device_setup)
    B = torch.from_numpy(Bm).to(dev)
    X = torch.zeros_like(B)
    S = A.to_scipy()

    def run_batch(prec):
        X.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = H.solve_batch(B, X, tol=args.tol, precision=prec)
        torch.cuda.synchronize()
        return time.perf_counter() - t, infos

    def run_single(prec):
        x = torch.zeros(A.n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = []
        for j in range(16):
            x.zero_()
            its.append(H.solve(B[j], x, tol=args.tol, precision=prec).iterations)
        torch.cuda.synchronize()
        return time.perf_counter() - t, its

    info = H.info()
    L = info.levels - 1

    def batch_iter_bytes(s):
        """Algorithmic bytes of one 16-column iteration: per level l < L two
        passes over the matrix (int32 columns) and the n x 16 vectors, the
        coarse GEMM, and the FP64 Krylov step at level 0."""
        B = 0
        for l in range(L):
            n, nc, nnz = info.n[l], info.n[l + 1], info.nnz[l]
            B += 2 * (nnz * (4 + s) + 4 * (n + 1)) + (10 * n + 2 * nc) * 16 * s
        nL = info.n[L]
        B += nL * nL * s + 2 * nL * 16 * s
        B += info.nnz[0] * 12 + 4 * (info.n[0] + 1) + 12 * info.n[0] * 16 * 8
        return B

    res = {}
    for name, prec in (("f64", pamg.PREC_F64), ("f32", pamg.PREC_F32)):
        run_batch(prec)                      # first call builds the engine and runs the autotuner
        run_single(prec)
        tb = min(run_batch(prec)[0] for _ in range(max(1, args.steps // 4)))
        _, infos = run_batch(prec)
        Xh = X.cpu().numpy()
        rel = max(float(np.linalg.norm(Bm[j] - S @ Xh[j]) / np.linalg.norm(Bm[j])) for j in range(16))
        ts, its = min((run_single(prec) for _ in range(max(1, args.steps // 8))), key=lambda r: r[0])
        res[name] = {"batch_ms": round(1e3 * tb, 3), "single16_ms": round(1e3 * ts, 3),
                     "batch_solves_per_s": round(16 / tb, 2), "single_solves_per_s": round(16 / ts, 2),
                     "batch_iterations": [i.iterations for i in infos], "single_iterations": its,
                     "max_true_relres": rel,
                     "batch_GBps": round(batch_iter_bytes(8 if name == "f64" else 4)
                                         * max(i.iterations for i in infos) / tb / 1e9, 1)}
        log(f"{name}: batch {1e3 * tb:.1f} ms, 16 singles {1e3 * ts:.1f} ms, max true relres {rel:.2e}")
    cfg = H.batch_config(pamg.PREC_F32)
    cfg64 = H.batch_config(pamg.PREC_F64)
    out = {
        "metric": "16-RHS batched FCG+AMG solve time to 1e-6 (solves/s)",
        "value": res["f32"]["batch_solves_per_s"],
        "unit": "solves/s",
        "higher_is_better": True,
        "config": {"workload": f"Q1 {args.n}^3 stretched, 16 RHS: base divergence field (seed 4) + 15 "
                               f"successive 5% perturbations; batched FCG, FP32 V-cycle / FP64 outer",
                   "n": A.n, "nnz": A.nnz},
        "f64": res["f64"], "f32": res["f32"],
        "speedup_batch_f32_vs_16_single_f64": round(res["f64"]["single16_ms"] / res["f32"]["batch_ms"], 3),
        "speedup_batch_f32_vs_16_single_f32": round(res["f32"]["single16_ms"] / res["f32"]["batch_ms"], 3),
        "speedup_batch_f64_vs_16_single_f64": round(res["f64"]["single16_ms"] / res["f64"]["batch_ms"], 3),
        "autotuned_f32": cfg, "autotuned_f64": cfg64,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_setup(args, A, torch, pamg, log) -> int:
    """Hierarchy setup time (FP64 and FP32 copies, as the solve benchmark
    builds it): the device construction of the large levels against the host
    construction, and a check that both give the same hierarchy."""
    import numpy as np

    def build(dev_setup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = pamg.Hierarchy(A, build_f32=1, device_setup=dev_setup, agg_steps=args.agg_steps)
        torch.cuda.synchronize()
        return H, time.perf_counter() - t0

    runs = []
    for r in range(args.steps):
        H, t = build(1)
        runs.append(t)
        log(f"device setup {r}: {t:.2f} s, {H.info().device_levels} device levels of {H.info().levels}")
        if r + 1 < args.steps:
            H.close()
            del H
    Hh, th = build(0)
    log(f"host setup: {th:.2f} s")
    i, ih = H.info(), Hh.info()
    same = i.levels == ih.levels and all(i.n[l] == ih.n[l] and i.nnz[l] == ih.nnz[l] for l in range(i.levels))
    probe = [0, min(3, i.levels - 2)]
    for l in probe:
        same = same and np.array_equal(H.aggregates(l), Hh.aggregates(l))
    out = {"metric": "hierarchy setup time (s)", "value": round(min(runs), 3), "unit": "s", "higher_is_better": False,
           "config": {"workload": f"Q1 {args.n}^3 stretched (ratio {args.ratio}), "
                                  + ("pairwise aggregation" if args.agg_steps == 1 else
                                     f"aggregates of up to {2 ** args.agg_steps} (composed pairwise)")
                                  + ", FP64 + FP32 hierarchy copies", "n": A.n, "nnz": A.nnz, "levels": i.levels},
           "device_setup_s": [round(t, 3) for t in runs], "device_levels": i.device_levels,
           "host_setup_s": round(th, 3), "speedup_vs_host": round(th / min(runs), 2),
           "same_hierarchy_sampled": bool(same)}
    print(json.dumps(out), flush=True)
    return 0 if same else 1


def bench_reuse(args, A, b, torch, np, pamg, log) -> int:
    """Coefficient-only reuse: the hierarchy of the 1.05-stretched mesh is
    updated to the values of the 1.06-stretched mesh (same pattern) on the
    device, versus a fresh setup of that matrix."""
    from workloads import q1_rhs, q1_stretched
    r2 = args.ratio + 0.01
    A2 = q1_stretched(args.n, r2)
    assert np.array_equal(A2.row_ptr, A.row_ptr) and np.array_equal(A2.col, A.col)
    b2 = torch.from_numpy(q1_rhs(args.n, r2, 2)).cuda()
    dev = torch.device("cuda:0")
    v1 = torch.from_numpy(A.val).to(dev)
    v2 = torch.from_numpy(A2.val).to(dev)
    t0 = time.perf_counter()
    H = pamg.Hierarchy(A, agg_steps=args.agg_steps)
    torch.cuda.synchronize()
    setup1_s = time.perf_counter() - t0
    info = H.info()
    t0 = time.perf_counter()
    H.update_values(v2)                       # first update also builds the summation plans
    first_ms = 1e3 * (time.perf_counter() - t0)
    log(f"setup {setup1_s:.2f}s; first update (plans) {first_ms:.1f} ms")
    times = []
    for k in range(max(2, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.update_values(v1 if k % 2 == 0 else v2)
        times.append(1e3 * (time.perf_counter() - t0))
    if max(2, args.steps) % 2 == 1:
        H.update_values(v2)
    t0 = time.perf_counter()
    H.update_values(A2.val)                   # host values: includes the PCIe copy
    host_ms = 1e3 * (time.perf_counter() - t0)
    upd_ms = sorted(times)[len(times) // 2]
    x = torch.zeros(A.n, dtype=torch.float64, device=dev)
    H.solve(b2, x, tol=args.tol)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inf_u = H.solve(b2, x, tol=args.tol)
    torch.cuda.synchronize()
    solve_u_ms = 1e3 * (time.perf_counter() - t0)
    xs = x.cpu().numpy()
    bh = b2.cpu().numpy()
    rel_u = float(np.linalg.norm(bh - A2.to_scipy() @ xs) / np.linalg.norm(bh))
    t0 = time.perf_counter()
    F = pamg.Hierarchy(A2, agg_steps=args.agg_steps)
    torch.cuda.synchronize()
    setup2_s = time.perf_counter() - t0
    x.zero_()
    F.solve(b2, x, tol=args.tol)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inf_f = F.solve(b2, x, tol=args.tol)
    torch.cuda.synchronize()
    solve_f_ms = 1e3 * (time.perf_counter() - t0)
    # algorithmic bytes of one update from device values (pairwise levels)
    L = info.levels - 1
    n = [info.n[l] for l in range(L + 1)]
    z = [info.nnz[l] for l in range(L + 1)]
    by = 16 * z[0] + 8 * z[0] + 12 * n[0]                           # copy in, validity check
    for m in range(L):
        by += 4 * (z[m + 1] + 1) + 20 * z[m] + 8 * z[m + 1]          # plan, fine values, coarse values
    for l in range(L + 1):
        by += 4 * (n[l] + 1) + 8 * z[l] + 8 * n[l]                   # l1 diagonal
        by += 20 * z[l] + 20 * n[l]                                  # device-order values and diagonal
        if l < L:
            by += 20 * z[l] + 8 * n[l]                               # column-scaled values
    log(f"update {upd_ms:.2f} ms (device values), {host_ms:.1f} ms (host values); fresh setup {setup2_s:.2f}s; "
        f"iterations {inf_u.iterations} (updated) vs {inf_f.iterations} (fresh)")
    out = {
        "metric": "coefficient-only hierarchy update time (values already in HBM)",
        "value": round(upd_ms, 3), "unit": "ms", "higher_is_better": False,
        "config": {"workload": f"Q1 {args.n}^3 stretched: hierarchy of ratio {args.ratio} updated to the "
                               f"values of ratio {r2} (same mesh pattern); FCG + AMG to {args.tol}",
                   "n": A.n, "nnz": A.nnz, "levels": info.levels, "aggregate_steps": args.agg_steps},
        "update_ms_median": round(upd_ms, 3), "update_ms_all": [round(t, 3) for t in times],
        "first_update_ms_with_plans": round(first_ms, 1), "update_host_values_ms": round(host_ms, 1),
        "fresh_setup_s": round(setup2_s, 3), "speedup_vs_fresh_setup": round(1e3 * setup2_s / upd_ms, 1),
        "update_algorithmic_bytes": by, "update_GBps": round(by / (upd_ms * 1e-3) / 1e9, 1),
        "iterations_updated": inf_u.iterations, "iterations_fresh": inf_f.iterations,
        "solve_ms_updated": round(solve_u_ms, 2), "solve_ms_fresh": round(solve_f_ms, 2),
        "true_relres_updated": rel_u,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args, torch, np, pamg, log) -> int:
    """Serving stream: a pool of variable-coefficient 7-point operators
    -div(k grad p) on n^3 grids, n = floor(24 (161/24)^u) capped at 160
    (log-uniform), k = exp(N(0,1)) per cell; each request picks an operator
    uniformly and carries a U[-1,1] right-hand side; Poisson arrivals."""
    import threading
    from workloads import SplitMix64, varcoef7
    rng = SplitMix64(5)
    sizes = [min(160, int(np.floor(24 * (161 / 24) ** u))) for u in rng.uniform01(args.pool)]
    t0 = time.perf_counter()
    ops = [varcoef7(n, seed=5000 + k) for k, n in enumerate(sizes)]
    picks = rng.integers(args.requests, 0, args.pool - 1)
    log(f"{args.pool} operators (n^3, n in [{min(sizes)}, {max(sizes)}], {sum(A.n for A in ops)} dofs) "
        f"in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    # right-hand sides, generated up front and kept on the device
    t0 = time.perf_counter()
    rhs = [torch.from_numpy(SplitMix64(50000 + t).uniform(ops[int(picks[t])].n)).to(dev) for t in range(args.requests)]
    torch.cuda.current_stream().synchronize()
    log(f"{args.requests} right-hand sides in {time.perf_counter() - t0:.1f}s")
    budget = int(args.budget_gib * (1 << 30))
    S = pamg.Server(hbm_budget_bytes=budget, block_iters=4, precision=pamg.PREC_F32, use_graph=1,
                    single_path=args.single_path, batch_from=args.batch_from,
                    setup_workers=args.setup_workers)

    def wait_for(count, what):
        comps = []
        last_report = time.perf_counter()
        last_progress = (time.perf_counter(), 0)
        while len(comps) < count:
            comps.extend(S.poll())
            now = time.perf_counter()
            if len(comps) != last_progress[1]:
                last_progress = (now, len(comps))
            elif now - last_progress[0] > 300:
                raise RuntimeError(f"{what}: no progress for 300 s")
            if now - last_report > 10:
                st = S.stats()
                log(f"  {what}: {len(comps)}/{count} done, {st.active_columns} running, {st.pending} waiting, "
                    f"{st.cached_operators} cached, {st.setups} setups, {st.evictions} evictions")
                last_report = now
            time.sleep(0.0005)
        return comps

    # warm-up: one zero right-hand side per operator builds and caches every
    # hierarchy (setup happens once per operator, Sec. 2); not timed below
    t0 = time.perf_counter()
    zeros = {}
    for k in range(args.pool):
        zeros[k] = (torch.zeros(ops[k].n, dtype=torch.float64, device=dev),
                    torch.zeros(ops[k].n, dtype=torch.float64, device=dev))
    torch.cuda.current_stream().synchronize()
    for k in range(args.pool):
        S.submit(k, ops[k], zeros[k][0], zeros[k][1], tol=1e-6, tag=1 << 40 | k)
    wait_for(args.pool, "warm-up")
    warm = S.stats()
    warm_s = time.perf_counter() - t0
    log(f"warm-up: {warm.setups} operators set up in {warm_s:.1f}s (host phases {warm.host_setup_ms / 1e3:.1f}s, "
        f"uploads + coarsest factorizations {warm.device_setup_ms / 1e3:.1f}s), "
        f"{warm.bytes_in_use / 2**30:.2f} GiB cached")
    del zeros

    def run(first, count, arrivals):
        """Requests first .. first+count-1 (arrivals: offsets in s, or None = all at once)."""
        xs = [torch.zeros(ops[int(picks[t])].n, dtype=torch.float64, device=dev) for t in range(first, first + count)]
        torch.cuda.current_stream().synchronize()
        res = {}

        def poller():
            res["comps"] = wait_for(count, "closed loop" if arrivals is None else "open loop")

        th = threading.Thread(target=poller)
        th.start()
        t_start = time.perf_counter()
        for q in range(count):
            t = first + q
            if arrivals is not None:
                wait = t_start + arrivals[q] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            k = int(picks[t])
            S.submit(k, None, rhs[t], xs[q], tol=1e-6, tag=t)
        th.join()
        if "comps" not in res:
            raise RuntimeError("serving stalled")
        return res["comps"], time.perf_counter() - t_start

    # closed loop: a batch of requests queued at once -> capacity
    ncl = min(args.requests // 4, 500)
    comps, wall = run(0, ncl, None)
    capacity = ncl / wall
    log(f"closed loop: {ncl} requests in {wall:.2f}s -> {capacity:.1f} solves/s")
    # open loop: Poisson arrivals at half the capacity over the remaining requests
    lam = args.serve_load * capacity
    nol = args.requests - ncl
    arrivals = np.cumsum(SplitMix64(55).exponential(nol, lam))
    st1 = S.stats()
    comps, wall = run(ncl, nol, arrivals)
    st = S.stats()
    S.close()
    lat = np.array([c.latency_ms for c in comps])
    ok = sum(1 for c in comps if c.status == pamg.OK)
    its = np.array([c.iterations for c in comps])
    worst = max(c.relres_true for c in comps)
    out = {
        "metric": "serving: p50/p99 latency and solves/s at 1e-6",
        "value": round(capacity, 2),
        "unit": "solves/s",
        "higher_is_better": True,
        "config": {"workload": f"{args.requests} requests ({ncl} queued at once for the capacity, then {nol} "
                               f"with Poisson arrivals at lambda = {args.serve_load:g} x capacity) after a warm-up that caches every "
                               f"operator's hierarchy; "
                               f"variable-coefficient 7-point operators (pool of {args.pool}, n^3 with n log-uniform "
                               f"in [24, 160], lognormal sigma=1 cell coefficients); U[-1,1] right-hand sides; "
                               f"FP32 V-cycle / FP64 FCG, accepted on the true residual",
                   "hbm_budget_gib": args.budget_gib, "block_iters": 4, "single_path": args.single_path,
                   "batch_from": args.batch_from, "setup_workers": args.setup_workers},
        "lambda_per_s": round(lam, 2),
        "closed_loop_capacity_per_s": round(capacity, 2),
        "open_loop_rate_per_s": round(len(comps) / wall, 2),
        "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
        "mean_latency_ms": round(float(lat.mean()), 3),
        "completed_ok": ok,
        "iterations_median": int(np.median(its)),
        "max_true_relres": worst,
        "setups": st.setups, "evictions": st.evictions, "rejected": st.rejected,
        "aggregate_GBps": round((st.algorithmic_bytes - st1.algorithmic_bytes) / wall / 1e9, 1),
        "wall_s": round(wall, 2),
        "warmup": {"operators": int(warm.setups), "wall_s": round(warm_s, 2),
                   "host_setup_s": round(warm.host_setup_ms / 1e3, 2),
                   "device_setup_s": round(warm.device_setup_ms / 1e3, 2),
                   "cached_GiB": round(warm.bytes_in_use / 2**30, 2)},
    }
    print(json.dumps(out), flush=True)
    return 0 if ok == len(comps) else 1


if __name__ == "__main__":
    sys.exit(main())
