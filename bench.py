"""Benchmark: FCG + AMG V-cycle solve of the 128^3 stretched-mesh Q1 pressure
system to a 1e-6 relative residual on one MI355X.

A step is one complete solve from x0 = 0 (every outer iteration: V-cycle
down-sweeps, coarse solve, up-sweeps, Krylov SpMV, dot products, axpys,
convergence test), with the hierarchy and all vectors resident in HBM.  The
hierarchy setup is timed separately.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 128]
                    [--precision f64|f32] [--no-cpu-baseline]
    python bench.py --mode kernels [--reps R]   (level-0 kernels and a plain
                    copy only, for hardware-counter runs under rocprofv3)
    python bench.py --mode batch [--steps K]    (16 right-hand sides from
                    consecutive time steps: one batched solve vs 16 single
                    solves, FP64 and FP32 V-cycles; prints its own JSON line)
    python bench.py --mode reuse [--steps K]    (coefficient-only update of the
                    hierarchy for a second stretching ratio on the same mesh,
                    against a fresh setup; prints its own JSON line)
    python bench.py --mode serve [--requests R] [--serve-load F]
                    [--single-path 0|1] [--batch-from B] [--setup-workers W]
                    (serving stream: variable-coefficient 7-point operators
                    from a pool of 64, a closed loop for the capacity, then
                    Poisson arrivals at F (default 0.5) x that capacity;
                    p50/p99 latency and solves/s; prints its own JSON line)

The roofline "traffic" figure comes from profiles/traffic_q1_128.json (HBM
bytes per launch from FETCH_SIZE/WRITE_SIZE counter runs, calibrated on a
plain copy); it is reported only while the kernel source it was measured on
is unchanged (SHA-256 of csrc/kernels.hpp), else null.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_q1_128.json")


def kernels_hash() -> str:
    return hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()


def traffic_for(kernel: str, measured_config: bool = True):
    """Counter-measured HBM bytes per launch of `kernel`, if measured on this
    source and this configuration (FP64 V-cycle, pairwise levels)."""
    if not measured_config:
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hpp_sha256") != kernels_hash():
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="Q1 mesh elements per direction")
    ap.add_argument("--ratio", type=float, default=1.05)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle iterations timed for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="solve", choices=["solve", "kernels", "batch", "serve", "mixed", "reuse"])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="serving: open-loop arrival rate as a fraction of the closed-loop capacity")
    ap.add_argument("--single-path", type=int, default=1, choices=[0, 1],
                    help="serving: a request alone on its operator runs on the single-right-hand-side solver")
    ap.add_argument("--batch-from", type=int, default=4,
                    help="serving: waiting requests of one operator from which they are batched")
    ap.add_argument("--setup-workers", type=int, default=4,
                    help="serving: host phases of new operators built at once")
    ap.add_argument("--reps", type=int, default=20)
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

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not supported "
                                   "(the row-block sharding design is described in DESIGN.md)",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_2210_16660_amd as pamg
    from workloads import q1_rhs, q1_rhs_sequence, q1_stretched

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.mode == "serve":
        return bench_serve(args, torch, np, pamg, log)
    if args.mode == "mixed":
        return bench_mixed(args, torch, np, pamg, log)
    t0 = time.perf_counter()
    A = q1_stretched(args.n, args.ratio)
    b = q1_rhs(args.n, args.ratio, 2)
    log(f"generated Q1 {args.n}^3: n={A.n} nnz={A.nnz} in {time.perf_counter() - t0:.1f}s")
    prec = pamg.PREC_F32 if args.precision == "f32" else pamg.PREC_F64
    if args.mode == "batch":
        return bench_batch(args, A, torch, np, pamg, log)
    if args.mode == "reuse":
        return bench_reuse(args, A, b, torch, np, pamg, log)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    smooth_kw = {} if args.smoother == "l1" else dict(smoother="hgs", sweeps=args.sweeps, gs_block=args.gs_block,
                                                      omega=args.omega)
    if args.smooth_prolongator:
        smooth_kw["smooth_prolongator"] = 1
    H = pamg.Hierarchy(A, build_f32=1 if prec == pamg.PREC_F32 else 0, agg_steps=args.agg_steps, **smooth_kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = H.info()
    log(f"setup {setup_s:.2f}s, {info.levels} levels, operator complexity {info.operator_complexity:.3f}")

    b_d = torch.from_numpy(b).to(dev)
    x_d = torch.zeros(A.n, dtype=torch.float64, device=dev)
    opts = dict(tol=args.tol, krylov="fcg", precision=prec)

    if args.mode == "kernels":
        # one warm solve fills every work vector with real data, then each
        # level-0 kernel and a plain copy are launched back to back
        H.solve(b_d, x_d, **opts)
        out = {}
        for name, op in (("vcycle_down_l0", pamg.OP_DOWN), ("vcycle_up_l0", pamg.OP_UP),
                         ("krylov_spmv_l0", pamg.OP_KRYLOV)):
            ms, nb = H.time_op(op, 0, reps=args.reps, precision=pamg.PREC_F64 if op == pamg.OP_KRYLOV else prec)
            out[name] = {"ms": ms, "bytes": nb, "GBps": nb / (ms * 1e-3) / 1e9}
        gbs, cms = copy_bandwidth(torch, reps=args.reps)
        out["copy_2GiB"] = {"ms": cms, "bytes": 2 * (1 << 31), "GBps": gbs}
        print(json.dumps(out), flush=True)
        return 0

    for k in range(args.warmup):
        x_d.zero_()
        t1 = time.perf_counter()
        inf = H.solve(b_d, x_d, **opts)
        log(f"warm-up solve {k}: {1e3 * (time.perf_counter() - t1):.1f} ms, {inf.iterations} iterations")
    torch.cuda.synchronize()
    times, iters = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        x_d.zero_()
        t1 = time.perf_counter()
        inf = H.solve(b_d, x_d, **opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        iters.append(inf.iterations)
        if inf.status != pamg.OK:
            log(f"solve status {inf.status}")
            return 1
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ms_per_step = 1e3 * total / args.steps
    x = x_d.cpu().numpy()
    relres_true = float(np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b))
    log(f"solve {ms_per_step:.2f} ms/step, iterations {iters[0]}, true relres {relres_true:.3e}")

    # V-cycle and SpMV throughput (back-to-back, HIP events on this stream)
    r_d = b_d.clone()
    v_ms, s_ms = H.time_kernels(r_d, reps=20, precision=prec)
    vbytes = info.vcycle_bytes_f32 if prec == pamg.PREC_F32 else info.vcycle_bytes_f64
    # (the algorithmic V-cycle bytes are those of the l1-Jacobi cycle)
    v_gbs = vbytes / (v_ms * 1e-3) / 1e9 if args.smoother == "l1" and not args.smooth_prolongator else float("nan")
    s_gbs = info.spmv_bytes / (s_ms * 1e-3) / 1e9

    # the kernels that stream the level-0 matrix, each timed live with HIP events
    kern = {}
    if args.smooth_prolongator:
        level0_ops = (("krylov_spmv_l0", pamg.OP_KRYLOV),)
    else:
        level0_ops = ((("vcycle_down_l0", pamg.OP_DOWN), ("vcycle_up_l0", pamg.OP_UP)) if args.smoother == "l1"
                      else (("hgs_sweep_l0", pamg.OP_SMOOTH),)) + (("krylov_spmv_l0", pamg.OP_KRYLOV),)
    for name, op in level0_ops:
        if op == pamg.OP_KRYLOV and prec == pamg.PREC_F32:
            ms, nb = H.time_op(op, 0, reps=20, precision=pamg.PREC_F64)
        else:
            ms, nb = H.time_op(op, 0, reps=20, precision=prec)
        kern[name] = {"ms": ms, "bytes": nb, "GBps": nb / (ms * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["ms"])
    dk = kern[dom]
    copy_gbs, _ = copy_bandwidth(torch)
    traffic = traffic_for(dom, prec == pamg.PREC_F64 and args.agg_steps == 1 and args.smoother == "l1"
                          and not args.smooth_prolongator)
    log(f"V-cycle {v_ms:.3f} ms ({v_gbs:.0f} GB/s), SpMV {s_ms:.3f} ms ({s_gbs:.0f} GB/s); "
        + ", ".join(f"{k} {v['ms']:.4f} ms {v['GBps']:.0f} GB/s" for k, v in kern.items()))

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
        "dtype": "f64" if prec == pamg.PREC_F64 else "f32-vcycle/f64-fcg",
        "data": "synthetic",
        "config": {
            "workload": f"Q1 hexahedral FE Laplacian, {args.n}^3 elements, vertical stretching {args.ratio}, "
                        f"divergence RHS seed 2; FCG + AMG V-cycle (pairwise matching aggregation"
                        + (", smoothed prolongators, " if args.smooth_prolongator else ", ")
                        + ("l1-Jacobi 1+1" if args.smoother == "l1" else
                           f"hybrid forward/backward Gauss-Seidel {H.params.sweeps or 4}+{H.params.sweeps or 4} "
                           f"(blocks of {H.params.gs_block or 256}, omega {H.params.omega or 1.5:g})")
                        + f", dense coarse solve) to {args.tol:g}",
            "n": A.n, "nnz": A.nnz, "levels": info.levels,
            "operator_complexity": round(info.operator_complexity, 4),
            "aggregate_steps": args.agg_steps,
            "smoother": args.smoother,
            "smoothed_prolongator": bool(args.smooth_prolongator),
        },
        "iterations": iters[0],
        "relres_true": relres_true,
        "setup_s": round(setup_s, 3),
        "vcycle_ms": round(v_ms, 4),
        "vcycle_GBps": round(v_gbs, 1) if v_gbs == v_gbs else None,
        "vcycle_pct_peak": round(100 * v_gbs / HBM_PEAK_GBS, 2) if v_gbs == v_gbs else None,
        "spmv_ms": round(s_ms, 4),
        "spmv_GBps": round(s_gbs, 1),
        "spmv_pct_peak": round(100 * s_gbs / HBM_PEAK_GBS, 2),
        "kernels": {k: {"ms": round(v["ms"], 5), "bytes": v["bytes"], "GBps": round(v["GBps"], 1)}
                    for k, v in kern.items()},
        "copy_GBps": round(copy_gbs, 1),
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": round(dk["GBps"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        O = oracle.Hierarchy(A, agg_steps=args.agg_steps)
        t_or_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, it_or, _, _ = O.solve(b, 0.0, krylov="fcg", fixed_iters=args.cpu_iters)
        t_or = time.perf_counter() - t0
        per_iter_ms = 1e3 * t_or / it_or
        result["cpu_baseline"] = {
            "value": round(per_iter_ms * iters[0], 2),
            "unit": "ms",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{it_or} FCG iterations of the same solve (single-threaded C oracle, its setup "
                      f"of {t_or_setup:.1f}s excluded), scaled to the {iters[0]} iterations of a full solve",
        }
        log(f"oracle {per_iter_ms:.1f} ms/iteration")
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
    H = pamg.Hierarchy(A, build_f32=1)
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
        "autotuned_f32": cfg,
    }
    print(json.dumps(out), flush=True)
    return 0


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


def bench_mixed(args, torch, np, pamg, log) -> int:
    """FP64 hierarchy versus FP32 hierarchy (both under the FP64 FCG) on the
    same stretched Q1 system (256^3 elements unless --n says otherwise,
    divergence right-hand side seed 3), each to a true FP64 relative residual
    of 1e-6; the solutions are compared with each other and with the oracle's
    stored FP64 solution samples when they exist for this workload."""
    from workloads import q1_rhs, q1_stretched
    n = args.n if args.n != 128 else 256
    t0 = time.perf_counter()
    A = q1_stretched(n, args.ratio, progress=log)
    b = q1_rhs(n, args.ratio, 3, progress=log)
    log(f"generated Q1 {n}^3: n={A.n} nnz={A.nnz} in {time.perf_counter() - t0:.1f}s")
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"q1_{n}_fcg.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            g = json.load(f)
        if g["workload"]["rhs_seed"] == 3 and g["workload"]["n"] == A.n and g["workload"]["ratio"] == args.ratio:
            golden = g
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    H = pamg.Hierarchy(A, build_f32=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = H.info()
    log(f"setup {setup_s:.2f}s, {info.levels} levels")
    b_d = torch.from_numpy(b).to(dev)
    S = A.to_scipy()
    bn = float(np.linalg.norm(b))
    res = {}
    xs = {}
    for name, prec in (("f64", pamg.PREC_F64), ("f32", pamg.PREC_F32)):
        x_d = torch.zeros(A.n, dtype=torch.float64, device=dev)
        opts = dict(tol=args.tol, krylov="fcg", precision=prec, true_residual=1)
        for _ in range(args.warmup):
            x_d.zero_()
            H.solve(b_d, x_d, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            x_d.zero_()
            inf = H.solve(b_d, x_d, **opts)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1) / args.steps
        x = x_d.cpu().numpy()
        xs[name] = x
        rel = float(np.linalg.norm(b - S @ x) / bn)
        r_d = b_d.clone()
        v_ms, _ = H.time_kernels(r_d, reps=10, precision=prec)
        vbytes = info.vcycle_bytes_f32 if prec == pamg.PREC_F32 else info.vcycle_bytes_f64
        entry = {"ms_per_solve": round(ms, 3), "iterations": inf.iterations, "status": inf.status,
                 "relres_true": rel, "vcycle_ms": round(v_ms, 4),
                 "vcycle_GBps": round(vbytes / (v_ms * 1e-3) / 1e9, 1)}
        if golden is not None:
            idx = np.array(golden["sample_index"])
            xo = np.array(golden["x_sample"])
            entry["err_vs_oracle_sample"] = float(np.linalg.norm(x[idx] - xo) / np.linalg.norm(xo))
        res[name] = entry
        log(f"{name}: {ms:.1f} ms/solve, {inf.iterations} iterations, true relres {rel:.3e}")
        if inf.status != pamg.OK or rel > args.tol:
            print(json.dumps({"error": f"{name} solve did not reach the tolerance", **entry}), flush=True)
            return 1
    err32 = float(np.linalg.norm(xs["f32"] - xs["f64"]) / np.linalg.norm(xs["f64"]))
    out = {
        "metric": "FP32-hierarchy speedup over FP64 at a true FP64 relative residual of 1e-6",
        "value": round(res["f64"]["ms_per_solve"] / res["f32"]["ms_per_solve"], 3),
        "unit": "x",
        "higher_is_better": True,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "dtype": "f64 | f32-vcycle/f64-fcg",
        "data": "synthetic",
        "config": {"workload": f"Q1 hexahedral FE Laplacian, {n}^3 elements, vertical stretching {args.ratio}, "
                               f"divergence RHS seed 3; FCG + AMG V-cycle to a true residual of {args.tol:g}",
                   "n": A.n, "nnz": A.nnz, "levels": info.levels},
        "setup_s": round(setup_s, 2),
        "f64": res["f64"],
        "f32": res["f32"],
        "f32_vs_f64_solution_relerr": err32,
        "oracle_reference": "stored oracle FP64 solution samples (512 entries)" if golden is not None else None,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
