"""Serving loop (continuous batching) through the C ABI.

* every served result meets its tolerance on the true FP64 residual and
  agrees with the oracle's FP64 solution;
* a request's result is bitwise the same alone and in a mix of requests on
  several operators (columns are independent and the hierarchy is
  deterministic), also against a one-column batched solve;
* a tiny HBM budget forces queueing and LRU eviction, and every request
  still completes correctly; an operator larger than the budget is refused;
* a zero right-hand side completes with x = 0;
* graph-replayed blocks give bitwise the results of direct launches;
* with the single-right-hand-side path on, every result is bitwise that of
  pamg_solve or of a one-column batched solve (the path depends on the mix),
  and a request alone takes the single path;
* the host phase of a new operator's setup runs beside the solving of
  cached operators (their requests finish first), and several setup workers
  give bitwise the results of one;
* operators large enough for the device construction are built on the
  device by the setup workers, within a reservation of the budget, and give
  bitwise the results of host-built ones.
"""
import time

import numpy as np
import pytest

import oracle
import paper_2210_16660_amd as pamg
from workloads import SplitMix64, varcoef7

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


def wait_all(S, n, timeout=120.0):
    got = []
    t0 = time.time()
    while len(got) < n:
        got += S.poll()
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(got)} of {n} completions after {timeout}s")
        time.sleep(0.002)
    return {int(c.tag): c for c in got}


OPS = {k: (n, 40 + k) for k, n in enumerate([10, 14, 17, 12])}


@pytest.fixture(scope="module")
def ops():
    return {k: varcoef7(n, seed=s) for k, (n, s) in OPS.items()}


def make_requests(ops, count, seed=7):
    rng = SplitMix64(seed)
    keys = rng.integers(count, 0, len(ops) - 1)
    reqs = []
    for t in range(count):
        k = int(keys[t])
        b = SplitMix64(1000 + t).uniform(ops[k].n)
        reqs.append((t, k, b))
    return reqs


def serve(ops, reqs, **kw):
    S = pamg.Server(**kw)
    xs = {}
    torch.cuda.current_stream().synchronize()
    for tag, k, b in reqs:
        x = torch.zeros(ops[k].n, dtype=torch.float64, device="cuda:0")
        bd = dev(b)
        torch.cuda.current_stream().synchronize()
        xs[tag] = x
        S.submit(k, ops[k], bd, x, tol=1e-6, tag=tag)
    done = wait_all(S, len(reqs))
    stats = S.stats()
    S.close()
    return {t: xs[t].cpu().numpy() for t in xs}, done, stats


def test_served_results_correct_and_independent_of_the_mix(ops):
    reqs = make_requests(ops, 40)
    xs, done, stats = serve(ops, reqs)
    assert stats.completed == 40 and stats.rejected == 0 and stats.setups == len(ops)
    hier = {k: oracle.Hierarchy(A) for k, A in ops.items()}
    for tag, k, b in reqs:
        c = done[tag]
        assert c.status == pamg.OK, (tag, c.status)
        A = ops[k].to_scipy()
        rel = np.linalg.norm(b - A @ xs[tag]) / np.linalg.norm(b)
        assert rel <= 1e-6 and abs(rel - c.relres_true) <= 1e-9
        x_or, _, _, _ = hier[k].solve(b, 1e-6)
        assert np.linalg.norm(xs[tag] - x_or) <= 1e-4 * np.linalg.norm(x_or)
    # alone: the same request through a fresh server, and as a one-column batch
    for tag, k, b in reqs[:4]:
        xa, da, _ = serve(ops, [(tag, k, b)])
        assert da[tag].iterations == done[tag].iterations
        assert np.array_equal(xa[tag].view(np.uint64), xs[tag].view(np.uint64)), f"request {tag} differs alone"
        H = pamg.Hierarchy(ops[k], build_f32=1)
        X = torch.zeros((1, ops[k].n), dtype=torch.float64, device="cuda:0")
        inf = H.solve_batch(dev(b[None, :]), X, tol=1e-6, precision=pamg.PREC_F32)
        assert inf[0].iterations == done[tag].iterations
        assert np.array_equal(X[0].cpu().numpy().view(np.uint64), xs[tag].view(np.uint64))


def test_graph_replay_server_matches_direct_launches(ops):
    # blocks replayed as HIP graphs give bitwise the results of direct launches
    # (the application synchronizes its own stream while the server captures)
    reqs = make_requests(ops, 16, seed=5)
    xd, dd, _ = serve(ops, reqs)
    xg, dg, st = serve(ops, reqs, use_graph=1)
    assert st.completed == 16
    for tag, k, b in reqs:
        assert dg[tag].status == pamg.OK and dg[tag].iterations == dd[tag].iterations
        assert np.array_equal(xg[tag].view(np.uint64), xd[tag].view(np.uint64))


def test_setup_workers_give_the_same_results(ops):
    # host phases built by several workers at once (each with a share of the
    # cores) give the same hierarchies: results bitwise those of one worker
    reqs = make_requests(ops, 12, seed=17)
    x1, d1, _ = serve(ops, reqs)
    x4, d4, st = serve(ops, reqs, setup_workers=4)
    assert st.setups == len({k for _, k, _ in reqs}) and st.completed == 12
    for tag, k, b in reqs:
        assert d4[tag].status == pamg.OK and d4[tag].iterations == d1[tag].iterations
        assert np.array_equal(x4[tag].view(np.uint64), x1[tag].view(np.uint64))


def test_fp64_vcycle_server(ops):
    reqs = make_requests(ops, 12, seed=3)
    xs, done, stats = serve(ops, reqs, precision=pamg.PREC_F64)
    for tag, k, b in reqs:
        O = oracle.Hierarchy(ops[k])
        x_or, it_or, _, _ = O.solve(b, 1e-6)
        assert done[tag].status == pamg.OK and abs(done[tag].iterations - it_or) <= 1
        if done[tag].iterations == it_or:
            assert np.linalg.norm(xs[tag] - x_or) <= 1e-8 * np.linalg.norm(x_or)


@pytest.mark.parametrize("prec,graph,batch_from", [(pamg.PREC_F32, 0, 100), (pamg.PREC_F64, 0, 4),
                                                   (pamg.PREC_F32, 1, 4), (pamg.PREC_F64, 1, 100)])
def test_single_path_results(ops, prec, graph, batch_from):
    # with single_path, an operator's requests run one at a time on the
    # single-right-hand-side solver while fewer than batch_from are waiting:
    # every result is bitwise either that of pamg_solve (same tolerance, maxit
    # and precision) or that of a one-column batched solve, whichever path the
    # mix gave it; with a threshold above the request count nothing is batched
    reqs = make_requests(ops, 24, seed=13)
    reqs.append((24, 2, np.zeros(ops[2].n)))
    xs, done, stats = serve(ops, reqs, single_path=1, batch_from=batch_from, precision=prec, use_graph=graph)
    assert stats.completed == 25 and stats.rejected == 0
    H = {k: pamg.Hierarchy(A, build_f32=1) for k, A in ops.items()}
    paths = {"single": 0, "batch": 0}
    for tag, k, b in reqs:
        c = done[tag]
        assert c.status == pamg.OK, (tag, c.status)
        if tag == 24:
            assert c.iterations == 0 and not xs[tag].any()
            continue
        rel = np.linalg.norm(b - ops[k].to_scipy() @ xs[tag]) / np.linalg.norm(b)
        assert rel <= (1e-6 if prec == pamg.PREC_F32 else 2e-6), (tag, rel)
        x1 = torch.zeros(ops[k].n, dtype=torch.float64, device="cuda:0")
        inf1 = H[k].solve(dev(b), x1, tol=1e-6, maxit=1000, precision=prec)
        X = torch.zeros((1, ops[k].n), dtype=torch.float64, device="cuda:0")
        infb = H[k].solve_batch(dev(b[None, :]), X, tol=1e-6, precision=prec)
        xb = X[0].cpu().numpy()
        if inf1.iterations == infb[0].iterations:
            # the two solvers agree to rounding when their iteration counts do
            assert np.linalg.norm(x1.cpu().numpy() - xb) <= 1e-8 * np.linalg.norm(xb), tag
        if np.array_equal(x1.cpu().numpy().view(np.uint64), xs[tag].view(np.uint64)):
            assert c.iterations == inf1.iterations
            paths["single"] += 1
        else:
            assert np.array_equal(xb.view(np.uint64), xs[tag].view(np.uint64)), tag
            assert c.iterations == infb[0].iterations
            paths["batch"] += 1
    if batch_from > len(reqs):
        assert paths["batch"] == 0, paths
    # a request alone on the server always takes the single path
    tag, k, b = reqs[0]
    xa, da, _ = serve(ops, [(tag, k, b)], single_path=1, batch_from=batch_from, precision=prec, use_graph=graph)
    x1 = torch.zeros(ops[k].n, dtype=torch.float64, device="cuda:0")
    H[k].solve(dev(b), x1, tol=1e-6, maxit=1000, precision=prec)
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), xa[tag].view(np.uint64))


@pytest.mark.parametrize("prec", [pamg.PREC_F32, pamg.PREC_F64])
def test_admission_estimate_bounds_the_cached_bytes(ops, prec):
    # the admission charge of an operator (its hierarchy; a 16-column engine is
    # charged when it is built) is an upper bound of the bytes it holds once
    # cached, and not a loose one
    from workloads import q1_stretched
    cases = [ops[0], ops[2], varcoef7(40, seed=91), q1_stretched(16, 1.05)]
    for A in cases:
        S = pamg.Server(precision=prec, single_path=1)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda:0")
        S.submit(1, A, dev(np.zeros(A.n)), x, tag=1)
        d = wait_all(S, 1)
        st = S.stats()
        S.close()
        assert d[1].status == pamg.OK and st.setups == 1
        est = pamg.server_estimate_bytes(A, prec)
        assert st.bytes_in_use <= est, (A.n, st.bytes_in_use, est)
        assert st.bytes_in_use >= est // 16, (A.n, st.bytes_in_use, est)


def test_tiny_budget_queues_and_evicts(ops):
    # room for about one batched operator (hierarchy and 16-column engine) at
    # a time: requests for the others wait, idle operators give up their
    # engines or are evicted, everything still completes
    est = max(pamg.server_estimate_bytes(A) for A in ops.values())
    reqs = make_requests(ops, 24, seed=11)
    xs, done, stats = serve(ops, reqs, hbm_budget_bytes=int(est * 1.02))
    assert stats.completed == 24 and stats.rejected == 0
    # the four batched operators do not fit together (which ones fit beside
    # each other decides how many engines are freed and operators evicted)
    assert stats.engines_built >= len(ops) and stats.setups >= len(ops)
    assert stats.engines_freed + stats.evictions >= 1
    assert stats.bytes_in_use <= stats.hbm_budget_bytes
    for tag, k, b in reqs:
        assert done[tag].status == pamg.OK
        rel = np.linalg.norm(b - ops[k].to_scipy() @ xs[tag]) / np.linalg.norm(b)
        assert rel <= 1e-6


def test_oversized_operator_refused_and_zero_rhs(ops):
    S = pamg.Server(hbm_budget_bytes=1 << 20)
    x = torch.zeros(ops[1].n, dtype=torch.float64, device="cuda:0")
    S.submit(1, ops[1], dev(np.ones(ops[1].n)), x, tag=1)
    d = wait_all(S, 1)
    assert d[1].status == pamg.E_BUSY
    S.close()
    S = pamg.Server()
    x = torch.ones(ops[0].n, dtype=torch.float64, device="cuda:0")
    S.submit(0, ops[0], dev(np.zeros(ops[0].n)), x, tag=2)
    d = wait_all(S, 1)
    assert d[2].status == pamg.OK and d[2].iterations == 0 and not x.cpu().numpy().any()
    S.close()


def test_setup_runs_beside_solves(ops):
    S = pamg.Server()
    x0 = torch.zeros(ops[0].n, dtype=torch.float64, device="cuda:0")
    S.submit(0, ops[0], dev(np.zeros(ops[0].n)), x0, tag=1000)
    wait_all(S, 1)
    big = varcoef7(90, seed=77)                  # 729,000 unknowns: a long host phase
    xb = torch.zeros(big.n, dtype=torch.float64, device="cuda:0")
    bb = dev(SplitMix64(78).uniform(big.n))
    xs = [torch.zeros(ops[0].n, dtype=torch.float64, device="cuda:0") for _ in range(8)]
    bs = [dev(SplitMix64(2000 + t).uniform(ops[0].n)) for t in range(8)]
    torch.cuda.current_stream().synchronize()
    S.submit(99, big, bb, xb, tag=99)
    for t in range(8):
        S.submit(0, None, bs[t], xs[t], tag=t)
    done = wait_all(S, 9, timeout=300)
    st = S.stats()
    S.close()
    assert all(done[t].status == pamg.OK for t in done)
    assert max(done[t].latency_ms for t in range(8)) < done[99].latency_ms
    assert st.host_setup_ms > 0 and st.setups == 2
    rel = np.linalg.norm(bb.cpu().numpy() - big.to_scipy() @ xb.cpu().numpy()) / np.linalg.norm(bb.cpu().numpy())
    assert rel <= 1e-6


def test_engines_are_built_on_demand_and_freed_before_evictions(ops):
    # single-right-hand-side path on: an operator whose requests come alone
    # holds only its hierarchy; several waiting requests build its 16-column
    # engine; with room for every hierarchy and the largest engine but not
    # for every engine, idle operators give up their engines (an operator
    # waits on the single path while the room is busy) and none is evicted
    reqs = make_requests(ops, 40, seed=13)
    big = 1 << 36
    _, _, st_hier = serve(ops, reqs, hbm_budget_bytes=big, single_path=1, batch_from=1000)
    assert st_hier.engines_built == 0 and st_hier.setups == len(ops)
    _, _, st_all = serve(ops, reqs, hbm_budget_bytes=big, single_path=1, batch_from=2)
    assert st_all.engines_built == len(ops) and st_all.engines_freed == 0
    hier = st_hier.bytes_in_use
    engines = st_all.bytes_in_use - hier
    # admission charges an upper estimate until the hierarchy exists
    room = max(max(pamg.server_estimate_bytes(A) for A in ops.values()), engines // 2)
    assert room < engines, (room, engines)
    budget = hier + room

    S = pamg.Server(hbm_budget_bytes=budget, single_path=1, batch_from=2)
    xs = {}

    def submit(batch):
        for tag, k, b in batch:
            x = torch.zeros(ops[k].n, dtype=torch.float64, device="cuda:0")
            bd = dev(b)
            torch.cuda.current_stream().synchronize()
            xs[tag] = (x, bd)
            S.submit(k, ops[k], bd, x, tol=1e-6, tag=tag)
        return wait_all(S, len(batch))

    # one lone request per operator: every hierarchy cached, no engine
    first = [(100 + k, k, SplitMix64(500 + k).uniform(ops[k].n)) for k in ops]
    done = submit(first)
    st = S.stats()
    assert st.setups == len(ops) and st.engines_built == 0 and st.bytes_in_use == hier
    done.update(submit(reqs))
    st = S.stats()
    S.close()
    assert st.completed == 40 + len(ops) and st.rejected == 0
    assert st.evictions == 0 and st.setups == len(ops)
    assert st.engines_built >= 2 and st.engines_freed >= 1
    assert st.bytes_in_use <= budget
    for tag, k, b in first + reqs:
        assert done[tag].status == pamg.OK
        x = xs[tag][0].cpu().numpy()
        rel = np.linalg.norm(b - ops[k].to_scipy() @ x) / np.linalg.norm(b)
        assert rel <= 1e-6


def test_device_built_operators_serve_like_host_built_ones(ops):
    # two operators above the device construction's size floor among the
    # small ones: workers build them on the device (beside the solving, in
    # a reserved share of the budget); every result is bitwise the
    # host-built server's (batch engine only: results independent of the mix)
    from workloads import q1_stretched
    big = dict(ops)
    big[4] = varcoef7(44, seed=51)
    big[5] = q1_stretched(42, 1.05)
    reqs = make_requests(big, 30, seed=17)
    reqs += [(100 + t, k, SplitMix64(700 + t).uniform(big[k].n)) for t, k in enumerate([4, 5, 4, 5])]
    xd, dd, sd = serve(big, reqs, setup_workers=2, device_setup=1)
    xh, dh, sh = serve(big, reqs, setup_workers=2, device_setup=0)
    assert sd.completed == sh.completed == len(reqs) and sd.rejected == 0
    assert sd.setups == sh.setups == len(big)
    assert sd.device_setup_ms > 0
    for tag, k, b in reqs:
        assert dd[tag].status == dh[tag].status == pamg.OK
        assert dd[tag].iterations == dh[tag].iterations
        assert np.array_equal(xd[tag], xh[tag]), tag
        rel = np.linalg.norm(b - big[k].to_scipy() @ xd[tag]) / np.linalg.norm(b)
        assert rel <= 1e-6
