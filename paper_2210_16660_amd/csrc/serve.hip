// Serving loop: continuous batching of pressure solves on one GPU.
//
// Requests name an operator (a caller-chosen key plus its CSR, read only the
// first time the key is seen) and carry a device right-hand side, a device
// output vector and a tolerance.  A scheduler thread owns all GPU work:
//   * setup off the critical path: an operator's setup runs on a worker
//     thread while the scheduler keeps iterating the cached operators: its
//     large levels on the device, on the worker's own stream, once the
//     scheduler has reserved room for it in the budget; otherwise (or for
//     the configurations only the host builds) the host phase (matching,
//     Galerkin products, layout), uploaded by the scheduler;
//   * admission: an operator's hierarchy is admitted if its bytes fit the HBM
//     budget, freeing idle operators' 16-column engines and then evicting
//     idle cached operators in least-recently-used order; otherwise it waits;
//   * batching: every cached operator is a group with its own stream and 16
//     columns; a waiting request takes a free column between iteration blocks
//     and its recurrence starts there (columns are independent, so a result
//     is the same whatever else is in the group);
//   * overlap: every group with running columns has one iteration block in
//     flight on its own stream; a group whose block has finished (its event)
//     is served at once, without waiting for the others, so small operators
//     are not held back by large ones and the groups' work overlaps;
//   * retirement: a column whose stopping test holds (or hit maxit) is copied
//     out and freed at once; with the FP32 V-cycle its true residual is
//     checked first and the recurrence restarted from it if needed.
// The problem setting is the paper's: the same pressure operator is solved
// many times (Sec. 2), and hierarchies are reused (Sec. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "batch.hpp"
#include "dsetup.hpp"

extern "C" int pamg_hierarchy_destroy(pamg_hierarchy* h);

namespace pamg {

using Clock = std::chrono::steady_clock;

struct ServeRequest {
    pamg_request r;
    Clock::time_point t_submit, t_admit;
    int restarts = 0;
};

// One operator's setup, done by a worker thread: the host phase (built), or
// the whole hierarchy built on the device (h, on the job's stream) after the
// scheduler reserved `need` bytes for it.
struct SetupJob {
    uint64_t key = 0;
    pamg_csr A{};                    // the caller's CSR (valid until its requests complete)
    std::unique_ptr<HostBuild> built;
    pamg_hierarchy* h = nullptr;     // device-built (owned by the job until admitted)
    hipStream_t stream = nullptr;    // the device build's stream (becomes the group's)
    uint64_t need = 0;               // bytes to reserve before the device build
    uint64_t reserved = 0;           // reserved in bytes_in_use (guarded by mu)
    int room = 0;                    // guarded by mu: 1 reserved, -1 refused (over the budget)
    double build_ms = 0.0;
    bool returned = false;           // handed back by the worker (scheduler-owned flag)
    int status = PAMG_OK;
    std::string error;
    ~SetupJob() {
        if (h) pamg_hierarchy_destroy(h);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

struct ServeGroup {
    uint64_t key = 0;
    pamg_hierarchy* h = nullptr;
    BatchEngine* E = nullptr;
    hipStream_t stream = nullptr;
    ServeRequest* col[kW] = {};
    int active = 0;
    uint64_t last_used = 0;
    uint64_t bytes = 0;          // device bytes: hierarchy, and the engine while it exists
    uint64_t engine = 0;         // of which the 16-column engine
    uint64_t iter_bytes = 0;     // algorithmic bytes of one batched iteration
    hipEvent_t ev = nullptr;     // recorded behind the state copy of the block in flight
    bool in_flight = false;
    int iter_before[kW] = {};    // column iteration counts when the block was launched
    // single-right-hand-side path: one request on the hierarchy's own solver
    // (its vectors are n, not n x 16), on the same stream (a second stream
    // per operator would also take a share of the hardware queues, which
    // streams get round-robin)
    ServeRequest* single = nullptr;
    hipEvent_t single_ev = nullptr;
    bool single_in_flight = false;
    int single_iter_before = 0;  // its iteration count at the last state copy read
    uint64_t single_iter_bytes = 0;
    bool idle() const { return active == 0 && !in_flight && !single && !single_in_flight; }
};

}  // namespace pamg

struct pamg_server {
    pamg_server_opts opts{};
    pamg_context* ctx = nullptr;                     // allocator of every hierarchy built here
    int device = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<pamg::ServeRequest*> incoming;        // guarded by mu
    std::vector<pamg_completion> done;               // guarded by mu
    pamg_server_stats stats{};                       // guarded by mu (copied out)
    // setup worker
    std::vector<std::thread> setup_th;               // setup workers
    std::condition_variable setup_cv;
    std::deque<pamg::SetupJob*> setup_queue;         // guarded by mu
    bool sched_done = false;                         // guarded by mu: scheduler thread has ended
    std::vector<pamg::SetupJob*> setup_done;         // guarded by mu
    std::deque<pamg::SetupJob*> room_wait;           // guarded by mu: device builds waiting for room
    // scheduler-owned
    std::deque<pamg::ServeRequest*> pending;
    std::map<uint64_t, pamg::ServeGroup*> groups;
    std::map<uint64_t, pamg::SetupJob*> setups;      // keys queued, in progress or waiting for room
    uint64_t tick = 0;
    std::string fatal;
    bool progressed = false;                         // scheduler-owned: the last tick did something
};

namespace pamg {

static double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Upper estimate of the device bytes of an operator's hierarchy before it is
// built (replaced by the exact figure after): per level index arrays, values
// and the restriction values (plus their FP32 copies), vectors; coarse levels
// add at most 1.3x the finest (pairwise coarsening), fixed buffers ~0.2 MB.
// The 16-column engine (eight n x 16 FP64 vectors at level 0 and two
// n_l x 16 vectors per level) is built only when the operator's requests run
// as a batch, and is charged then.
static uint64_t dense_bytes(uint64_t nL, int prec) { return nL * nL * (prec == PAMG_PREC_F32 ? 12 : 8); }

static uint64_t estimate_core(const pamg_csr& A, int prec) {
    const double cx = 2.3;
    const double n = (double)A.n, nnz = (double)A.nnz;
    double hier = cx * (nnz * (4 + 8 + 8) + n * 80) + 96.0 * n + (1 << 18);
    if (prec == PAMG_PREC_F32) hier += cx * (nnz * 8 + n * 32) + 4.0 * n;
    return (uint64_t)hier;
}

// ... plus the dense inverse of a coarsest level of the usual size (at most
// the default max_coarse rows); a stalled coarsening can leave a larger one,
// which admission charges once the host phase has fixed n_L.
static uint64_t hierarchy_estimate(const pamg_csr& A, int prec) {
    return estimate_core(A, prec) + dense_bytes(std::min<uint64_t>((uint64_t)A.n, 200), prec);
}

// Upper estimate of the 16-column engine before the hierarchy exists (the
// exact figure, engine_bytes, needs its level sizes): eight FP64 n x 16
// vectors at level 0 (plus the FP32 copy of the right-hand side), two
// n_l x 16 vectors per level with the levels' rows summing to at most 2.3 n,
// the coarsest right-hand side and the reduction partials.
static uint64_t engine_estimate(uint64_t n, int prec) {
    const double s = prec == PAMG_PREC_F32 ? 4 : 8;
    const double per_row = 8 * 8 + (prec == PAMG_PREC_F32 ? 4 : 0) + 2 * 2.3 * s;
    return (uint64_t)((double)kW * (per_row * (double)n + 200 * s)) + 2ull * kMaxGrid * kW * 2 * 8 + 4096;
}

// What an operator can hold in the server: its hierarchy and, once its
// requests run as a batch, its engine.
uint64_t estimate_bytes(const pamg_csr& A, int prec) {
    return hierarchy_estimate(A, prec) + engine_estimate((uint64_t)A.n, prec);
}

static uint64_t batch_iteration_bytes(const pamg_hierarchy* h, int prec) {
    const uint64_t s = prec == PAMG_PREC_F32 ? 4 : 8;
    uint64_t B = 0;
    for (int l = 0; l < h->L; ++l) {
        const uint64_t n = h->idx[l].n, nc = h->idx[l + 1].n, nnz = h->idx[l].nnz;
        B += 2 * (nnz * (4 + s) + 4 * (n + 1)) + (10 * n + 2 * nc) * kW * s;
    }
    const uint64_t n0 = h->idx[0].n, nnz0 = h->idx[0].nnz;
    B += nnz0 * 12 + 4 * (n0 + 1) + 12 * n0 * kW * 8;
    return B;
}

static void complete(pamg_server* S, ServeRequest* q, int status, int iters, double relres, double relres_true) {
    pamg_completion c{};
    c.tag = q->r.tag;
    c.status = status;
    c.iterations = iters;
    c.relres = relres;
    c.relres_true = relres_true;
    const auto now = Clock::now();
    c.queue_ms = ms_between(q->t_submit, q->t_admit.time_since_epoch().count() ? q->t_admit : now);
    c.latency_ms = ms_between(q->t_submit, now);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->done.push_back(c);
        S->stats.completed += 1;
        if (status == PAMG_E_BUSY) S->stats.rejected += 1;
    }
    delete q;
}

static void release_streams(ServeGroup* g) {
    (void)hipEventDestroy(g->ev);
    if (g->single_ev) (void)hipEventDestroy(g->single_ev);
    (void)hipStreamDestroy(g->stream);
}

static void evict(pamg_server* S, ServeGroup* g) {
    HIP_CHECK(hipStreamSynchronize(g->stream));
    pamg_hierarchy_destroy(g->h);
    release_streams(g);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.bytes_in_use -= g->bytes;
        S->stats.evictions += 1;
        S->stats.cached_operators -= 1;
    }
    S->groups.erase(g->key);
    delete g;
}

// Free the 16-column engine of an idle operator (its hierarchy stays cached).
static void drop_engine(pamg_server* S, ServeGroup* g) {
    HIP_CHECK(hipStreamSynchronize(g->stream));
    release_engine(g->h, S->opts.precision);
    g->E = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.bytes_in_use -= g->engine;
        S->stats.engines_freed += 1;
    }
    g->bytes -= g->engine;
    g->engine = 0;
}

static uint64_t bytes_in_use(pamg_server* S) {
    std::lock_guard<std::mutex> lk(S->mu);
    return S->stats.bytes_in_use;
}

// Make `need` more bytes fit the budget: first free the engines of idle
// operators, then (evict_operators) evict idle operators, least recently used
// first (never `keep`).  False if what is left is busy.
static bool make_room(pamg_server* S, uint64_t need, const ServeGroup* keep, bool evict_operators) {
    const uint64_t budget = S->opts.hbm_budget_bytes;
    while (bytes_in_use(S) + need > budget) {
        ServeGroup* lru = nullptr;
        for (auto& kv : S->groups) {
            ServeGroup* g = kv.second;
            if (g != keep && g->E && g->active == 0 && !g->in_flight && (!lru || g->last_used < lru->last_used))
                lru = g;
        }
        if (lru) {
            drop_engine(S, lru);
            continue;
        }
        if (!evict_operators) return false;
        for (auto& kv : S->groups)
            if (kv.second != keep && kv.second->idle() && (!lru || kv.second->last_used < lru->last_used))
                lru = kv.second;
        if (!lru) return false;
        evict(S, lru);
    }
    return true;
}

// The operator's 16-column engine, built when its requests first run as a
// batch (with the kernel variants tuned for its hierarchy, kept across
// engines) if its bytes fit the budget, freeing idle operators' engines and,
// with evict_operators (no single-column path to fall back on), evicting idle
// operators for it; false: not now.
static bool ensure_engine(pamg_server* S, ServeGroup* g, bool evict_operators) {
    if (g->E) return true;
    const int prec = S->opts.precision;
    const uint64_t need = engine_bytes(g->h, prec);
    if (need > S->opts.hbm_budget_bytes || !make_room(S, need, g, evict_operators)) return false;
    g->E = get_engine(g->h, prec, g->stream);
    if (S->opts.use_graph) batch_prepare_graph(g->E, PAMG_KRYLOV_FCG, S->opts.block_iters);
    g->engine = batch_bytes(g->E);
    g->bytes += g->engine;
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.bytes_in_use += g->engine;
    S->stats.engines_built += 1;
    return true;
}

// Upper bound of the device bytes of an operator whose host phase is done:
// the estimate with the dense coarsest inverse at its actual size.
static uint64_t bound_bytes(const SetupJob& j, int prec) {
    return estimate_core(j.A, prec) + dense_bytes((uint64_t)coarsest_n(*j.built), prec);
}

static void fail_key(pamg_server* S, uint64_t key, int status) {
    for (auto it = S->pending.begin(); it != S->pending.end();) {
        if ((*it)->r.op_key == key) {
            complete(S, *it, status, 0, 0.0, -1.0);
            it = S->pending.erase(it);
        } else {
            ++it;
        }
    }
}

// Queue the host phase for an uncached operator named by a pending request
// (once per key); refuse an operator whose estimate alone exceeds the budget.
static void request_setup(pamg_server* S, ServeRequest* q) {
    const uint64_t key = q->r.op_key;
    if (S->groups.count(key) || S->setups.count(key)) return;
    if (!q->r.A) throw Error(PAMG_E_INVALID, "request for an uncached operator carries no matrix");
    if (hierarchy_estimate(*q->r.A, S->opts.precision) > S->opts.hbm_budget_bytes) throw Error(PAMG_E_BUSY, "");
    SetupJob* j = new SetupJob();
    j->key = key;
    j->A = *q->r.A;
    S->setups[key] = j;
    std::lock_guard<std::mutex> lk(S->mu);
    S->setup_queue.push_back(j);
    S->setup_cv.notify_one();
}

// Upload operators whose host phase is done, as the budget allows (evicting
// idle cached operators, least recently used first).
// Give the device builds waiting for room their reservation, in order
// (freeing idle engines and evicting idle operators as for an admission);
// a build whose bound exceeds the whole budget is refused.
static void grant_room(pamg_server* S) {
    const uint64_t budget = S->opts.hbm_budget_bytes;
    for (;;) {
        SetupJob* j = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->room_wait.empty()) return;
            j = S->room_wait.front();
            if (j->need > budget) {
                j->room = -1;
                S->room_wait.pop_front();
                S->setup_cv.notify_all();
                continue;
            }
        }
        if (!make_room(S, j->need, nullptr, true)) return;   // everything busy: next tick
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.bytes_in_use += j->need;
        j->reserved = j->need;
        j->room = 1;
        S->room_wait.pop_front();
        S->setup_cv.notify_all();
        S->progressed = true;
    }
}

static void release_reservation(pamg_server* S, SetupJob* j) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.bytes_in_use -= j->reserved;
    j->reserved = 0;
}

static void admit_ready(pamg_server* S) {
    grant_room(S);
    std::vector<SetupJob*> fin;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        fin.swap(S->setup_done);
    }
    for (SetupJob* j : fin) {
        j->returned = true;
        if (j->status != PAMG_OK) {
            release_reservation(S, j);
            S->setups.erase(j->key);
            fail_key(S, j->key, j->status);
            delete j;
        }
    }
    const int prec = S->opts.precision;
    const uint64_t budget = S->opts.hbm_budget_bytes;
    for (auto it = S->setups.begin(); it != S->setups.end();) {
        SetupJob* j = it->second;
        if (!j->returned) { ++it; continue; }
        if (j->h) {
            // built on the device within its reservation: the exact bytes replace it
            std::unique_ptr<ServeGroup> g(new ServeGroup());
            g->key = j->key;
            g->stream = j->stream;
            j->stream = nullptr;
            g->h = j->h;
            j->h = nullptr;
            HIP_CHECK(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming));
            if (S->opts.single_path) HIP_CHECK(hipEventCreateWithFlags(&g->single_ev, hipEventDisableTiming));
            const auto t0 = Clock::now();
            if (S->opts.use_graph && S->opts.single_path) single_prepare_graph(g->h, prec, S->opts.block_iters);
            g->bytes = g->h->info.device_bytes;
            g->iter_bytes = batch_iteration_bytes(g->h, prec);
            g->single_iter_bytes = single_iteration_bytes(g->h, prec);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->stats.bytes_in_use += g->bytes;
                S->stats.bytes_in_use -= j->reserved;
                S->stats.setups += 1;
                S->stats.cached_operators += 1;
                S->stats.device_setup_ms += j->build_ms + ms_between(t0, Clock::now());
            }
            j->reserved = 0;
            ServeGroup* raw = g.release();
            S->groups[raw->key] = raw;
            it = S->setups.erase(it);
            delete j;
            S->progressed = true;
            continue;
        }
        if (j->reserved) release_reservation(S, j);   // the device construction did not apply
        const uint64_t need = bound_bytes(*j, prec);
        if (need > budget) {
            it = S->setups.erase(it);
            fail_key(S, j->key, PAMG_E_BUSY);
            delete j;
            continue;
        }
        if (!make_room(S, need, nullptr, true)) { ++it; continue; }   // everything busy: try again next tick
        std::unique_ptr<ServeGroup> g(new ServeGroup());
        g->key = j->key;
        HIP_CHECK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming));
        if (S->opts.single_path) HIP_CHECK(hipEventCreateWithFlags(&g->single_ev, hipEventDisableTiming));
        const double host_ms = j->built->host_ms;
        const auto t0 = Clock::now();
        try {
            g->h = finish_build(std::move(j->built), g->stream, S->ctx);
        } catch (const Error& e) {
            release_streams(g.get());
            it = S->setups.erase(it);
            fail_key(S, j->key, e.code);
            delete j;
            continue;
        }
        if (S->opts.use_graph && S->opts.single_path)   // capture now, not on the first request
            single_prepare_graph(g->h, prec, S->opts.block_iters);
        g->bytes = g->h->info.device_bytes;
        g->iter_bytes = batch_iteration_bytes(g->h, prec);
        g->single_iter_bytes = single_iteration_bytes(g->h, prec);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.bytes_in_use += g->bytes;
            S->stats.setups += 1;
            S->stats.cached_operators += 1;
            S->stats.host_setup_ms += host_ms;
            S->stats.device_setup_ms += ms_between(t0, Clock::now());
        }
        ServeGroup* raw = g.release();
        S->groups[raw->key] = raw;
        it = S->setups.erase(it);
        delete j;
    }
}

// Bytes a device build of A may hold at once: the hierarchy estimate plus
// the canonical levels and per-level scratch of the construction (about 40
// bytes per stored entry and 128 per row of the input, with the coarse
// levels' share).
static uint64_t device_build_bound(const pamg_csr& A, int prec) {
    return hierarchy_estimate(A, prec) + 40ull * (uint64_t)A.nnz + 128ull * (uint64_t)A.n + (1ull << 20);
}

// Ask the scheduler for `need` bytes of the budget; false if refused (more
// than the budget) or if the server ended.
static bool wait_for_room(pamg_server* S, SetupJob* j) {
    std::unique_lock<std::mutex> lk(S->mu);
    S->room_wait.push_back(j);
    S->cv.notify_one();
    S->setup_cv.wait(lk, [&] { return j->room != 0 || S->sched_done; });
    return j->room > 0;
}

static void setup_main(pamg_server* S, int threads) {
    set_num_threads(threads);        // this worker's share of the host cores
    (void)hipSetDevice(S->device);
    for (;;) {
        SetupJob* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // the scheduler may queue jobs until it has finished (it drains the
            // outstanding requests first), so only its end stops the worker
            S->setup_cv.wait(lk, [&] { return S->sched_done || !S->setup_queue.empty(); });
            if (S->setup_queue.empty()) return;
            j = S->setup_queue.front();
            S->setup_queue.pop_front();
        }
        pamg_params prm;
        pamg_params_default(&prm);
        prm.build_f32 = S->opts.precision == PAMG_PREC_F32 ? 1 : 0;
        prm.num_threads = threads;
        prm.device_setup = S->opts.device_setup ? 1 : 0;
        try {
            if (device_setup_applies(prm) && j->A.n > std::max({kDeviceMinRows, prm.max_dense, prm.max_coarse})) {
                validate_csr_header(j->A);   // the rows are checked by the build
                j->need = device_build_bound(j->A, S->opts.precision);
                // refused (the build's bound exceeds the whole budget): the
                // host construction, whose admission needs only the hierarchy
                if (wait_for_room(S, j)) {
                    HIP_CHECK(hipStreamCreateWithFlags(&j->stream, hipStreamNonBlocking));
                    const auto t0 = Clock::now();
                    j->h = device_setup_build(j->A, prm, j->stream, S->ctx);
                    j->build_ms = ms_between(t0, Clock::now());
                    if (!j->h) {
                        (void)hipStreamDestroy(j->stream);
                        j->stream = nullptr;
                    }
                }
            }
            if (!j->h) j->built = host_build(j->A, prm);
        } catch (const Error& e) {
            j->status = e.code;
            j->error = e.what();
        } catch (const std::bad_alloc&) {
            j->status = PAMG_E_OOM;
        } catch (const std::exception& e) {
            j->status = PAMG_E_DEVICE;
            j->error = e.what();
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (j->status != PAMG_OK) j->built.reset();
        S->setup_done.push_back(j);
        S->cv.notify_one();
    }
}

// Copy out and free the finished columns of a group (state host copy current).
static void retire(pamg_server* S, ServeGroup* g) {
    BatchState& st = batch_state_host(g->E);
    int finished = 0;
    for (int c = 0; c < kW; ++c)
        if (g->col[c] && st.col[c].active && st.col[c].done) finished |= 1 << c;
    if (!finished) return;
    double rel[kW];
    for (double& v : rel) v = -1.0;
    if (S->opts.precision == PAMG_PREC_F32) {
        // the FP32 V-cycle: accept a column on its true FP64 residual only
        batch_true_residual(g->E, 0, rel, g->stream);
        int restart = 0;
        for (int c = 0; c < kW; ++c) {
            if (!((finished >> c) & 1)) continue;
            const BatchCol& C = st.col[c];
            ServeRequest* q = g->col[c];
            if (C.status == PAMG_OK && C.done == 1 && rel[c] > C.tol && q->restarts < 10 && C.iter < C.maxit) {
                restart |= 1 << c;
                q->restarts += 1;
            }
        }
        if (restart) {
            double tmp[kW];
            batch_true_residual(g->E, restart, tmp, g->stream);
            finished &= ~restart;
        }
    }
    if (!finished) return;
    double* dst[kW] = {};
    for (int c = 0; c < kW; ++c)
        if ((finished >> c) & 1) dst[c] = g->col[c]->r.x_dev;
    batch_store(g->E, dst, g->stream);
    for (int c = 0; c < kW; ++c) {
        if (!((finished >> c) & 1)) continue;
        const BatchCol& C = st.col[c];
        complete(S, g->col[c], C.status, C.iter, C.bnorm > 0 ? C.rnorm / C.bnorm : 0.0, rel[c]);
        g->col[c] = nullptr;
        g->active -= 1;
    }
    batch_retire(g->E, finished);
    batch_write_state(g->E, g->stream);
}

// The single-path request of a group after a block (state host copy current):
// finished -> (FP32 V-cycle: accepted on its true residual, else restarted
// from it, as in pamg_solve) result written and completed.
static void retire_single(pamg_server* S, ServeGroup* g) {
    const SolveState& st = single_state(g->h);
    if (!st.done) return;
    ServeRequest* q = g->single;
    double rel = -1.0;
    if (st.done == 1 && S->opts.precision == PAMG_PREC_F32) {
        rel = single_true_relres(g->h, g->stream);
        if (st.status == PAMG_OK && rel > st.tol && q->restarts < 10 && st.iter < st.maxit) {
            q->restarts += 1;
            single_restart(g->h, g->stream);   // the next block continues from it
            return;
        }
    }
    single_end(g->h, q->r.x_dev, g->stream);
    complete(S, q, st.status, st.iter, st.bnorm > 0 ? st.rnorm / st.bnorm : 0.0, rel);
    g->single = nullptr;
}

static void scheduler_tick(pamg_server* S) {
    ++S->tick;
    // 1. groups whose block has finished: account, retire finished columns
    //    (before admission, so that waiting requests join between blocks)
    uint64_t moved = 0;
    for (auto& kv : S->groups) {
        ServeGroup* g = kv.second;
        if (!g->in_flight) continue;
        const hipError_t q = hipEventQuery(g->ev);
        if (q == hipErrorNotReady) continue;
        HIP_CHECK(q);
        g->in_flight = false;
        int ran = 0;
        for (int c = 0; c < kW; ++c) ran = std::max(ran, batch_state_host(g->E).col[c].iter - g->iter_before[c]);
        moved += (uint64_t)ran * g->iter_bytes;
        retire(S, g);
        S->progressed = true;
    }
    for (auto& kv : S->groups) {
        ServeGroup* g = kv.second;
        if (!g->single_in_flight) continue;
        const hipError_t q = hipEventQuery(g->single_ev);
        if (q == hipErrorNotReady) continue;
        HIP_CHECK(q);
        g->single_in_flight = false;
        const int it_now = single_state(g->h).iter;
        moved += (uint64_t)std::max(0, it_now - g->single_iter_before) * g->single_iter_bytes;
        g->single_iter_before = it_now;
        retire_single(S, g);
        S->progressed = true;
    }
    // 2. finished host phases become cached operators as the budget allows;
    //    waiting requests take free columns of cached operators
    admit_ready(S);
    std::map<ServeGroup*, int> loads;
    std::map<uint64_t, int> waiting;     // pending requests per operator not yet placed
    if (S->opts.single_path)
        for (ServeRequest* q : S->pending) waiting[q->r.op_key] += 1;
    for (auto it = S->pending.begin(); it != S->pending.end();) {
        ServeRequest* q = *it;
        auto gi = S->groups.find(q->r.op_key);
        if (gi == S->groups.end()) {
            try {
                request_setup(S, q);
                ++it;
            } catch (const Error& e) {
                it = S->pending.erase(it);
                complete(S, q, e.code, 0, 0.0, -1.0);
            }
            continue;
        }
        ServeGroup* g = gi->second;
        // an engine that can never fit the budget beside the hierarchy: the
        // operator's requests run on the single-right-hand-side path (or are
        // refused without it)
        const bool no_batch = !g->E && g->bytes + engine_bytes(g->h, S->opts.precision) > S->opts.hbm_budget_bytes;
        if (no_batch && !S->opts.single_path) {
            it = S->pending.erase(it);
            complete(S, q, PAMG_E_BUSY, 0, 0.0, -1.0);
            continue;
        }
        // with the single path: a batch only once batch_from requests wait and
        // its engine exists or can be built now (not behind a single block in
        // flight on the operator's stream, which would skew the variant tuning)
        const bool batch = !S->opts.single_path || g->active > 0 ||
                           (waiting[g->key] >= S->opts.batch_from && !no_batch && !g->in_flight &&
                            (g->E || !g->single_in_flight) && ensure_engine(S, g, false));
        if (S->opts.single_path && g->active == 0 && !batch) {
            // few requests for this operator and no batch running: one at a
            // time on the single-right-hand-side solver (its iterations move
            // about a sixth of the bytes of a 16-column batched iteration)
            if (g->single || g->single_in_flight) {
                ++it;
                continue;
            }
            single_begin(g->h, q->r.b_dev, q->r.tol, q->r.maxit > 0 ? q->r.maxit : 1000, g->stream);
            g->single = q;
            g->single_iter_before = 0;
            waiting[g->key] -= 1;
            q->t_admit = Clock::now();
            it = S->pending.erase(it);
            S->progressed = true;
            continue;
        }
        if (g->active >= kW || g->in_flight || !ensure_engine(S, g, !S->opts.single_path)) {   // joins happen between blocks
            ++it;
            continue;
        }
        int c = 0;
        while (g->col[c]) ++c;
        g->col[c] = q;
        g->active += 1;
        loads[g] |= 1 << c;
        if (S->opts.single_path) waiting[g->key] -= 1;
        q->t_admit = Clock::now();
        it = S->pending.erase(it);
    }
    for (auto& kv : loads) {
        ServeGroup* g = kv.first;
        const double* src[kW] = {};
        double tol[kW];
        int maxit[kW], fixed[kW];
        for (int c = 0; c < kW; ++c) {
            tol[c] = 1e-6;
            maxit[c] = 1000;
            fixed[c] = 0;
            if ((kv.second >> c) & 1) {
                src[c] = g->col[c]->r.b_dev;
                tol[c] = g->col[c]->r.tol;
                maxit[c] = g->col[c]->r.maxit > 0 ? g->col[c]->r.maxit : 1000;
            }
        }
        batch_read_state(g->E, g->stream);
        batch_load(g->E, src, tol, maxit, fixed, PAMG_KRYLOV_FCG, g->stream);
        retire(S, g);                    // zero right-hand sides finish at once
        S->progressed = true;
    }
    // 3. every idle group with running columns gets its next block, followed
    //    by an asynchronous copy of its state and an event
    const int k = S->opts.block_iters;
    uint64_t blocks = 0;
    for (auto& kv : S->groups) {
        ServeGroup* g = kv.second;
        if (!g->single || g->single_in_flight) continue;
        single_block(g->h, S->opts.precision, k, S->opts.use_graph != 0, g->stream);
        HIP_CHECK(hipEventRecord(g->single_ev, g->stream));
        g->single_in_flight = true;
        g->last_used = S->tick;
        ++blocks;
        S->progressed = true;
    }
    for (auto& kv : S->groups) {
        ServeGroup* g = kv.second;
        if (g->in_flight || g->active == 0 || !g->E || batch_state_host(g->E).all_done) continue;
        for (int c = 0; c < kW; ++c) g->iter_before[c] = batch_state_host(g->E).col[c].iter;
        batch_run_block(g->E, PAMG_KRYLOV_FCG, k, S->opts.use_graph != 0, g->stream);
        batch_read_state_async(g->E, g->stream);
        HIP_CHECK(hipEventRecord(g->ev, g->stream));
        g->in_flight = true;
        g->last_used = S->tick;
        ++blocks;
        S->progressed = true;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.blocks += blocks;
    S->stats.algorithmic_bytes += moved;
    int active = 0;
    for (auto& kv : S->groups) active += kv.second->active + (kv.second->single ? 1 : 0);
    S->stats.active_columns = active;
    S->stats.pending = (int32_t)S->pending.size();
}

static void scheduler_main(pamg_server* S) {
    try {
        HIP_CHECK(hipSetDevice(S->device));
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(S->mu);
                // nothing to iterate and nothing new: wait for a submission or
                // a finished host phase (requests waiting on a setup cannot run)
                bool busy = false;
                for (auto& kv : S->groups)
                    if (!kv.second->idle()) busy = true;
                bool waiting_only = true;
                for (ServeRequest* q : S->pending)
                    if (!S->setups.count(q->r.op_key)) waiting_only = false;
                if (!busy && waiting_only && S->incoming.empty() && S->setup_done.empty() && S->room_wait.empty() &&
                    !S->stop)
                    S->cv.wait_for(lk, std::chrono::milliseconds(2));
                if (S->stop && S->incoming.empty() && S->pending.empty() && !busy) return;
                while (!S->incoming.empty()) {
                    S->pending.push_back(S->incoming.front());
                    S->incoming.pop_front();
                }
            }
            auto t0 = Clock::now();
            S->progressed = false;
            scheduler_tick(S);
            if (!S->progressed) {
                // blocks in flight, nothing finished yet: poll again shortly
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                continue;
            }
            const double dt = ms_between(t0, Clock::now());
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.busy_ms += dt;
        }
    } catch (const std::exception& e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = e.what();
    }
}

}  // namespace pamg

extern "C" {

int pamg_server_opts_default(pamg_server_opts* o) {
    if (!o) return PAMG_E_INVALID;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget_bytes = 64ull << 30;
    o->block_iters = 4;
    o->precision = PAMG_PREC_F32;
    o->device_setup = 1;
    return PAMG_OK;
}

int pamg_server_estimate_bytes(const pamg_csr* A, int32_t precision, uint64_t* out) {
    return pamg::guarded([&]() -> int {
        if (!A || !out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        *out = pamg::estimate_bytes(*A, precision == PAMG_PREC_F32 ? PAMG_PREC_F32 : PAMG_PREC_F64);
        return PAMG_OK;
    });
}

int pamg_server_create(pamg_context* ctx, const pamg_server_opts* opts, pamg_server** out) {
    return pamg::guarded([&]() -> int {
        if (!out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        *out = nullptr;
        std::unique_ptr<pamg_server> S(new pamg_server());
        if (!ctx) {
            int dev = 0;
            HIP_CHECK(hipGetDevice(&dev));
            ctx = pamg::default_context(dev);
        }
        HIP_CHECK(hipSetDevice(ctx->device));
        S->ctx = ctx;
        if (opts) S->opts = *opts; else pamg_server_opts_default(&S->opts);
        if (S->opts.block_iters < 2) S->opts.block_iters = 2;
        if (S->opts.block_iters & 1) S->opts.block_iters += 1;
        if (S->opts.precision != PAMG_PREC_F32) S->opts.precision = PAMG_PREC_F64;
        if (S->opts.batch_from <= 0) S->opts.batch_from = 4;
        if (S->opts.setup_workers <= 0) S->opts.setup_workers = 1;
        if (S->opts.setup_workers > 16) S->opts.setup_workers = 16;
        if (S->opts.hbm_budget_bytes == 0) throw pamg::Error(PAMG_E_INVALID, "zero HBM budget");
        S->device = ctx->device;
        S->stats.hbm_budget_bytes = S->opts.hbm_budget_bytes;
        ctx->users.fetch_add(1);
        pamg_server* raw = S.release();
        raw->th = std::thread(pamg::scheduler_main, raw);
        const int workers = raw->opts.setup_workers;
        const int cores = pamg::num_threads();
        for (int w = 0; w < workers; ++w)
            raw->setup_th.emplace_back(pamg::setup_main, raw, std::max(1, cores / workers));
        *out = raw;
        return PAMG_OK;
    });
}

int pamg_server_submit(pamg_server* S, const pamg_request* req) {
    return pamg::guarded([&]() -> int {
        if (!S || !req || !req->b_dev || !req->x_dev) throw pamg::Error(PAMG_E_INVALID, "null argument");
        if (!(req->tol >= 0.0)) throw pamg::Error(PAMG_E_INVALID, "bad tolerance");
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->fatal.empty()) throw pamg::Error(PAMG_E_DEVICE, "server stopped: " + S->fatal);
        if (S->stop) throw pamg::Error(PAMG_E_INVALID, "server is shutting down");
        pamg::ServeRequest* q = new pamg::ServeRequest();
        q->r = *req;
        q->t_submit = pamg::Clock::now();
        S->incoming.push_back(q);
        S->stats.submitted += 1;
        S->cv.notify_one();
        return PAMG_OK;
    });
}

int pamg_server_poll(pamg_server* S, pamg_completion* out, int32_t max, int32_t* n_out) {
    return pamg::guarded([&]() -> int {
        if (!S || !n_out || (max > 0 && !out)) throw pamg::Error(PAMG_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(S->mu);
        const int32_t n = (int32_t)std::min<size_t>(S->done.size(), (size_t)std::max(0, max));
        for (int32_t i = 0; i < n; ++i) out[i] = S->done[i];
        S->done.erase(S->done.begin(), S->done.begin() + n);
        *n_out = n;
        if (!S->fatal.empty()) throw pamg::Error(PAMG_E_DEVICE, "server stopped: " + S->fatal);
        return PAMG_OK;
    });
}

int pamg_server_stats_get(pamg_server* S, pamg_server_stats* out) {
    return pamg::guarded([&]() -> int {
        if (!S || !out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(S->mu);
        *out = S->stats;
        return PAMG_OK;
    });
}

int pamg_server_destroy(pamg_server* S) {
    return pamg::guarded([&]() -> int {
        if (!S) return PAMG_OK;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
            S->cv.notify_all();
        }
        if (S->th.joinable()) S->th.join();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->sched_done = true;
            S->setup_cv.notify_all();
        }
        for (auto& t : S->setup_th)
            if (t.joinable()) t.join();
        for (auto& kv : S->setups) delete kv.second;     // every job not yet admitted or failed
        // outstanding requests (only after a fatal error) are dropped
        for (auto* q : S->pending) delete q;
        for (auto* q : S->incoming) delete q;
        for (auto& kv : S->groups) {
            (void)hipStreamSynchronize(kv.second->stream);
            pamg_hierarchy_destroy(kv.second->h);
            release_streams(kv.second);
            for (auto* q : kv.second->col) delete q;
            delete kv.second->single;
            delete kv.second;
        }
        S->ctx->users.fetch_sub(1);
        delete S;
        return PAMG_OK;
    });
}

}  // extern "C"
