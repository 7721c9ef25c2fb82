// Multi-right-hand-side solves: up to 16 independent FCG/PCG recurrences
// share every pass over the hierarchy's matrices.  The engine owns the
// n x 16 work vectors of one V-cycle precision, the per-level kernel variants
// chosen by the autotuner, and a HIP graph of one block of iterations.
// Columns can be loaded and retired between blocks (the serving loop uses
// this); a column's arithmetic never depends on the other columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "batch.hpp"

namespace pamg {

// The 16-column engine runs the l1-Jacobi V-cycle with tentative prolongators only.
static void require_l1_smoother(const pamg_hierarchy* h) {
    if (h->smoother != PAMG_SMOOTHER_L1_JACOBI)
        throw Error(PAMG_E_INVALID, "batched solves support the l1-Jacobi smoother only");
    if (h->smoothed_p) throw Error(PAMG_E_INVALID, "batched solves support tentative prolongators only");
}

// kernel variants tried by the autotuner: unroll depth (entries of a row
// whose loads are in flight together) x columns per lane (1, 2 or 4)
constexpr int kNumVariants = 15;
static inline int variant_unroll(int v) { return 1 << (v % 5); }
static inline int variant_cpl(int v) { return v < 5 ? 1 : v < 10 ? 2 : 4; }

template <typename F>
static void with_variant(int v, F&& f) {
    using std::integral_constant;
    switch (v) {
        case 0: f(integral_constant<int, 1>{}, integral_constant<int, 1>{}); break;
        case 1: f(integral_constant<int, 2>{}, integral_constant<int, 1>{}); break;
        case 2: f(integral_constant<int, 4>{}, integral_constant<int, 1>{}); break;
        case 3: f(integral_constant<int, 8>{}, integral_constant<int, 1>{}); break;
        case 4: f(integral_constant<int, 16>{}, integral_constant<int, 1>{}); break;
        case 5: f(integral_constant<int, 1>{}, integral_constant<int, 2>{}); break;
        case 6: f(integral_constant<int, 2>{}, integral_constant<int, 2>{}); break;
        case 7: f(integral_constant<int, 4>{}, integral_constant<int, 2>{}); break;
        case 8: f(integral_constant<int, 8>{}, integral_constant<int, 2>{}); break;
        case 9: f(integral_constant<int, 16>{}, integral_constant<int, 2>{}); break;
        case 10: f(integral_constant<int, 1>{}, integral_constant<int, 4>{}); break;
        case 11: f(integral_constant<int, 2>{}, integral_constant<int, 4>{}); break;
        case 12: f(integral_constant<int, 4>{}, integral_constant<int, 4>{}); break;
        case 13: f(integral_constant<int, 8>{}, integral_constant<int, 4>{}); break;
        default: f(integral_constant<int, 16>{}, integral_constant<int, 4>{}); break;
    }
}

struct BatchEngine {
    pamg_hierarchy* h = nullptr;
    int prec = 0;
    std::vector<void*> r, zp;                 // V-cycle vectors per level (n_l x 16, V-cycle precision)
    void* zc = nullptr;                       // coarse result scratch (n_L x 16)
    double *X = nullptr, *R = nullptr, *Z = nullptr, *P[2] = {nullptr, nullptr}, *Q = nullptr, *B = nullptr,
           *Y = nullptr;
    float* R32 = nullptr;                     // FP32 V-cycle: R rounded once per cycle for level 0
    float* Z32 = nullptr;                     // FP32 V-cycle (L >= 1): its result z, exact in FP32
    double *partial = nullptr, *partial_b = nullptr;
    BatchState* st = nullptr;
    BatchState* st_host = nullptr;            // pinned
    const double** src_dev = nullptr;         // kW column pointers (device copy)
    double** dst_dev = nullptr;
    void** ptr_host = nullptr;                // pinned staging for the pointer tables (2 * kW)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_k[2] = {0, 0};
    std::vector<int> cfg_down, cfg_up;        // variant per level
    std::vector<DevAlloc> allocs;             // from the hierarchy's context
    uint64_t bytes = 0;
};

void destroy_batch(BatchEngine* E) {
    if (!E) return;
    (void)hipDeviceSynchronize();
    for (auto& g : E->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (E->cap_stream) (void)hipStreamDestroy(E->cap_stream);
    if (E->h) ctx_free_all(E->h->ctx, E->allocs);
    if (E->st_host) (void)hipHostFree(E->st_host);
    if (E->ptr_host) (void)hipHostFree(E->ptr_host);
    delete E;
}

template <typename T>
static T* balloc(BatchEngine* E, size_t count, hipStream_t s) {
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    void* p = ctx_alloc(E->h->ctx, bytes, s);
    E->allocs.push_back({p, bytes});
    E->bytes += bytes;
    HIP_CHECK(hipMemsetAsync(p, 0, bytes, s));
    return static_cast<T*>(p);
}

// ---------------------------------------------------------------- schedule

template <typename T>
static void launch_down_b(const DevLevelIdx& I, int v, const T* vd, const void* r, bool r_is_f64, const T* p, T* rc,
                          const int* done, hipStream_t s) {
    with_variant(v, [&](auto u, auto c) {
        constexpr int U = decltype(u)::value, CPL = decltype(c)::value;
        const int grid = unit_grid(I.nc, kBlock / (kW / CPL));
        if (r_is_f64)
            hipLaunchKernelGGL((kb_down<U, CPL, T, double>), dim3(grid), dim3(kBlock), 0, s, I.nc, (const int*)I.rp,
                               (const int*)I.ci, vd, (const double*)r, p, (const int*)I.aggptr, rc, done);
        else
            hipLaunchKernelGGL((kb_down<U, CPL, T, T>), dim3(grid), dim3(kBlock), 0, s, I.nc, (const int*)I.rp,
                               (const int*)I.ci, vd, (const T*)r, p, (const int*)I.aggptr, rc, done);
    });
}

template <typename T>
static void launch_up_b(const DevLevelIdx& I, const DevLevelIdx& F, int v, const T* av, const T* zp, const T* r,
                        const T* dinv, const void* r_f, bool rf_is_f64, const T* dinv_f, const T* p_f, T* zp_f,
                        const int* done, hipStream_t s) {
    with_variant(v, [&](auto u, auto c) {
        constexpr int U = decltype(u)::value, CPL = decltype(c)::value;
        const int grid = unit_grid(I.n, kBlock / (kW / CPL));
        if (rf_is_f64)
            hipLaunchKernelGGL((kb_up<U, CPL, T, T, double>), dim3(grid), dim3(kBlock), 0, s, I.n, (const int*)I.rp,
                               (const int*)I.ci, av, zp, r, dinv, (const int*)F.aggptr, (const double*)r_f, dinv_f,
                               p_f, zp_f, done);
        else
            hipLaunchKernelGGL((kb_up<U, CPL, T, T, T>), dim3(grid), dim3(kBlock), 0, s, I.n, (const int*)I.rp,
                               (const int*)I.ci, av, zp, r, dinv, (const int*)F.aggptr, (const T*)r_f, dinv_f, p_f,
                               zp_f, done);
    });
}

// z = B r (E->R), per column; partials of z . dv.  Returns their count.  z is
// E->Z, or E->Z32 with the FP32 cycle on a hierarchy of several levels (the
// cycle's last step computes it in FP32).
// The level-0 right-hand side as the V-cycle reads it: with the FP32 cycle,
// R rounded to FP32 (the kernels would round each load the same way), so
// that its gathers move 64-byte lines instead of 128-byte ones; every kernel
// that writes R (load, update, true-residual restart) writes R32 beside it.
template <typename T>
static const void* level0_rhs(BatchEngine* E, const int* done, hipStream_t s) {
    (void)done;
    (void)s;
    if constexpr (std::is_same<T, float>::value)
        return E->R32;
    else
        return E->R;
}

template <typename T>
static int enqueue_vcycle_b(BatchEngine* E, DevVals<T>& V, const double* dv, const int* done, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const int L = h->L;
    constexpr bool r0_f64 = std::is_same<T, double>::value;
    const void* r0 = L > 0 ? level0_rhs<T>(E, done, s) : E->R;
    for (int l = 0; l < L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        if (l == 0)
            launch_down_b<T>(I, E->cfg_down[0], V.vd[0], r0, r0_f64, V.p[0], (T*)E->r[1], done, s);
        else
            launch_down_b<T>(I, E->cfg_down[l], V.vd[l], E->r[l], false, V.p[l], (T*)E->r[l + 1], done, s);
    }
    const int nL = h->idx[L].n;
    if (L == 0) {
        hipLaunchKernelGGL((kb_coarse<T, double, double, true>), dim3(1), dim3(kCoarseThreads), 0, s, nL,
                           (const T*)V.ainv, (const double*)E->R, (T*)E->zc, (const int*)nullptr,
                           (const double*)nullptr, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, E->Z, dv,
                           E->partial, done);
        return 1;
    }
    const DevLevelIdx& F = h->idx[L - 1];
    if (nL > coarse_rows_min_b<T>()) {
        const dim3 g(coarse_rows_grid_b<T>(nL));
        if (L - 1 == 0)
            hipLaunchKernelGGL((kb_coarse_rows<T, T, double>), g, dim3(kBlock), 0, s, nL, (const T*)V.ainv,
                               (const T*)E->r[L], (const int*)F.aggptr, (const double*)E->R, (const T*)V.dinv[0],
                               (const T*)V.p[0], (T*)E->zp[0], (double*)nullptr, done);
        else
            hipLaunchKernelGGL((kb_coarse_rows<T, T, T>), g, dim3(kBlock), 0, s, nL, (const T*)V.ainv,
                               (const T*)E->r[L], (const int*)F.aggptr, (const T*)E->r[L - 1],
                               (const T*)V.dinv[L - 1], (const T*)V.p[L - 1], (T*)E->zp[L - 1], (double*)nullptr,
                               done);
    } else if (L - 1 == 0)
        hipLaunchKernelGGL((kb_coarse<T, T, double, false>), dim3(1), dim3(kCoarseThreads), 0, s, nL,
                           (const T*)V.ainv, (const T*)E->r[L], (T*)E->zc, (const int*)F.aggptr, (const double*)E->R,
                           (const T*)V.dinv[0], (const T*)V.p[0], (T*)E->zp[0], (double*)nullptr,
                           (const double*)nullptr, (double*)nullptr, done);
    else
        hipLaunchKernelGGL((kb_coarse<T, T, T, false>), dim3(1), dim3(kCoarseThreads), 0, s, nL, (const T*)V.ainv,
                           (const T*)E->r[L], (T*)E->zc, (const int*)F.aggptr, (const T*)E->r[L - 1],
                           (const T*)V.dinv[L - 1], (const T*)V.p[L - 1], (T*)E->zp[L - 1], (double*)nullptr,
                           (const double*)nullptr, (double*)nullptr, done);
    for (int l = L - 1; l >= 1; --l) {
        const DevLevelIdx& I = h->idx[l];
        const DevLevelIdx& Fi = h->idx[l - 1];
        if (l - 1 == 0)
            launch_up_b<T>(I, Fi, E->cfg_up[l], V.v[l], (const T*)E->zp[l], (const T*)E->r[l], V.dinv[l], r0, r0_f64,
                           V.dinv[0], V.p[0], (T*)E->zp[0], done, s);
        else
            launch_up_b<T>(I, Fi, E->cfg_up[l], V.v[l], (const T*)E->zp[l], (const T*)E->r[l], V.dinv[l],
                           E->r[l - 1], false, V.dinv[l - 1], V.p[l - 1], (T*)E->zp[l - 1], done, s);
    }
    const DevLevelIdx& I0 = h->idx[0];
    const int g = unit_grid(I0.n, up0_rows_per_block<T>());
    T* zout;
    if constexpr (std::is_same<T, float>::value) zout = E->Z32; else zout = E->Z;
    hipLaunchKernelGGL((kb_up0<T>), dim3(g), dim3(kBlock), 0, s, I0.n, (const int*)I0.rp, (const int*)I0.ci,
                       (const T*)V.v[0], (const T*)E->zp[0], (const T*)r0, (const T*)V.dinv[0], zout, dv,
                       E->partial, done);
    return g;
}

template <typename T>
static void enqueue_iteration_b(BatchEngine* E, DevVals<T>& V, int krylov, int parity, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const int* done = &E->st->all_done;
    const double* dv = (krylov == PAMG_KRYLOV_CG) ? E->R : E->Q;
    const int cnt = enqueue_vcycle_b<T>(E, V, dv, done, s);
    hipLaunchKernelGGL(kb_fin_beta, dim3(1), dim3(kFinThreads), 0, s, E->st, (const double*)E->partial, cnt);
    const DevLevelIdx& I0 = h->idx[0];
    const int gk = unit_grid(I0.n, kKrylovRowsPerBlock);
    if (std::is_same<T, float>::value && h->L > 0)
        hipLaunchKernelGGL(kb_krylov_pq<float>, dim3(gk), dim3(kBlock), 0, s, I0.n, (const int*)I0.rp,
                           (const int*)I0.ci, (const double*)h->f64.v[0], (const float*)E->Z32,
                           (const double*)E->P[parity], E->P[1 - parity], E->Q, (const double*)E->R,
                           (const BatchState*)E->st, E->partial, done);
    else
        hipLaunchKernelGGL(kb_krylov_pq<double>, dim3(gk), dim3(kBlock), 0, s, I0.n, (const int*)I0.rp,
                           (const int*)I0.ci, (const double*)h->f64.v[0], (const double*)E->Z,
                           (const double*)E->P[parity], E->P[1 - parity], E->Q, (const double*)E->R,
                           (const BatchState*)E->st, E->partial, done);
    hipLaunchKernelGGL(kb_fin_alpha, dim3(1), dim3(kFinThreads), 0, s, E->st, (const double*)E->partial, gk);
    const int g = unit_grid(I0.n, kBlock / kW);
    hipLaunchKernelGGL(kb_update, dim3(g), dim3(kBlock), 0, s, I0.n, E->X, E->R, E->R32,
                       (const double*)E->P[1 - parity], (const double*)E->Q, (const BatchState*)E->st, E->partial,
                       done);
    hipLaunchKernelGGL(kb_fin_norm, dim3(1), dim3(kFinThreads), 0, s, E->st, (const double*)E->partial, g);
}

template <typename T>
static void enqueue_block_b(BatchEngine* E, DevVals<T>& V, int krylov, int k, hipStream_t s) {
    for (int j = 0; j < k; ++j) enqueue_iteration_b<T>(E, V, krylov, j & 1, s);
}

// ---------------------------------------------------------------- autotuner

template <typename F>
static float time_variant(F&& launch, hipStream_t s) {
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    launch();
    HIP_CHECK(hipEventRecord(e0, s));
    for (int i = 0; i < 3; ++i) launch();
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

// Pick, per level, the fastest down-sweep and up-sweep variant (unroll depth
// x columns per lane) by timing each on the real level.  The variants do not
// change any column's arithmetic, only how it is scheduled.
template <typename T>
static void autotune(BatchEngine* E, DevVals<T>& V, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const int L = h->L;
    const int* nodone = h->zero_flag;
    E->cfg_down.assign(L + 1, 2);              // unroll 4, one column per lane until tuned
    E->cfg_up.assign(L + 1, 2);
    constexpr bool r0_f64 = std::is_same<T, double>::value;
    const void* r0 = L > 0 ? level0_rhs<T>(E, nodone, s) : E->R;
    for (int l = 0; l < L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        float best = 1e30f;
        for (int v = 0; v < kNumVariants; ++v) {
            const float t = time_variant([&]() {
                if (l == 0)
                    launch_down_b<T>(I, v, V.vd[0], r0, r0_f64, V.p[0], (T*)E->r[1], nodone, s);
                else
                    launch_down_b<T>(I, v, V.vd[l], E->r[l], false, V.p[l], (T*)E->r[l + 1], nodone, s);
            }, s);
            if (t < best) { best = t; E->cfg_down[l] = v; }
        }
        if (l == 0) continue;
        const DevLevelIdx& Fi = h->idx[l - 1];
        best = 1e30f;
        for (int v = 0; v < kNumVariants; ++v) {
            const float t = time_variant([&]() {
                if (l - 1 == 0)
                    launch_up_b<T>(I, Fi, v, V.v[l], (const T*)E->zp[l], (const T*)E->r[l], V.dinv[l], r0, r0_f64,
                                   V.dinv[0], V.p[0], (T*)E->zp[0], nodone, s);
                else
                    launch_up_b<T>(I, Fi, v, V.v[l], (const T*)E->zp[l], (const T*)E->r[l], V.dinv[l], E->r[l - 1],
                                   false, V.dinv[l - 1], V.p[l - 1], (T*)E->zp[l - 1], nodone, s);
            }, s);
            if (t < best) { best = t; E->cfg_up[l] = v; }
        }
    }
}

// ---------------------------------------------------------------- engine

template <typename T>
static BatchEngine* create_engine(pamg_hierarchy* h, DevVals<T>& V, int prec, hipStream_t s) {
    std::unique_ptr<BatchEngine, BatchDeleter> E(new BatchEngine());
    E->h = h;
    E->prec = prec;
    const int L = h->L;
    E->r.assign(L + 1, nullptr);
    E->zp.assign(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) {
        const size_t n = (size_t)h->idx[l].n * kW;
        if (l >= 1) E->r[l] = balloc<T>(E.get(), n, s);
        if (l < L) E->zp[l] = balloc<T>(E.get(), n, s);
    }
    E->zc = balloc<T>(E.get(), (size_t)h->idx[L].n * kW, s);
    const size_t n0 = (size_t)h->idx[0].n * kW;
    E->X = balloc<double>(E.get(), n0, s);
    E->R = balloc<double>(E.get(), n0, s);
    if (std::is_same<T, float>::value) {
        E->R32 = balloc<float>(E.get(), n0, s);
        E->Z32 = balloc<float>(E.get(), n0, s);
    }
    E->Z = balloc<double>(E.get(), n0, s);
    E->P[0] = balloc<double>(E.get(), n0, s);
    E->P[1] = balloc<double>(E.get(), n0, s);
    E->Q = balloc<double>(E.get(), n0, s);
    E->B = balloc<double>(E.get(), n0, s);
    E->Y = balloc<double>(E.get(), n0, s);
    E->partial = balloc<double>(E.get(), (size_t)kMaxGrid * kW * 2, s);
    E->partial_b = balloc<double>(E.get(), (size_t)kMaxGrid * kW * 2, s);
    E->st = balloc<BatchState>(E.get(), 1, s);
    E->src_dev = (const double**)balloc<void*>(E.get(), kW, s);
    E->dst_dev = (double**)balloc<void*>(E.get(), kW, s);
    HIP_CHECK(hipHostMalloc((void**)&E->st_host, sizeof(BatchState), hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void**)&E->ptr_host, 2 * kW * sizeof(void*), hipHostMallocDefault));
    HIP_CHECK(hipStreamCreateWithFlags(&E->cap_stream, hipStreamNonBlocking));
    // every column starts inactive
    std::memset(E->st_host, 0, sizeof(BatchState));
    for (int c = 0; c < kW; ++c) E->st_host->col[c].done = 1;
    E->st_host->all_done = 1;
    HIP_CHECK(hipMemcpyAsync(E->st, E->st_host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (!h->batch_cfg_down[prec].empty()) {
        // variants tuned for an earlier engine of this hierarchy
        E->cfg_down = h->batch_cfg_down[prec];
        E->cfg_up = h->batch_cfg_up[prec];
    } else {
        autotune<T>(E.get(), V, s);
        HIP_CHECK(hipStreamSynchronize(s));
        h->batch_cfg_down[prec] = E->cfg_down;
        h->batch_cfg_up[prec] = E->cfg_up;
    }
    return E.release();
}

BatchEngine* get_engine(pamg_hierarchy* h, int prec, hipStream_t s) {
    auto& slot = h->batch[prec];
    if (!slot) {
        if (prec == PAMG_PREC_F32) {
            if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built (set params.build_f32)");
            slot.reset(create_engine<float>(h, h->f32, prec, s));
        } else {
            slot.reset(create_engine<double>(h, h->f64, prec, s));
        }
    }
    return slot.get();
}

static hipGraphExec_t block_graph(BatchEngine* E, int krylov, int k) {
    hipGraphExec_t& ex = E->graph[krylov];
    if (ex && E->graph_k[krylov] == k) return ex;
    if (ex) {
        HIP_CHECK(hipGraphExecDestroy(ex));
        ex = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamBeginCapture(E->cap_stream, hipStreamCaptureModeThreadLocal));
    if (E->prec == PAMG_PREC_F32)
        enqueue_block_b<float>(E, E->h->f32, krylov, k, E->cap_stream);
    else
        enqueue_block_b<double>(E, E->h->f64, krylov, k, E->cap_stream);
    HIP_CHECK(hipStreamEndCapture(E->cap_stream, &g));
    HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    HIP_CHECK(hipGraphDestroy(g));
    E->graph_k[krylov] = k;
    return ex;
}

void batch_prepare_graph(BatchEngine* E, int krylov, int k) { (void)block_graph(E, krylov, k); }

void release_engine(pamg_hierarchy* h, int prec) { h->batch[prec].reset(); }   // destroy_batch synchronizes

// Device bytes of the 16-column engine of h (the allocations create_engine makes).
uint64_t engine_bytes(const pamg_hierarchy* h, int prec) {
    const uint64_t s = prec == PAMG_PREC_F32 ? 4 : 8;
    const int L = h->L;
    uint64_t b = 0;
    for (int l = 0; l <= L; ++l) {
        const uint64_t n = (uint64_t)h->idx[l].n * kW;
        if (l >= 1) b += n * s;
        if (l < L) b += n * s;
    }
    const uint64_t n0 = (uint64_t)h->idx[0].n * kW;
    b += (uint64_t)h->idx[L].n * kW * s + 8 * n0 * 8 + (prec == PAMG_PREC_F32 ? 2 * n0 * 4 : 0);
    b += 2 * (uint64_t)kMaxGrid * kW * 2 * 8 + sizeof(BatchState) + 2 * kW * sizeof(void*);
    return b;
}

// One block of k iterations (graph replay or direct launches).
void batch_run_block(BatchEngine* E, int krylov, int k, bool use_graph, hipStream_t s) {
    if (use_graph) {
        HIP_CHECK(hipGraphLaunch(block_graph(E, krylov, k), s));
    } else if (E->prec == PAMG_PREC_F32) {
        enqueue_block_b<float>(E, E->h->f32, krylov, k, s);
    } else {
        enqueue_block_b<double>(E, E->h->f64, krylov, k, s);
    }
}

void batch_read_state(BatchEngine* E, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(E->st_host, E->st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

void batch_read_state_async(BatchEngine* E, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(E->st_host, E->st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
}

void batch_write_state(BatchEngine* E, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(E->st, E->st_host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

// Load the columns whose src[c] is non-null (caller-order device vectors):
// b into B, x = 0, r = b, then start their recurrences.  The host copy of
// the state must be current (batch_read_state) and is written back with the
// new columns' parameters.
void batch_load(BatchEngine* E, const double* const* src, const double* tol, const int* maxit, const int* fixed,
                int krylov, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const DevLevelIdx& I0 = h->idx[0];
    int mask = 0;
    for (int c = 0; c < kW; ++c) {
        E->ptr_host[c] = (void*)src[c];
        if (src[c]) {
            mask |= 1 << c;
            BatchCol& C = E->st_host->col[c];
            std::memset(&C, 0, sizeof(C));
            C.tol = tol[c];
            C.maxit = maxit[c];
            C.fixed_iters = fixed[c];
            C.done = 1;          // inactive until kb_fin_init starts it
        }
    }
    E->st_host->krylov = krylov;
    E->st_host->all_done = 0;
    HIP_CHECK(hipMemcpyAsync(E->st, E->st_host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync((void*)E->src_dev, E->ptr_host, kW * sizeof(void*), hipMemcpyHostToDevice, s));
    const int g = std::min(kMaxGrid, std::max(1, (I0.n + 15) / 16));
    hipLaunchKernelGGL(kb_load, dim3(g), dim3(kBlock), 0, s, I0.n, (const int*)I0.iperm,
                       (const double* const*)E->src_dev, E->B, E->R, E->R32, E->X, E->partial_b);
    hipLaunchKernelGGL(kb_fin_init, dim3(1), dim3(kFinThreads), 0, s, E->st, (const double*)E->partial_b, g,
                       (const double*)E->partial_b, g, mask);
    HIP_CHECK(hipGetLastError());
    batch_read_state(E, s);
}

// Copy X[:, c] out (caller order) for the columns whose dst[c] is non-null.
void batch_store(BatchEngine* E, double* const* dst, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const DevLevelIdx& I0 = h->idx[0];
    for (int c = 0; c < kW; ++c) E->ptr_host[kW + c] = (void*)dst[c];
    HIP_CHECK(hipMemcpyAsync((void*)E->dst_dev, E->ptr_host + kW, kW * sizeof(void*), hipMemcpyHostToDevice, s));
    const int g = std::min(kMaxGrid, std::max(1, (I0.n + 15) / 16));
    hipLaunchKernelGGL(kb_store, dim3(g), dim3(kBlock), 0, s, I0.n, (const int*)I0.perm, (double* const*)E->dst_dev,
                       (const double*)E->X, (const BatchState*)E->st);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

// ||b - A x|| / ||b|| of every column; with `restart_mask`, those columns
// also restart their recurrence from the true residual.
void batch_true_residual(BatchEngine* E, int restart_mask, double* relres, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const DevLevelIdx& I0 = h->idx[0];
    const int g = unit_grid(I0.n, kBlock / kW);
    hipLaunchKernelGGL(kb_resid, dim3(g), dim3(kBlock), 0, s, I0.n, (const int*)I0.rp, (const int*)I0.ci,
                       (const double*)h->f64.v[0], (const double*)E->X, (const double*)E->B, E->Y,
                       restart_mask ? E->R : (double*)nullptr, restart_mask ? E->R32 : (float*)nullptr, restart_mask,
                       E->partial_b);
    std::vector<double> part((size_t)g * kW);
    HIP_CHECK(hipMemcpyAsync(part.data(), E->partial_b, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < kW; ++c) {
        double t = 0.0;
        for (int b = 0; b < g; ++b) t += part[(size_t)b * kW + c];
        const double bn = E->st_host->col[c].bnorm;
        relres[c] = bn > 0 ? std::sqrt(t) / bn : 0.0;
    }
    if (restart_mask) {
        hipLaunchKernelGGL(kb_fin_init, dim3(1), dim3(kFinThreads), 0, s, E->st, (const double*)E->partial_b, 0,
                           (const double*)E->partial_b, g, restart_mask);
        HIP_CHECK(hipGetLastError());
        batch_read_state(E, s);
    }
}

int solve_batch(pamg_hierarchy* h, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                const pamg_solve_opts& o, hipStream_t s, pamg_solve_info* infos) {
    require_device(h);
    require_l1_smoother(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    auto t0 = std::chrono::steady_clock::now();
    const int n = h->idx[0].n;
    if (nrhs < 1 || nrhs > kW) throw Error(PAMG_E_INVALID, "nrhs must be in [1, 16]");
    if (ldb < n || ldx < n) throw Error(PAMG_E_INVALID, "ldb and ldx must be >= n");
    if (o.use_x0) throw Error(PAMG_E_INVALID, "batched solves start from x0 = 0");
    const int prec = o.precision == PAMG_PREC_F32 ? PAMG_PREC_F32 : PAMG_PREC_F64;
    const int krylov = o.krylov == PAMG_KRYLOV_CG ? PAMG_KRYLOV_CG : PAMG_KRYLOV_FCG;
    BatchEngine* E = get_engine(h, prec, s);
    batch_read_state(E, s);
    const double* src[kW];
    double tol[kW];
    int maxit[kW], fixed[kW];
    for (int c = 0; c < kW; ++c) {
        src[c] = c < nrhs ? B + (size_t)c * ldb : nullptr;
        tol[c] = o.tol;
        maxit[c] = o.maxit;
        fixed[c] = o.fixed_iters;
        if (c >= nrhs) {          // unused columns stay inactive
            std::memset(&E->st_host->col[c], 0, sizeof(BatchCol));
            E->st_host->col[c].done = 1;
        }
    }
    batch_write_state(E, s);
    batch_load(E, src, tol, maxit, fixed, krylov, s);
    int k = o.check_every > 0 ? o.check_every : 4;
    if (k & 1) ++k;
    int restarts[kW] = {0};
    double relres_true[kW];
    for (int c = 0; c < kW; ++c) relres_true[c] = -1.0;
    for (;;) {
        while (!E->st_host->all_done) {
            batch_run_block(E, krylov, k, o.use_graph != 0, s);
            batch_read_state(E, s);
        }
        const bool want_true = o.true_residual || prec == PAMG_PREC_F32;
        if (!want_true || o.fixed_iters > 0) break;
        double rel[kW];
        batch_true_residual(E, 0, rel, s);
        int mask = 0;
        for (int c = 0; c < nrhs; ++c) {
            const BatchCol& C = E->st_host->col[c];
            relres_true[c] = rel[c];
            if (prec == PAMG_PREC_F32 && C.status == PAMG_OK && C.done == 1 && rel[c] > o.tol && restarts[c] < 10 &&
                C.iter < o.maxit) {
                mask |= 1 << c;
                ++restarts[c];
            }
        }
        if (!mask) break;
        batch_true_residual(E, mask, rel, s);   // r = b - A x for the restarted columns
        for (int c = 0; c < nrhs; ++c)
            if ((mask >> c) & 1) relres_true[c] = -1.0;
    }
    double* dst[kW];
    for (int c = 0; c < kW; ++c) dst[c] = c < nrhs ? X + (size_t)c * ldx : nullptr;
    batch_store(E, dst, s);
    auto t1 = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    int worst = PAMG_OK;
    for (int c = 0; c < nrhs; ++c) {
        const BatchCol& C = E->st_host->col[c];
        if (infos) {
            infos[c].status = C.status;
            infos[c].iterations = C.iter;
            infos[c].restarts = restarts[c];
            infos[c].relres = C.bnorm > 0 ? C.rnorm / C.bnorm : 0.0;
            infos[c].relres_true = relres_true[c];
            infos[c].solve_ms = ms;
        }
        if (C.status < 0 && worst >= 0) worst = C.status;
        else if (C.status == PAMG_NOT_CONVERGED && worst == PAMG_OK) worst = PAMG_NOT_CONVERGED;
    }
    // leave the engine idle for the next call
    for (int c = 0; c < kW; ++c) {
        E->st_host->col[c].active = 0;
        E->st_host->col[c].done = 1;
    }
    E->st_host->all_done = 1;
    batch_write_state(E, s);
    return worst;
}

// Batched operators for parity checks: 16 vectors in, 16 out (caller layout:
// column c at ptr + c*n_level, canonical numbering).
template <typename T>
static void debug_batch_impl(BatchEngine* E, DevVals<T>& V, int op, const double* in, double* out, hipStream_t s) {
    pamg_hierarchy* h = E->h;
    const int L = h->L;
    const int* nodone = h->zero_flag;
    if (op == PAMG_OP_COARSE) {
        const DevLevelIdx& I = h->idx[L];
        const int g = std::min(kMaxGrid, std::max(1, (I.n * kW + kBlock - 1) / kBlock));
        T* rin = L >= 1 ? (T*)E->r[L] : (T*)E->zc;
        hipLaunchKernelGGL((kb_cols_in<T>), dim3(g), dim3(kBlock), 0, s, I.n, (const int*)I.iperm, in, rin);
        // the kernel the cycle runs at this size (a single-level hierarchy
        // always takes the single-workgroup product)
        if (L >= 1 && I.n > coarse_rows_min_b<T>())
            hipLaunchKernelGGL((kb_coarse_rows<T, T, double, true>), dim3(coarse_rows_grid_b<T>(I.n)), dim3(kBlock), 0,
                               s, I.n, (const T*)V.ainv, (const T*)rin, (const int*)nullptr, (const double*)nullptr,
                               (const T*)nullptr, (const T*)nullptr, (T*)nullptr, E->Z, nodone);
        else
            hipLaunchKernelGGL((kb_coarse<T, T, double, true>), dim3(1), dim3(kCoarseThreads), 0, s, I.n,
                               (const T*)V.ainv, (const T*)rin, (T*)E->Y, (const int*)nullptr, (const double*)nullptr,
                               (const T*)nullptr, (const T*)nullptr, (T*)nullptr, E->Z, (const double*)E->Z,
                               E->partial, nodone);
        hipLaunchKernelGGL(kb_cols_out<double>, dim3(g), dim3(kBlock), 0, s, I.n, (const int*)I.perm,
                           (const double*)E->Z, out);
    } else if (op == PAMG_OP_VCYCLE) {
        const DevLevelIdx& I = h->idx[0];
        const int g = std::min(kMaxGrid, std::max(1, (I.n * kW + kBlock - 1) / kBlock));
        hipLaunchKernelGGL((kb_cols_in<double>), dim3(g), dim3(kBlock), 0, s, I.n, (const int*)I.iperm, in, E->R);
        if (E->R32) {
            const long long cnt = (long long)I.n * kW;
            hipLaunchKernelGGL(kb_narrow, dim3(vec_grid(cnt)), dim3(kBlock), 0, s, cnt, (const double*)E->R, E->R32,
                               nodone);
        }
        enqueue_vcycle_b<T>(E, V, E->Q, nodone, s);
        if (std::is_same<T, float>::value && L > 0)
            hipLaunchKernelGGL(kb_cols_out<float>, dim3(g), dim3(kBlock), 0, s, I.n, (const int*)I.perm,
                               (const float*)E->Z32, out);
        else
            hipLaunchKernelGGL(kb_cols_out<double>, dim3(g), dim3(kBlock), 0, s, I.n, (const int*)I.perm,
                               (const double*)E->Z, out);
    } else {
        throw Error(PAMG_E_INVALID, "batched debug operators: COARSE or VCYCLE");
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

void debug_batch(pamg_hierarchy* h, int op, int prec, const double* in, double* out, hipStream_t s) {
    require_device(h);
    require_l1_smoother(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    BatchEngine* E = get_engine(h, prec, s);
    if (prec == PAMG_PREC_F32)
        debug_batch_impl<float>(E, h->f32, op, in, out, s);
    else
        debug_batch_impl<double>(E, h->f64, op, in, out, s);
}

BatchState& batch_state_host(BatchEngine* E) { return *E->st_host; }
const BatchState& batch_state(const BatchEngine* E) { return *E->st_host; }
uint64_t batch_bytes(const BatchEngine* E) { return E->bytes; }

void batch_retire(BatchEngine* E, int mask) {
    for (int c = 0; c < kW; ++c)
        if ((mask >> c) & 1) {
            E->st_host->col[c].active = 0;
            E->st_host->col[c].done = 1;
        }
    int all = 1;
    for (int c = 0; c < kW; ++c)
        if (E->st_host->col[c].active && !E->st_host->col[c].done) all = 0;
    E->st_host->all_done = all;
}

// Variant index of (unroll, columns per lane), or -1.
static int variant_of(int unroll, int cpl) {
    for (int v = 0; v < kNumVariants; ++v)
        if (variant_unroll(v) == unroll && variant_cpl(v) == cpl) return v;
    return -1;
}

void batch_set_config(pamg_hierarchy* h, int prec, const int32_t* cfg) {
    require_device(h);
    require_l1_smoother(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    const int L = h->L;
    std::vector<int> down(L + 1, 2), up(L + 1, 2);
    for (int l = 0; l < L; ++l) {
        down[l] = variant_of(cfg[4 * l + 0], cfg[4 * l + 1]);
        up[l] = l > 0 ? variant_of(cfg[4 * l + 2], cfg[4 * l + 3]) : 2;
        if (down[l] < 0 || up[l] < 0)
            throw Error(PAMG_E_INVALID, "kernel variant must be unroll 1, 2, 4, 8 or 16 with 1, 2 or 4 columns "
                                        "per lane (level " + std::to_string(l) + ")");
    }
    BatchEngine* E = get_engine(h, prec, nullptr);
    HIP_CHECK(hipDeviceSynchronize());
    for (int k = 0; k < 2; ++k)
        if (E->graph[k]) {
            HIP_CHECK(hipGraphExecDestroy(E->graph[k]));
            E->graph[k] = nullptr;
            E->graph_k[k] = 0;
        }
    for (int l = 0; l < L; ++l) {
        E->cfg_down[l] = down[l];
        if (l > 0) E->cfg_up[l] = up[l];
    }
    h->batch_cfg_down[prec] = E->cfg_down;
    h->batch_cfg_up[prec] = E->cfg_up;
}

void batch_config(pamg_hierarchy* h, int prec, int32_t* cfg) {
    require_device(h);
    require_l1_smoother(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    BatchEngine* E = get_engine(h, prec, nullptr);
    const int L = h->L;
    for (int l = 0; l < L; ++l) {
        cfg[4 * l + 0] = variant_unroll(E->cfg_down[l]);
        cfg[4 * l + 1] = variant_cpl(E->cfg_down[l]);
        cfg[4 * l + 2] = l > 0 ? variant_unroll(E->cfg_up[l]) : 8;     // level 0: the fixed-shape kb_up0
        cfg[4 * l + 3] = l > 0 ? variant_cpl(E->cfg_up[l]) : (prec == PAMG_PREC_F32 ? up0_cols<float>() : up0_cols<double>());
    }
}

}  // namespace pamg

extern "C" {

int pamg_solve_batch(pamg_hierarchy* h, int32_t nrhs, const double* B_dev, int64_t ldb, double* X_dev, int64_t ldx,
                     const pamg_solve_opts* opts, void* stream, pamg_solve_info* infos) {
    return pamg::guarded([&]() -> int {
        if (!h || !B_dev || !X_dev) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg_solve_opts o;
        if (opts) o = *opts; else pamg_solve_opts_default(&o);
        if (!(o.tol >= 0.0) || o.maxit < 1 || o.fixed_iters < 0)
            throw pamg::Error(PAMG_E_INVALID, "bad solve options (need tol >= 0, maxit >= 1)");
        return pamg::solve_batch(h, nrhs, B_dev, ldb, X_dev, ldx, o, (hipStream_t)stream, infos);
    });
}

int pamg_debug_apply_batch(pamg_hierarchy* h, int32_t op, int32_t precision, const double* in_dev, double* out_dev,
                           void* stream) {
    return pamg::guarded([&]() -> int {
        if (!h || !in_dev || !out_dev) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg::debug_batch(h, op, precision == PAMG_PREC_F32 ? PAMG_PREC_F32 : PAMG_PREC_F64, in_dev, out_dev,
                          (hipStream_t)stream);
        return PAMG_OK;
    });
}

int pamg_batch_set_config(pamg_hierarchy* h, int32_t precision, const int32_t* cfg) {
    return pamg::guarded([&]() -> int {
        if (!h || !cfg) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg::batch_set_config(h, precision == PAMG_PREC_F32 ? PAMG_PREC_F32 : PAMG_PREC_F64, cfg);
        return PAMG_OK;
    });
}

int pamg_batch_config(pamg_hierarchy* h, int32_t precision, int32_t* cfg) {
    return pamg::guarded([&]() -> int {
        if (!h || !cfg) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg::batch_config(h, precision == PAMG_PREC_F32 ? PAMG_PREC_F32 : PAMG_PREC_F64, cfg);
        return PAMG_OK;
    });
}

}  // extern "C"
