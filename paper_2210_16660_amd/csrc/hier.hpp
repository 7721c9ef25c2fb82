// Internal device-side structures shared by the single- and multi-RHS drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

#define HIP_CHECK(call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            throw ::pamg::Error(e_ == hipErrorOutOfMemory ? PAMG_E_OOM : PAMG_E_DEVICE,              \
                                std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

// Device and allocator of a family of hierarchies, engines and servers.
struct pamg_context {
    int device = 0;
    pamg_allocator a{};                     // a.alloc == nullptr: hipMalloc / hipFree
    std::atomic<uint64_t> allocs{0}, frees{0}, failed{0}, live{0}, peak{0};
    std::atomic<int> users{0};
};

namespace pamg {

// A device buffer and its size, as the context handed it out.
struct DevAlloc {
    void* p;
    size_t bytes;
};

// The per-device context of callers that pass none (hipMalloc / hipFree;
// created on first use, kept until the process ends).
pamg_context* default_context(int device);
// bytes (> 0) from the context's allocator for use on stream s; throws
// PAMG_E_OOM when the allocator fails.
void* ctx_alloc(pamg_context* c, size_t bytes, hipStream_t s);
void ctx_free(pamg_context* c, void* p, size_t bytes, hipStream_t s);
// Free a list of buffers (the device must be idle) and clear it.
void ctx_free_all(pamg_context* c, std::vector<DevAlloc>& list);

template <typename T>
struct DevVals {
    bool built = false;
    std::vector<T*> v, vd, dinv, p;   // per level (vd, p for l < L)
    std::vector<T*> r, zp;            // V-cycle workspace: r_l (l >= 1), zp_l (l < L)
    std::vector<T*> gsa, zt;          // hybrid GS: 1 / a_ii and a second iterate buffer (l < L)
    std::vector<T*> gst;              // hybrid GS: residual of the old iterate (l < L)
    std::vector<T*> sa_pv, sa_tv;     // smoothed prolongator: values of P and P^T (l < L)
    T* zc = nullptr;                  // hybrid GS: coarsest-level solution
    T* ainv = nullptr;                // dense A_L^{-1}
    T* dbg_in = nullptr;              // scratch in this precision (max n)
    T* dbg_in2 = nullptr;
};

struct BatchEngine;
void destroy_batch(BatchEngine* b);
struct BatchDeleter {
    void operator()(BatchEngine* b) const { destroy_batch(b); }
};

// A matrix in the tile kernels' layout (row tiles, column dictionaries):
// the smoothed prolongator's P and P^T.
struct DevTiled {
    const int *rp = nullptr, *ci = nullptr;
    const int4* tiles = nullptr;
    int ntiles = 0, items = 1;
    const int2* span = nullptr;
    const int* col = nullptr;
    const uint16_t* loc = nullptr;
    int dmax = 1;                       // longest dictionary
};

struct DevLevelIdx {
    int n = 0, nc = 0, items = 8;
    int max_agg = 0;                    // most rows in one aggregate of this level (l < L)
    long long nnz = 0;
    int *rp = nullptr, *ci = nullptr, *aggptr = nullptr, *perm = nullptr, *iperm = nullptr;
    const int4 *down_tiles = nullptr, *up_tiles = nullptr;
    int n_down = 0, n_up = 0;
    // tile column dictionaries (per tile: first entry, length; the columns;
    // per matrix entry: its 16-bit position in its tile's dictionary)
    const int2 *up_span = nullptr, *down_span = nullptr;
    const int *up_col = nullptr, *down_col = nullptr;
    const uint16_t *up_loc = nullptr, *down_loc = nullptr;
    int up_dmax = 1, down_dmax = 1;     // longest dictionary (dynamic LDS of the tile kernels)
    long long up_dlen = 0, down_dlen = 0;  // total dictionary entries
    // hybrid Gauss-Seidel schedule (l < L): per-row depths, per-block largest depths
    const uint8_t *gs_df = nullptr, *gs_db = nullptr;
    const int* gs_maxd = nullptr;
    const int2* gs_fresh = nullptr;     // per row: first in-block entry, counts (GsLevel::fresh)
    int gs_nblk = 0;
    // smoothed prolongator (l < L): P and P^T patterns, hierarchical numbering
    DevTiled sa_p, sa_t;
    long long sa_nnz = 0;
};

// Coefficient-only reuse: built on the first value update and kept.  Its
// device arrays belong to the hierarchy's allocation list.
struct ReusePlan {
    int npw = 0;                          // pairwise levels (composition condenses them)
    std::vector<long long> nnz;           // entries of each pairwise level
    std::vector<double*> vcan;            // each pairwise level's values, canonical CSR order
    std::vector<int*> gptr, gk;           // Galerkin plan of each pairwise step m -> m+1
    std::vector<double*> gpp;
    std::vector<int> kept_pw;             // pairwise level of each kept level
    std::vector<int*> crp;                // canonical row pointer of each kept level
    std::vector<int*> hperm;              // device CSR entry -> canonical entry, each kept level
    std::vector<double*> dcan;            // canonical l1 inverse diagonal, each kept level
    int* dpos0 = nullptr;                 // canonical position of each diagonal entry of A_0
    int* flag = nullptr;
    double plan_ms = 0.0;
};

}  // namespace pamg

struct pamg_hierarchy {
    pamg_context* ctx = nullptr;
    int device = 0;
    int L = 0;
    bool host_only = false;
    int smoother = PAMG_SMOOTHER_L1_JACOBI;   // hybrid GS: sweeps per side, block size, damping
    int sweeps = 1, gs_block = 256;
    double omega = 1.0;
    bool smoothed_p = false;                  // smoothed prolongators (general sparse P)
    std::vector<pamg::DevLevelIdx> idx;
    pamg::DevVals<double> f64;
    pamg::DevVals<float> f32;
    double *x = nullptr, *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr, *b = nullptr;
    double *dbg0 = nullptr, *dbg1 = nullptr, *dbg2 = nullptr;
    float* r32 = nullptr;             // FP32 cycle: the level-0 residual rounded to FP32 (n0; build_f32)
    float* z32 = nullptr;             // FP32 cycle: its output z, exactly, for the Krylov pass (n0; build_f32)
    double *partial = nullptr, *partial_b = nullptr;
    int* zero_flag = nullptr;
    pamg::SolveState* st = nullptr;
    pamg::SolveState* st_host = nullptr;   // pinned
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int graph_k[2][2] = {{0, 0}, {0, 0}};
    std::vector<pamg::DevAlloc> allocs;
    pamg::HostHierarchy host;
    int lazy_levels = 0;                      // finest levels built on the device: host copies made on first use
    pamg_params prm{};                        // the setup's parameters (device-built hierarchies)
    std::mutex host_mu;
    pamg_hier_info info{};
    std::mutex mu;
    std::unique_ptr<pamg::BatchEngine, pamg::BatchDeleter> batch[2];   // multi-RHS workspaces (FP64 / FP32 V-cycle)
    std::vector<int> batch_cfg_down[2], batch_cfg_up[2];   // their tuned kernel variants, kept across engines
    std::unique_ptr<pamg::ReusePlan> reuse;   // coefficient-only updates
    bool values_updated = false;              // host copies of the values are stale
};

namespace pamg {

// A device array of the hierarchy (freed with it), from its context.
template <typename T>
inline T* dalloc(pamg_hierarchy* h, size_t count, hipStream_t s = nullptr) {
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    void* p = ctx_alloc(h->ctx, bytes, s);
    h->allocs.push_back({p, bytes});
    h->info.device_bytes += bytes;
    return static_cast<T*>(p);
}

inline int vec_grid(long long n) {
    long long g = (n + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    return g < 1 ? 1 : (int)g;
}
void require_device(const pamg_hierarchy* h);

// Setup in two phases: the host phase (validation, hierarchy, layout) needs
// no device; the device phase uploads it, factorizes the coarsest level and
// returns the hierarchy (or, with host_only, keeps it on the host).
struct HostBuild {
    HostHierarchy H;
    std::vector<LayoutLevel> lay;
    pamg_params prm{};
    double host_ms = 0.0;
};
std::unique_ptr<HostBuild> host_build(const pamg_csr& A, const pamg_params& prm);
int coarsest_n(const HostBuild& b);
// ctx: the context the hierarchy allocates from (null: the current device's default)
pamg_hierarchy* finish_build(std::unique_ptr<HostBuild> b, hipStream_t stream, pamg_context* ctx);
// The hierarchy with its large levels built on the device, or null when the
// device construction does not apply (prm already checked; A's rows are
// validated on the device, as validate_csr would).
pamg_hierarchy* device_setup_build(const pamg_csr& A, const pamg_params& prm, hipStream_t stream, pamg_context* ctx);
// Host copies (canonical numbering) of the device-built levels, made once
// from the device arrays: matrix, l1 inverse diagonal, aggregates and
// prolongator entries (no near-null vector).
void ensure_host_levels(pamg_hierarchy* h);
void check_params(const pamg_params& prm);

// Dense limit of the coarsest level (its FP64 inverse is n_L^2 doubles).
constexpr int kMaxDense = 8192;
// A_L^{-1} (FP64, n x n row-major, symmetric) of the coarsest level from its
// device CSR: Cholesky and inverse on the matrix cores (dense.hip).  Throws
// PAMG_E_NOT_SPD on a non-positive pivot.  Synchronizes the stream.
// Device workspace of the dense factorization of an n-row coarsest level,
// from the context (allocated before anything it is used for is changed).
struct DenseWork {
    pamg_context* ctx = nullptr;
    std::vector<DevAlloc> bufs;
    double *M = nullptr, *X = nullptr, *D = nullptr;
    int* flag = nullptr;
    ~DenseWork() {
        if (ctx) ctx_free_all(ctx, bufs);
    }
};
std::unique_ptr<DenseWork> dense_work(pamg_context* ctx, int n, hipStream_t s);
void coarse_inverse_device(DenseWork& w, int n, const int* rp, const int* ci, const double* v, double* ainv,
                           hipStream_t s);
// Single-right-hand-side FCG (x0 = 0) in steps on a caller's stream, with the
// arithmetic of pamg_solve: begin, blocks of k iterations each followed by an
// asynchronous copy of the state to its host copy, the true residual and a
// restart from it, and the result in the caller's numbering (synchronizes).
void single_begin(pamg_hierarchy* h, const double* b, double tol, int maxit, hipStream_t s);
void single_block(pamg_hierarchy* h, int prec, int k, bool use_graph, hipStream_t s);
void single_prepare_graph(pamg_hierarchy* h, int prec, int k);   // capture only, no launch
const SolveState& single_state(const pamg_hierarchy* h);
double single_true_relres(pamg_hierarchy* h, hipStream_t s);
void single_restart(pamg_hierarchy* h, hipStream_t s);
void single_end(pamg_hierarchy* h, double* x, hipStream_t s);
uint64_t single_iteration_bytes(const pamg_hierarchy* h, int prec);
// Canonical values of a kept level after a coefficient-only update (reuse.hip).
void updated_level_values(const pamg_hierarchy* h, int level, double* v);
}  // namespace pamg

namespace pamg {
// Run an entry point body: C++ exceptions become status codes plus the
// thread-local message.
template <class F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return PAMG_E_OOM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return PAMG_E_DEVICE;
    }
}
}  // namespace pamg
