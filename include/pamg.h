/*
 * pamg — PCG/FCG with an aggregation-based AMG V-cycle on one MI355X (gfx950).
 *
 * C ABI.  All entry points return a pamg_status; on a negative status the
 * outputs are untouched and pamg_last_error() describes the failure.  No C++
 * exception crosses this boundary.  Pointers named *_dev are device pointers
 * (hipMalloc'd or from a framework allocator) on the current HIP device;
 * every other pointer is host memory.  `stream` is a hipStream_t (NULL = the
 * default stream); work is enqueued on it and the call returns after the
 * result it reports is known on the host.
 *
 * The method (arXiv 2210.16660, Sec. 3.1 and Sec. 5):
 *   solve A x = b with A symmetric positive definite, by preconditioned CG or
 *   flexible CG, where the preconditioner B is the V-cycle of
 *   eq. (multiplicative_composition) with nu = 1 pre-/post-sweep of the
 *   l1-Jacobi smoother (or, optionally, nu sweeps of the paper's hybrid
 *   forward/backward Gauss-Seidel), tentative piecewise-constant prolongators of
 *   eq. (prolongator) built from a maximum-product matching of the weights
 *   of eq. (weights), Galerkin coarse matrices A_{l+1} = P_l^T A_l P_l, and a
 *   dense direct solve on the coarsest level.  Stopping test: ||r||_2 no
 *   larger than tol * ||b||_2 (Sec. 5).
 */
#ifndef PAMG_H
#define PAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PAMG_OK = 0,
    PAMG_NOT_CONVERGED = 1,   /* warning: outputs valid, maxit reached */
    PAMG_E_INVALID = -1,      /* bad argument or malformed CSR */
    PAMG_E_NOT_SPD = -2,      /* non-positive Cholesky pivot or p.Ap <= 0 */
    PAMG_E_NUMERIC = -3,      /* NaN/Inf met in the iteration */
    PAMG_E_OOM = -4,          /* host or device allocation failed */
    PAMG_E_DEVICE = -5,       /* HIP runtime error */
    PAMG_E_STALLED = -6,      /* coarsening found no pair and the level is too large for the dense solve */
    PAMG_E_BUSY = -7          /* server admission refused (budget / capacity) */
} pamg_status;

enum { PAMG_PREC_F64 = 0, PAMG_PREC_F32 = 1 };   /* storage/arithmetic of the V-cycle */
enum { PAMG_KRYLOV_CG = 0, PAMG_KRYLOV_FCG = 1 };
enum { PAMG_SMOOTHER_L1_JACOBI = 0, PAMG_SMOOTHER_HYBRID_GS = 1 };

typedef struct pamg_hierarchy pamg_hierarchy;

/* ------------------------------------------------------------- context
 *
 * Sec. 4: the preconditioner module declares, allocates and initialises the
 * library's data.  A context fixes the device and the allocator through
 * which every device buffer of the hierarchies, multi-RHS engines and
 * servers made with it is allocated and freed (a framework's caching
 * allocator, or hipMalloc/hipFree).
 *   alloc(bytes, stream, user): a device pointer, aligned to at least 16
 *       bytes (256 recommended), usable on
 *       `stream` (the stream of the call that allocates; NULL = the default
 *       stream); NULL on failure, which the calling entry point reports as
 *       PAMG_E_OOM after freeing whatever it had allocated in that call.
 *   free(ptr, stream, user): releases a pointer returned by alloc.  The
 *       library has synchronized the device before it frees, so no work on
 *       any stream still uses the memory.
 * The callbacks may be called from the library's own threads (a server's
 * scheduler and setup workers), and from several threads at once. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} pamg_allocator;

typedef struct pamg_context pamg_context;

typedef struct {
    uint64_t allocs, frees;       /* successful alloc calls, free calls */
    uint64_t failed;              /* alloc calls that returned NULL */
    uint64_t live_bytes, peak_bytes;
    int32_t device, users;        /* users: hierarchies and servers made with the context */
} pamg_context_stats;

/* device: HIP device ordinal; allocator NULL: hipMalloc/hipFree (the
 * allocator struct is copied).  Errors: INVALID (device out of range),
 * OOM (host). */
int pamg_context_create(int32_t device, const pamg_allocator *allocator, pamg_context **out);
/* Errors: BUSY while hierarchies or servers made with it still exist. */
int pamg_context_destroy(pamg_context *ctx);
int pamg_context_stats_get(const pamg_context *ctx, pamg_context_stats *out);

/* A in CSR, host memory, 0-based, full symmetric storage, columns strictly
 * ascending in every row, a positive diagonal entry present in every row.
 * (Sec. 4: the application hands the matrix over in CSR.) */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr;   /* n+1 */
    const int32_t *col_idx;   /* nnz */
    const double *val;        /* nnz */
} pamg_csr;

typedef struct {
    int32_t max_coarse;       /* coarsen while n_l > max_coarse (default 200, Sec. 3.1 coarsest size) */
    int32_t max_levels;       /* default 50 */
    int32_t max_dense;        /* largest coarsest level accepted for the dense solve (default 8192,
                                 at most 8192; the factorization runs on the device) */
    int32_t match_all_edges;  /* 0: only edges with weight > 1 may be matched (default) */
    int32_t build_f32;        /* 1: also keep an FP32 copy of the hierarchy (mixed-precision V-cycle) */
    int32_t num_threads;      /* host threads for setup (0 = hardware concurrency) */
    int32_t check_symmetry;   /* 1: reject A unless bitwise symmetric */
    int32_t host_only;        /* 1: build the hierarchy on the host only (no device upload and no
                                 coarse factorization; info, aggregates and level queries work,
                                 solves return PAMG_E_INVALID) */
    double min_ratio;         /* a level with n_l <= max_dense whose matching would give
                                 n_l < min_ratio * n_{l+1} is the coarsest (default 1.5; <= 1: off).
                                 The paper does not say when coarsening stops if matching stalls
                                 (weakly coupled vertices that stay singletons on every level). */
    int32_t agg_steps;        /* aggregate-size composition (Sec. 3.1): keep every agg_steps-th level of
                                 the pairwise hierarchy, prolongators multiplied in between, so that
                                 aggregates hold up to 2^agg_steps unknowns (default 1: pairs; 1..4) */
    int32_t smoother;         /* PAMG_SMOOTHER_L1_JACOBI (default: one pre- and one post-sweep) or
                                 PAMG_SMOOTHER_HYBRID_GS (Sec. 3.1: hybrid forward/backward
                                 Gauss-Seidel, M = blockdiag(omega (L_pp + D_pp)) over row blocks of
                                 gs_block unknowns in nested-aggregate order; `sweeps` forward sweeps
                                 before and as many backward sweeps after the coarse correction) */
    int32_t sweeps;           /* hybrid GS sweeps per side, 1..16 (0: 4, the paper's nu); l1-Jacobi: 0 or 1 */
    int32_t gs_block;         /* hybrid GS block size, 1..256 (0: 256) */
    double omega;             /* hybrid GS damping of M = omega (L + D), > 0 (0: 1.5; omega = 1, the
                                 plain method, lets the Jacobi coupling between the small blocks
                                 diverge on large 3D meshes) */
    int32_t smooth_prolongator; /* 1: P = (I - w D^-1 A) P^ with w = 1/||D^-1 A||_inf, D = diag(A)
                                 (Sec. 3.1 smoothed aggregation) and A_{l+1} = P^T A P, with
                                 either smoother.  With agg_steps = s > 1 each kept level's
                                 composed tentative prolongator is smoothed; with the hybrid
                                 Gauss-Seidel smoother (4 + 4 sweeps) and agg_steps = 3 this is
                                 the paper's preconditioner (Sec. 3.1, Table 1) but for the
                                 coarsest solver.  With pairwise aggregates the coarse matrices
                                 fill in quickly.  Default 0. */
    int32_t device_setup;     /* 1: build the large levels on the device (pairwise aggregates or
                                 their composition, tentative prolongators, either smoother (the
                                 Gauss-Seidel schedule of those levels too), weight-eligible
                                 edges; smoothed prolongators, match_all_edges, inputs whose
                                 pattern is not symmetric and small inputs are built on the
                                 host).  The hierarchy is bitwise the host-built one: the
                                 matching is the greedy matching under the same strict order,
                                 computed as locally dominant edges in parallel rounds (Sec.
                                 3.1, eq. (approximatematch)), and every Galerkin entry sums its
                                 terms in the same order.  Default 1 (0: host only). */
    int32_t device_min_rows;  /* device_setup: levels with at most this many rows (or max_dense or
                                 max_coarse, if larger) are built on the host (0: 65536) */
    int32_t reserved[2];
} pamg_params;

typedef struct {
    double tol;               /* relative residual target (default 1e-6) */
    int32_t maxit;            /* default 1000 */
    int32_t use_x0;           /* 1: x_dev holds the initial guess on entry (warm start, Sec. 5) */
    int32_t krylov;           /* PAMG_KRYLOV_CG or PAMG_KRYLOV_FCG (default FCG) */
    int32_t precision;        /* PAMG_PREC_F64 or PAMG_PREC_F32 (needs build_f32) */
    int32_t check_every;      /* iterations enqueued between host convergence checks (default 4) */
    int32_t fixed_iters;      /* > 0: run exactly this many iterations, ignore tol */
    int32_t use_graph;        /* 1: replay the check_every-iteration block as a HIP graph (default 1) */
    int32_t true_residual;    /* 1: recompute ||b - A x|| at the end; with FP32 restart if above tol */
    int32_t reserved[8];
} pamg_solve_opts;

typedef struct {
    int32_t status;
    int32_t iterations;
    int32_t restarts;
    double relres;            /* recurrence residual / ||b|| */
    double relres_true;       /* ||b - A x|| / ||b|| (if requested, else -1) */
    double solve_ms;          /* wall time of the call (host clock, stream synchronised) */
} pamg_solve_info;

#define PAMG_MAX_LEVELS 64
typedef struct {
    int32_t levels;
    int32_t n[PAMG_MAX_LEVELS];
    int64_t nnz[PAMG_MAX_LEVELS];
    int32_t pairs[PAMG_MAX_LEVELS];
    double setup_ms;          /* host setup + upload */
    double operator_complexity;
    uint64_t device_bytes;
    uint64_t vcycle_bytes_f64;   /* algorithmic HBM bytes of one FP64 V-cycle */
    uint64_t vcycle_bytes_f32;   /* same for the FP32 V-cycle (0 if not built) */
    uint64_t spmv_bytes;         /* algorithmic bytes of one level-0 FP64 SpMV */
    int32_t tile_items[PAMG_MAX_LEVELS];  /* matrix entries per thread of the level's tiles (tiles of
                                             256 x items entries; items >= 8: column dictionaries) */
    uint64_t csr_vcycle_bytes_f64;  /* one FP64 V-cycle counted with plain CSR matrices (int32 columns,
                                       s-byte values, int32 row pointers): sum over l < L of
                                       2 (nnz_l (4 + s) + 4 (n_l + 1)) + (10 n_l + 2 n_{l+1}) s,
                                       plus (n_L^2 + 2 n_L) s */
    uint64_t csr_vcycle_bytes_f32;  /* same with s = 4 (0 if not built) */
    int32_t device_levels;    /* levels built on the device (device_setup), the finest ones */
    int32_t reserved0;
} pamg_hier_info;

/* Fill defaults. */
int pamg_params_default(pamg_params *p);
int pamg_solve_opts_default(pamg_solve_opts *o);

/* Build the hierarchy from A (copied; the caller may free A on return), then
 * upload it to the context's device; every device buffer of the hierarchy
 * comes from the context's allocator (ctx NULL: hipMalloc on the current
 * device).  The context must outlive the hierarchy.  Deterministic:
 * aggregates and coarse matrices are bitwise reproducible (Sec. 3.1
 * construction, readings listed in the design notes).  Errors: INVALID (bad
 * CSR), NOT_SPD (coarsest factorisation), STALLED, OOM (everything allocated
 * by the call is freed again), DEVICE. */
int pamg_setup(pamg_context *ctx, const pamg_csr *A, const pamg_params *params, void *stream,
               pamg_hierarchy **out);

int pamg_hierarchy_destroy(pamg_hierarchy *h);
int pamg_hierarchy_info(const pamg_hierarchy *h, pamg_hier_info *out);

/* Level-l aggregate index of every level-l unknown (canonical numbering:
 * level-0 unknowns in the caller's order, coarse unknowns numbered by their
 * smallest member).  agg_host has n_l entries; l < levels-1. */
int pamg_hierarchy_aggregates(const pamg_hierarchy *h, int32_t level, int32_t *agg_host);

/* Level-l Galerkin matrix in canonical numbering (host buffers of n_l+1 and
 * nnz_l entries).  After pamg_hierarchy_update_values the values are the
 * updated ones (read back from the device). */
int pamg_hierarchy_level_csr(const pamg_hierarchy *h, int32_t level, int32_t *row_ptr,
                             int32_t *col_idx, double *val);

/* Coefficient-only reuse (Sec. 4: when only the matrix coefficients change,
 * the prolongators are kept and the coarse matrices and smoothers rebuilt).
 * val: nnz new values of the setup matrix A_0 in its CSR order (same row_ptr
 * and col_idx as given to pamg_setup); host memory, or device memory if
 * on_device != 0; read only, the caller keeps ownership.  The aggregates and
 * prolongators of every level are kept; the Galerkin matrices (with
 * aggregate-size composition: of the whole pairwise chain), l1 diagonals,
 * FP32 copies and the coarsest factorization are recomputed on the device,
 * bitwise equal to what a setup with the same aggregates gives.  The first
 * call also builds the summation plans (host work, kept on the device, about
 * 24 bytes per matrix entry of every pairwise level).  Runs on `stream`
 * (HIP stream, NULL = default) and returns when the hierarchy holds the new
 * values; batched engines of the hierarchy see them too.  Errors: INVALID
 * (null, host_only hierarchy, a non-finite value or non-positive diagonal:
 * checked before anything is changed), NOT_SPD (coarsest factorization: the
 * hierarchy must be updated again before use), OOM, DEVICE. */
int pamg_hierarchy_update_values(pamg_hierarchy *h, const double *val, int32_t on_device, void *stream);

/* Solve A x = b.  b_dev, x_dev: n doubles in the caller's numbering.  On
 * return x_dev holds the last iterate (also for NOT_CONVERGED). */
int pamg_solve(pamg_hierarchy *h, const double *b_dev, double *x_dev, const pamg_solve_opts *opts,
               void *stream, pamg_solve_info *info);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): pamg_solve that makes no
 * allocation of any kind (device, pinned or host heap).  The solve state and
 * the reduction partials live in one static device array of
 * PAMG_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on
 * holds until the process ends, instead of the hierarchy's own buffers; the
 * iterations are launched directly (opts->use_graph is ignored, since
 * instantiating a graph allocates).  Arguments, ownership and results are
 * those of pamg_solve, and x is bitwise what pamg_solve returns for the
 * same options.  Every call on one GPU shares that GPU's array (whatever the
 * hierarchy or stream), which keeps the last call's contents: calls that
 * overlap on one GPU race and must be serialized by the caller.  Errors: as
 * pamg_solve; INVALID also for a hierarchy whose reductions need more
 * partials than the array holds (2 * 2048 per buffer; hierarchies built by
 * pamg_setup never do: their launches use at most 2048 workgroups). */
#define PAMG_NOALLOC_SCRATCH_BYTES 66048
int pamg_solve_noalloc(pamg_hierarchy *h, const double *b_dev, double *x_dev, const pamg_solve_opts *opts,
                       void *stream, pamg_solve_info *info);

/* Solve A X = B for 1 <= nrhs <= 16 right-hand sides at once (successive time
 * steps, or independent requests on one operator; Sec. 2: one matrix, many
 * solves).  Column j of B is at B_dev + j*ldb, of X at X_dev + j*ldx (device,
 * caller numbering, ldb, ldx >= n).  Each column runs its own FCG (or PCG)
 * recurrence with its own step lengths and stopping test; every pass over a
 * level's matrix serves all columns.  x0 = 0 (use_x0 must be 0).  A column's
 * result does not depend on the other columns.  infos: nrhs entries.  The
 * return value is the worst column status.  l1-Jacobi hierarchies only
 * (INVALID for the hybrid Gauss-Seidel smoother). */
int pamg_solve_batch(pamg_hierarchy *h, int32_t nrhs, const double *B_dev, int64_t ldb, double *X_dev,
                     int64_t ldx, const pamg_solve_opts *opts, void *stream, pamg_solve_info *infos);

/* Batched operators for parity checks: op = PAMG_OP_COARSE (16 vectors of
 * the coarsest level, A_L^-1 applied on the matrix cores in FP64) or
 * PAMG_OP_VCYCLE (16 level-0 vectors through the batched V-cycle).  in_dev,
 * out_dev: 16 FP64 vectors, vector c at ptr + c*n_level, canonical numbering. */
int pamg_debug_apply_batch(pamg_hierarchy *h, int32_t op, int32_t precision, const double *in_dev, double *out_dev,
                           void *stream);

/* Kernel variants the multi-RHS autotuner chose for each level (timed on the
 * real hierarchy the first time a batch of this precision runs): cfg[4l+0..3]
 * = down-sweep unroll (1..16), down-sweep columns per lane (1, 2 or 4),
 * up-sweep unroll, up-sweep columns per lane, for l = 0 .. levels-2 (cfg holds
 * 4*(levels-1) entries; level 0's up-sweep is a fixed shape, reported as
 * unroll 8 with 4 columns per lane). */
int pamg_batch_config(pamg_hierarchy *h, int32_t precision, int32_t *cfg);

/* Pin the kernel variants of the multi-RHS engine instead of the autotuner's
 * choice (same layout as pamg_batch_config; level 0's up-sweep entries are
 * ignored, its shape is fixed).  Every variant computes each column with the
 * same operations in the same order, so the results do not depend on this
 * choice; it exists to check that claim and to time variants.  Builds the
 * engine (and runs the autotuner once) if needed; the pinned variants stay
 * until the next call.  Errors: INVALID (null, unknown variant, a hybrid
 * Gauss-Seidel or smoothed-prolongator hierarchy), OOM, DEVICE. */
int pamg_batch_set_config(pamg_hierarchy *h, int32_t precision, const int32_t *cfg);

/* Single operators of the V-cycle, for parity checks.  Vectors are FP64 in
 * canonical level numbering.
 *   PAMG_OP_SPMV     out = A_l in0
 *   PAMG_OP_DOWN     out = P_l^T (in0 - A_l D_l^-1 in0)        (pre-smooth, residual, restriction; n_{l+1})
 *   PAMG_OP_UP       out = in1 + D_l^-1 (in0 - A_l in1)         (post-smooth of in1 given r = in0)
 *   PAMG_OP_PROLONG  out = D_l^-1 in0 + P_l in1                 (in1 has n_{l+1} entries)
 *   PAMG_OP_COARSE   out = A_L^-1 in0                           (level = L)
 *   PAMG_OP_VCYCLE   out = B in0                                (level 0; the hierarchy's smoother)
 *   PAMG_OP_SMOOTH   hybrid GS hierarchies (level < L): in1 == NULL: out = `sweeps` forward
 *                    sweeps on A_l x = in0 from x = 0 (pre-smoothing); else out = `sweeps`
 *                    backward sweeps from x = in1 (post-smoothing)
 * DOWN, UP and PROLONG are the l1-Jacobi kernels whatever the smoother.
 */
enum { PAMG_OP_SPMV = 0, PAMG_OP_DOWN = 1, PAMG_OP_UP = 2, PAMG_OP_PROLONG = 3, PAMG_OP_COARSE = 4,
       PAMG_OP_VCYCLE = 5, PAMG_OP_SMOOTH = 7 };
int pamg_debug_apply(pamg_hierarchy *h, int32_t op, int32_t level, int32_t precision, const double *in0_dev,
                     const double *in1_dev, double *out_dev, void *stream);

/* Time `reps` back-to-back V-cycles (level 0 input r_dev, canonical order) and
 * `reps` level-0 SpMVs on `stream`, measured with HIP events; milliseconds per
 * operation.  Used by the benchmark. */
int pamg_time_kernels(pamg_hierarchy *h, int32_t precision, const double *r_dev, int32_t reps, void *stream,
                      double *vcycle_ms, double *spmv_ms);

/* Time `reps` back-to-back launches of one kernel of the solve on `stream`
 * with HIP events (milliseconds per launch), on the data currently held in
 * the hierarchy's buffers.  op: PAMG_OP_DOWN or PAMG_OP_UP (V-cycle kernels of
 * level `level`), PAMG_OP_SPMV (level-`level` SpMV), PAMG_OP_KRYLOV (level-0
 * FCG kernel: p = z + beta p, q = A p, p.q, p.r).  *bytes receives the
 * algorithmic HBM bytes of one launch (matrix, owned vector entries and
 * outputs counted once; gathered entries are not recounted). */
enum { PAMG_OP_KRYLOV = 6 };
int pamg_time_op(pamg_hierarchy *h, int32_t op, int32_t level, int32_t precision, int32_t reps, void *stream,
                 double *ms_per_launch, uint64_t *bytes);

/* ---------------------------------------------------------------- serving
 *
 * A request loop on one GPU for many pressure solves (the paper's setting:
 * one operator, many solves, Sec. 2; hierarchy reuse, Sec. 4).  A scheduler
 * thread owns all GPU work.  An operator (identified by a caller-chosen key)
 * gets its hierarchy built the first time a request names it: the host phase
 * of the setup runs on a worker thread while cached operators keep iterating,
 * and the upload happens once its device bytes fit the HBM budget next to the
 * operators already cached (idle ones are evicted least-recently-used first);
 * until then the request waits.  Every
 * cached operator batches up to 16 requests as independent columns; waiting
 * requests join between iteration blocks and finished ones retire at once.
 * Blocks of all operators are launched before any is waited on, so their
 * work overlaps.  A request's result does not depend on what it was batched
 * with (with single_path, a request alone on its operator runs on the
 * single-right-hand-side solver instead).  Calls that overlap on one server
 * from several threads are safe. */
typedef struct pamg_server pamg_server;

typedef struct {
    uint64_t hbm_budget_bytes;   /* device bytes for cached hierarchies + work vectors (default 64 GiB) */
    int32_t block_iters;         /* iterations per block between join/retire points (default 4, made even) */
    int32_t precision;           /* V-cycle precision, default PAMG_PREC_F32 (FP64 recurrences; a
                                    column is accepted on its true FP64 residual) */
    int32_t use_graph;           /* 1: replay each operator's block as a HIP graph, captured on the
                                    scheduler thread.  While a capture runs, device-wide calls from
                                    the application's threads (hipDeviceSynchronize) fail with
                                    hipErrorStreamCaptureUnsupported, so such programs must
                                    synchronize streams instead.  Default 0: direct launches. */
    int32_t single_path;         /* 1: while fewer than batch_from requests for an operator are
                                    waiting and its batch has no running column, its requests run
                                    one at a time on the single-right-hand-side solver (n-long
                                    vectors instead of n x 16; later ones wait for it), and such a
                                    result is bitwise that of pamg_solve with the same tolerance,
                                    maxit and precision; otherwise they join the batch engine.
                                    Which solver serves a request then depends on the mix.
                                    Default 0: every request is a column of the batch engine,
                                    bitwise independent of the mix. */
    int32_t batch_from;          /* with single_path: waiting requests of one operator from which
                                    they go to the batch engine (<= 0: 4) */
    int32_t setup_workers;       /* threads running host phases of new operators at once, each with
                                    an equal share of the host cores (<= 0: 1; at most 16) */
    int32_t device_setup;        /* 1 (default): a worker builds a new operator's large levels on
                                    the device (pamg_params.device_setup), on a stream of its own
                                    beside the solving, once the scheduler has reserved an upper
                                    bound of its bytes (hierarchy and build temporaries) in the
                                    budget; operators the device construction does not cover are
                                    built on the host as with 0 */
    int32_t reserved[3];
} pamg_server_opts;

typedef struct {
    uint64_t op_key;             /* operator identity chosen by the caller */
    const pamg_csr *A;           /* host CSR; read only if op_key is not cached (else may be NULL);
                                    must stay valid until the request completes */
    const double *b_dev;         /* device right-hand side (caller numbering); valid until completion */
    double *x_dev;               /* device result (caller numbering); written before completion */
    double tol;                  /* relative residual target */
    int32_t maxit;               /* <= 0: 1000 */
    int32_t reserved;
    uint64_t tag;                /* returned in the completion */
} pamg_request;

typedef struct {
    uint64_t tag;
    int32_t status;              /* pamg_status; PAMG_E_BUSY: the operator alone exceeds the budget */
    int32_t iterations;
    double relres;               /* recurrence residual / ||b|| */
    double relres_true;          /* true residual / ||b|| (FP32 V-cycle), else -1 */
    double queue_ms;             /* submit -> column assigned */
    double latency_ms;           /* submit -> result written */
} pamg_completion;

typedef struct {
    uint64_t submitted, completed, rejected;
    uint64_t bytes_in_use, hbm_budget_bytes;
    int32_t cached_operators, active_columns, pending, pad;
    uint64_t setups, evictions, blocks;
    double busy_ms;              /* scheduler time spent in ticks */
    uint64_t algorithmic_bytes;  /* HBM bytes the executed iterations had to move */
    double host_setup_ms;        /* host phases of the setups (worker thread, overlaps solving) */
    double device_setup_ms;      /* uploads and coarsest factorizations (scheduler thread) */
    uint64_t engines_built;      /* 16-column engines built (operators' first batches) */
    uint64_t engines_freed;      /* engines of idle operators freed to make room */
} pamg_server_stats;

int pamg_server_opts_default(pamg_server_opts *o);
/* An upper estimate of the device bytes an operator can hold in a server
 * (A: host CSR; precision: the V-cycle's): its hierarchy plus its 16-column
 * engine.  Admission charges the hierarchy part of it for an uncached
 * operator, then the exact figure once the hierarchy exists; the engine is
 * built (and charged, exactly) only when the operator's requests first run
 * as a batch.  Under budget pressure the engines of idle operators are freed
 * before idle operators are evicted; an engine that can never fit beside its
 * hierarchy sends the operator's requests to the single-right-hand-side path
 * (or, without it, refuses them with BUSY). */
int pamg_server_estimate_bytes(const pamg_csr *A, int32_t precision, uint64_t *out);
/* ctx: allocator and device of every hierarchy the server builds (NULL:
 * hipMalloc on the current device); it must outlive the server. */
int pamg_server_create(pamg_context *ctx, const pamg_server_opts *opts, pamg_server **out);
/* Queue a request (copied).  Errors: INVALID (null pointers, bad tol). */
int pamg_server_submit(pamg_server *s, const pamg_request *req);
/* Move up to `max` completions into out (non-blocking); *n_out = count. */
int pamg_server_poll(pamg_server *s, pamg_completion *out, int32_t max, int32_t *n_out);
int pamg_server_stats_get(pamg_server *s, pamg_server_stats *out);
/* Finish every queued and running request, then free all server resources. */
int pamg_server_destroy(pamg_server *s);

/* Thread-local description of the last failure on this thread. */
const char *pamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PAMG_H */
