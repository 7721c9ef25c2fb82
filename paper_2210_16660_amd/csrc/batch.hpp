// Internal interface of the multi-right-hand-side engine (batch.hip), used by
// the batched solve entry point and by the serving loop.
#pragma once

#include "hier.hpp"
#include "kernels_batch.hpp"

namespace pamg {

BatchEngine* get_engine(pamg_hierarchy* h, int prec, hipStream_t s);
const BatchState& batch_state(const BatchEngine* E);
BatchState& batch_state_host(BatchEngine* E);
uint64_t batch_bytes(const BatchEngine* E);
void batch_read_state(BatchEngine* E, hipStream_t s);
// Enqueue the state copy to the host without waiting (the host copy is valid
// once the stream has passed it, e.g. after an event recorded behind it).
void batch_read_state_async(BatchEngine* E, hipStream_t s);
void batch_write_state(BatchEngine* E, hipStream_t s);
void batch_load(BatchEngine* E, const double* const* src, const double* tol, const int* maxit, const int* fixed,
                int krylov, hipStream_t s);
void batch_store(BatchEngine* E, double* const* dst, hipStream_t s);
void batch_true_residual(BatchEngine* E, int restart_mask, double* relres, hipStream_t s);
void batch_run_block(BatchEngine* E, int krylov, int k, bool use_graph, hipStream_t s);
// Capture and instantiate the block graph batch_run_block replays (no launch).
void batch_prepare_graph(BatchEngine* E, int krylov, int k);
// Mark the columns in `mask` inactive in the host copy of the state (written
// back by the next batch_write_state / batch_load).
void batch_retire(BatchEngine* E, int mask);
// Free the engine of this precision (synchronizes the device); the tuned
// kernel variants stay with the hierarchy for the next engine.
void release_engine(pamg_hierarchy* h, int prec);
// Device bytes an engine of this precision takes for h.
uint64_t engine_bytes(const pamg_hierarchy* h, int prec);

}  // namespace pamg
