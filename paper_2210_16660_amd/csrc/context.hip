// Contexts: the device and the allocator every device buffer of the library
// comes from (Sec. 4: the module that declares, allocates and initialises
// the library's data).  Callers that pass no context get one per device that
// allocates with hipMalloc.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "hier.hpp"

namespace pamg {

namespace {
std::mutex g_default_mu;
std::map<int, pamg_context*> g_default;   // kept until the process ends
}  // namespace

pamg_context* default_context(int device) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    pamg_context*& c = g_default[device];
    if (!c) {
        c = new pamg_context();
        c->device = device;
    }
    return c;
}

void* ctx_alloc(pamg_context* c, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 1;
    void* p = nullptr;
    if (c->a.alloc) {
        p = c->a.alloc(bytes, (void*)s, c->a.user);
    } else {
        const hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            if (e != hipErrorOutOfMemory)
                throw Error(PAMG_E_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    if (!p) {
        c->failed.fetch_add(1);
        throw Error(PAMG_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) {
        if (c->a.free) c->a.free(p, (void*)s, c->a.user);
        else (void)hipFree(p);
        throw Error(PAMG_E_INVALID, "allocator returned a pointer that is not 16-byte aligned");
    }
    c->allocs.fetch_add(1);
    const uint64_t live = c->live.fetch_add(bytes) + bytes;
    uint64_t peak = c->peak.load();
    while (live > peak && !c->peak.compare_exchange_weak(peak, live)) {
    }
    return p;
}

void ctx_free(pamg_context* c, void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (c->a.free) c->a.free(p, (void*)s, c->a.user);
    else (void)hipFree(p);
    c->frees.fetch_add(1);
    c->live.fetch_sub(bytes == 0 ? 1 : bytes);
}

void ctx_free_all(pamg_context* c, std::vector<DevAlloc>& list) {
    for (const DevAlloc& a : list) ctx_free(c, a.p, a.bytes, nullptr);
    list.clear();
}

}  // namespace pamg

extern "C" {

int pamg_context_create(int32_t device, const pamg_allocator* allocator, pamg_context** out) {
    return pamg::guarded([&]() -> int {
        if (!out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        *out = nullptr;
        int count = 0;
        HIP_CHECK(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) throw pamg::Error(PAMG_E_INVALID, "device out of range");
        if (allocator && (!allocator->alloc || !allocator->free))
            throw pamg::Error(PAMG_E_INVALID, "allocator needs both alloc and free");
        pamg_context* c = new pamg_context();
        c->device = device;
        if (allocator) c->a = *allocator;
        *out = c;
        return PAMG_OK;
    });
}

int pamg_context_destroy(pamg_context* ctx) {
    return pamg::guarded([&]() -> int {
        if (!ctx) return PAMG_OK;
        if (ctx->users.load() > 0)
            throw pamg::Error(PAMG_E_BUSY, "context still has hierarchies or servers");
        delete ctx;
        return PAMG_OK;
    });
}

int pamg_context_stats_get(const pamg_context* ctx, pamg_context_stats* out) {
    return pamg::guarded([&]() -> int {
        if (!ctx || !out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        out->allocs = ctx->allocs.load();
        out->frees = ctx->frees.load();
        out->failed = ctx->failed.load();
        out->live_bytes = ctx->live.load();
        out->peak_bytes = ctx->peak.load();
        out->device = ctx->device;
        out->users = ctx->users.load();
        return PAMG_OK;
    });
}

}  // extern "C"
