// Coefficient-only reuse of a hierarchy (arXiv 2210.16660, Sec. 4: when
// only the coefficients of the matrix change, the prolongators are kept and
// the coarse matrices and smoothers are rebuilt).
//
// The aggregates and tentative prolongators of every level stay; from new
// values of A_0 (same pattern) the device recomputes, bitwise as a setup
// with the same aggregates would:
//   * the Galerkin matrix of every pairwise step, each coarse entry summed
//     left to right in the setup's canonical order from the terms
//     a_ij (p_i p_j) (plans built on the host once, on the first update);
//     with aggregate-size composition the whole pairwise chain is re-run and
//     the kept levels are taken from it;
//   * the l1 diagonals (canonical row order), the device-order values, the
//     column-scaled values a_ij / d_j, 1 / a_ii for the hybrid Gauss-Seidel
//     smoother, the FP32 copies;
//   * the coarsest level's Cholesky factor and inverse (dense.hip).
// Every product and sum is one IEEE operation (no contraction).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <mutex>

#include "hier.hpp"

// every product and sum below is rounded on its own, as in the setup
#pragma clang fp contract(off)

namespace pamg {

// Validity of new level-0 values: all finite, every diagonal positive.
static __global__ __launch_bounds__(kBlock) void k_reuse_check(long long nnz, int n, const double* __restrict__ v,
                                                        const int* __restrict__ dpos, int* __restrict__ flag) {
    const long long stride = (long long)gridDim.x * kBlock;
    const long long t0 = (long long)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    for (long long k = t0; k < nnz; k += stride) bad |= !isfinite(v[k]);
    for (long long i = t0; i < n; i += stride) bad |= !(v[dpos[i]] > 0.0);
    if (bad) flag[0] = 1;
}

// Coarse entry e = sum over its plan terms t, in order, of v_f[k_t] * pp_t.
static __global__ __launch_bounds__(kBlock) void k_galerkin_sum(int ne, const int* __restrict__ ptr,
                                                         const int* __restrict__ gk, const double* __restrict__ pp,
                                                         const double* __restrict__ vf, double* __restrict__ vc) {
    const int stride = gridDim.x * kBlock;
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < ne; e += stride) {
        const int t0 = ptr[e], t1 = ptr[e + 1];
        double acc = vf[gk[t0]] * pp[t0];
        for (int t = t0 + 1; t < t1; ++t) acc = acc + vf[gk[t]] * pp[t];
        vc[e] = acc;
    }
}

// dinv_i = 1 / sum_j |a_ij|, the row summed in canonical column order.
static __global__ __launch_bounds__(kBlock) void k_l1_inverse(int n, const int* __restrict__ rp,
                                                       const double* __restrict__ v, double* __restrict__ dinv) {
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        double d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) d = d + fabs(v[k]);
        dinv[i] = 1.0 / d;
    }
}

// vd_k = v_k * dinv[col_k] (the restriction pass's column-scaled values).
static __global__ __launch_bounds__(kBlock) void k_scale_columns(long long nnz, const int* __restrict__ ci,
                                                          const double* __restrict__ v,
                                                          const double* __restrict__ dinv,
                                                          double* __restrict__ vd) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride)
        vd[k] = v[k] * dinv[ci[k]];
}

// Hybrid Gauss-Seidel: 1 / a_ii of every row (device order).
static __global__ __launch_bounds__(kBlock) void k_diag_inverse(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ v,
                                                         double* __restrict__ ainv) {
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) ainv[i] = 1.0 / v[k];
}


// The pairwise chain behind the kept levels: pattern, aggregates and p of
// pairwise level m.
struct ChainView {
    const HostHierarchy& H;
    int levels() const { return H.chain.empty() ? (int)H.lev.size() : (int)H.chain.size(); }
    const HostCSR& pattern(int m) const {
        if (H.chain.empty()) return H.lev[m].A;
        const PairLevel& c = H.chain[m];
        return c.kept >= 0 ? H.lev[c.kept].A : c.S;
    }
    const std::vector<int32_t>& agg(int m) const { return H.chain.empty() ? H.lev[m].agg : H.chain[m].agg; }
    const std::vector<double>& p(int m) const { return H.chain.empty() ? H.lev[m].p : H.chain[m].p; }
    int kept_level(int m) const { return H.chain.empty() ? m : H.chain[m].kept; }
};

// The plan's device arrays: kept in a list of their own until the plan is
// complete, so that a failed allocation leaves the hierarchy as it was.
struct PlanAllocs {
    pamg_context* ctx;
    std::vector<DevAlloc> list;
    ~PlanAllocs() { ctx_free_all(ctx, list); }
};

static void build_plan(pamg_hierarchy* h, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<ReusePlan> R(new ReusePlan());
    PlanAllocs pa{h->ctx, {}};
    auto dalloc_plan = [&](size_t bytes) {
        void* p = ctx_alloc(h->ctx, bytes, s);
        pa.list.push_back({p, bytes});
        return p;
    };
    auto to_device = [&](const auto& src) {
        using T = typename std::decay<decltype(src)>::type::value_type;
        T* d = static_cast<T*>(dalloc_plan(std::max<size_t>(1, src.size()) * sizeof(T)));
        if (!src.empty()) {
            HIP_CHECK(hipMemcpyAsync(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        return d;
    };
    ensure_host_levels(h);
    const ChainView C{h->host};
    const int npw = C.levels(), nk = h->L + 1;
    R->npw = npw;
    R->kept_pw.assign(nk, -1);
    for (int m = 0; m < npw; ++m) {
        const int j = C.kept_level(m);
        if (j >= 0) R->kept_pw[j] = m;
    }
    for (int j = 0; j < nk; ++j)
        if (R->kept_pw[j] < 0) throw Error(PAMG_E_DEVICE, "reuse plan: kept level without a pairwise level");
    for (int m = 0; m < npw; ++m) {
        R->nnz.push_back(C.pattern(m).nnz());
        R->vcan.push_back(static_cast<double*>(dalloc_plan(sizeof(double) * std::max<size_t>(1, C.pattern(m).nnz()))));
    }
    for (int m = 0; m + 1 < npw; ++m) {
        GalerkinPlan g = galerkin_plan(C.pattern(m), C.agg(m), C.p(m), C.pattern(m + 1));
        R->gptr.push_back(to_device(g.ptr));
        R->gk.push_back(to_device(g.k));
        R->gpp.push_back(to_device(g.pp));
    }
    for (int j = 0; j < nk; ++j) {
        const HostCSR& A = h->host.lev[j].A;
        const DevLevelIdx& I = h->idx[j];
        std::vector<int32_t> perm(I.n), iperm(I.n);
        HIP_CHECK(hipMemcpy(perm.data(), I.perm, sizeof(int32_t) * I.n, hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(iperm.data(), I.iperm, sizeof(int32_t) * I.n, hipMemcpyDeviceToHost));
        R->crp.push_back(to_device(A.rp));
        R->hperm.push_back(to_device(entry_order(A, perm, iperm)));
        R->dcan.push_back(static_cast<double*>(dalloc_plan(sizeof(double) * std::max<size_t>(1, I.n))));
    }
    const HostCSR& A0 = h->host.lev[0].A;
    std::vector<int32_t> dpos(A0.n, 0);
    for (int32_t i = 0; i < A0.n; ++i)
        for (int32_t k = A0.rp[i]; k < A0.rp[i + 1]; ++k)
            if (A0.ci[k] == i) dpos[i] = k;
    R->dpos0 = to_device(dpos);
    R->flag = static_cast<int*>(dalloc_plan(sizeof(int)));
    R->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // complete: the arrays now belong to the hierarchy
    for (const DevAlloc& a : pa.list) {
        h->allocs.push_back(a);
        h->info.device_bytes += a.bytes;
    }
    pa.list.clear();
    h->reuse = std::move(R);
}

static void update_values(pamg_hierarchy* h, const double* val, bool on_device, hipStream_t s) {
    if (!h->reuse) build_plan(h, s);
    ReusePlan& R = *h->reuse;
    const int n0 = h->idx[0].n;
    const long long nnz0 = R.nnz[0];
    HIP_CHECK(hipMemcpyAsync(R.vcan[0], val, sizeof(double) * nnz0,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    // validate before anything the solver reads is touched
    HIP_CHECK(hipMemsetAsync(R.flag, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_reuse_check, dim3(vec_grid(nnz0)), dim3(kBlock), 0, s, nnz0, n0, (const double*)R.vcan[0],
                       (const int*)R.dpos0, R.flag);
    int bad = 0;
    HIP_CHECK(hipMemcpyAsync(&bad, R.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (bad) throw Error(PAMG_E_INVALID, "new values: non-finite value or non-positive diagonal");
    // workspace of the coarsest factorization, before any value is changed
    const DevLevelIdx& CL = h->idx[h->L];
    std::unique_ptr<DenseWork> dw = dense_work(h->ctx, CL.n, s);
    // the pairwise Galerkin chain
    for (int m = 0; m + 1 < R.npw; ++m) {
        const int ne = (int)R.nnz[m + 1];
        hipLaunchKernelGGL(k_galerkin_sum, dim3(vec_grid(ne)), dim3(kBlock), 0, s, ne, (const int*)R.gptr[m],
                           (const int*)R.gk[m], (const double*)R.gpp[m], (const double*)R.vcan[m], R.vcan[m + 1]);
    }
    // the kept levels in device order
    DevVals<double>& V = h->f64;
    for (int j = 0; j <= h->L; ++j) {
        const DevLevelIdx& I = h->idx[j];
        const double* vc = R.vcan[R.kept_pw[j]];
        hipLaunchKernelGGL(k_l1_inverse, dim3(vec_grid(I.n)), dim3(kBlock), 0, s, I.n, (const int*)R.crp[j], vc,
                           R.dcan[j]);
        hipLaunchKernelGGL((k_gather<double, double>), dim3(vec_grid(I.nnz)), dim3(kBlock), 0, s, (int)I.nnz,
                           (const int*)R.hperm[j], vc, V.v[j]);
        hipLaunchKernelGGL((k_gather<double, double>), dim3(vec_grid(I.n)), dim3(kBlock), 0, s, I.n,
                           (const int*)I.iperm, (const double*)R.dcan[j], V.dinv[j]);
        if (j < h->L)
            hipLaunchKernelGGL(k_scale_columns, dim3(vec_grid(I.nnz)), dim3(kBlock), 0, s, I.nnz, (const int*)I.ci,
                               (const double*)V.v[j], (const double*)V.dinv[j], V.vd[j]);
        const bool gs = h->smoother == PAMG_SMOOTHER_HYBRID_GS && j < h->L;
        if (gs)
            hipLaunchKernelGGL(k_diag_inverse, dim3(vec_grid(I.n)), dim3(kBlock), 0, s, I.n, (const int*)I.rp,
                               (const int*)I.ci, (const double*)V.v[j], V.gsa[j]);
        if (h->f32.built) {
            hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(I.nnz)), dim3(kBlock), 0, s, I.nnz,
                               (const double*)V.v[j], h->f32.v[j]);
            hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(I.n)), dim3(kBlock), 0, s, (long long)I.n,
                               (const double*)V.dinv[j], h->f32.dinv[j]);
            if (j < h->L)
                hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(I.nnz)), dim3(kBlock), 0, s, I.nnz,
                                   (const double*)V.vd[j], h->f32.vd[j]);
            if (gs)
                hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(I.n)), dim3(kBlock), 0, s,
                                   (long long)I.n, (const double*)V.gsa[j], h->f32.gsa[j]);
        }
    }
    HIP_CHECK(hipGetLastError());
    h->values_updated = true;
    // the coarsest level: factorization and inverse (synchronizes)
    coarse_inverse_device(*dw, CL.n, CL.rp, CL.ci, V.v[h->L], V.ainv, s);
    if (h->f32.built) {
        const long long nn = (long long)CL.n * CL.n;
        hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(nn)), dim3(kBlock), 0, s, nn,
                           (const double*)V.ainv, h->f32.ainv);
    }
    HIP_CHECK(hipStreamSynchronize(s));
}

// Canonical values of kept level `level` after an update (device to host).
void updated_level_values(const pamg_hierarchy* h, int level, double* v) {
    const ReusePlan& R = *h->reuse;
    const int m = R.kept_pw[level];
    HIP_CHECK(hipMemcpy(v, R.vcan[m], sizeof(double) * R.nnz[m], hipMemcpyDeviceToHost));
}

}  // namespace pamg

extern "C" int pamg_hierarchy_update_values(pamg_hierarchy* h, const double* val, int32_t on_device, void* stream) {
    return pamg::guarded([&]() -> int {
        if (!h || !val) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg::require_device(h);
        if (h->smoothed_p)
            throw pamg::Error(PAMG_E_INVALID, "smoothed prolongators depend on the values: set up again");
        std::lock_guard<std::mutex> lk(h->mu);
        HIP_CHECK(hipSetDevice(h->device));
        pamg::update_values(h, val, on_device != 0, (hipStream_t)stream);
        return PAMG_OK;
    });
}
