// Device side of the library: hierarchy upload, V-cycle and Krylov launch
// schedule, HIP-graph replay of iteration blocks, and the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "hier.hpp"
#include "kernels_gs.hpp"
#include "dsetup.hpp"

namespace pamg {

template <typename T, typename S>
static T* upload(pamg_hierarchy* h, const std::vector<S>& src, hipStream_t s) {
    T* d = dalloc<T>(h, src.size(), s);
    if (src.empty()) return d;
    if constexpr (std::is_same<T, S>::value) {
        HIP_CHECK(hipMemcpyAsync(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    } else {
        std::vector<T> tmp(src.begin(), src.end());
        HIP_CHECK(hipMemcpyAsync(d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    return d;
}

// A device array converted to another precision (the FP32 copy of a
// device-built level: each value rounded as on the host).
template <typename D, typename S>
static D* convert_copy(pamg_hierarchy* h, const S* src, long long n, hipStream_t s) {
    D* d = dalloc<D>(h, (size_t)n, s);
    if (n > 0)
        hipLaunchKernelGGL((k_convert<S, D>), dim3(vec_grid(n)), dim3(kBlock), 0, s, n, src, d);
    return d;
}

// Values of every level: levels below db->m from the device build (FP64 as
// built, FP32 converted on the device), the others uploaded from `lay`
// (level db->m + j is lay[j]).
template <typename T>
static void upload_values(pamg_hierarchy* h, DevVals<T>& V, const std::vector<LayoutLevel>& lay,
                          const DeviceBuild* db, hipStream_t s) {
    const int m = db ? db->m : 0;
    const int nl = m + (int)lay.size();
    V.v.resize(nl); V.dinv.resize(nl);
    V.vd.assign(nl, nullptr); V.p.assign(nl, nullptr); V.r.assign(nl, nullptr); V.zp.assign(nl, nullptr);
    size_t maxn = 0;
    for (int l = 0; l < nl; ++l) {
        const size_t n = (size_t)h->idx[l].n;
        if (l < m) {
            const DevLevelOut& D = db->dev[l];
            if constexpr (std::is_same<T, double>::value) {
                V.v[l] = D.v;
                V.dinv[l] = D.dinv;
                V.vd[l] = D.vd;
                V.p[l] = D.p;
            } else {
                V.v[l] = convert_copy<T>(h, D.v, D.nnz, s);
                V.dinv[l] = convert_copy<T>(h, D.dinv, D.n, s);
                V.vd[l] = convert_copy<T>(h, D.vd, D.nnz, s);
                V.p[l] = convert_copy<T>(h, D.p, D.n, s);
            }
        } else {
            const LayoutLevel& Ly = lay[l - m];
            V.v[l] = upload<T>(h, Ly.v, s);
            V.dinv[l] = upload<T>(h, Ly.dinv, s);
            if (l + 1 < nl) {
                V.vd[l] = upload<T>(h, Ly.vd, s);
                V.p[l] = upload<T>(h, Ly.p, s);
            }
        }
        if (l + 1 < nl) V.zp[l] = dalloc<T>(h, n, s);
        if (l >= 1) V.r[l] = dalloc<T>(h, n, s);
        maxn = std::max(maxn, n);
    }
    if (h->smoother == PAMG_SMOOTHER_HYBRID_GS || h->smoothed_p) {   // smoothed: host-built hierarchies only
        V.gsa.assign(nl, nullptr);
        V.gst.assign(nl, nullptr);
        V.zt.assign(nl, nullptr);
        V.sa_pv.assign(nl, nullptr);
        V.sa_tv.assign(nl, nullptr);
        for (int l = 0; l + 1 < nl; ++l) {
            const size_t n = (size_t)h->idx[l].n;
            if (h->smoother == PAMG_SMOOTHER_HYBRID_GS) {
                if (l < m) {
                    // 1 / a_ii from the device schedule (FP32: its rounding)
                    const DevLevelOut& D = db->dev[l];
                    if constexpr (std::is_same<T, double>::value)
                        V.gsa[l] = D.gs_ainv;
                    else
                        V.gsa[l] = convert_copy<T>(h, D.gs_ainv, D.n, s);
                } else {
                    V.gsa[l] = upload<T>(h, lay[l - m].gs.ainv, s);
                }
                V.gst[l] = dalloc<T>(h, n, s);
            }
            if (h->smoothed_p) {
                V.sa_pv[l] = upload<T>(h, lay[l - m].sa_pv, s);
                V.sa_tv[l] = upload<T>(h, lay[l - m].sa_tv, s);
            }
            V.zt[l] = dalloc<T>(h, n, s);
        }
        V.zc = dalloc<T>(h, (size_t)h->idx[nl - 1].n, s);
    }
    // A_L^{-1}: factorized on the device in FP64; the FP32 copy is its rounding
    const DevLevelIdx& C = h->idx[nl - 1];
    V.ainv = dalloc<T>(h, (size_t)C.n * C.n, s);
    if constexpr (std::is_same<T, double>::value) {
        std::unique_ptr<DenseWork> w = dense_work(h->ctx, C.n, s);
        coarse_inverse_device(*w, C.n, C.rp, C.ci, V.v[nl - 1], V.ainv, s);
    } else {
        const long long nn = (long long)C.n * C.n;
        hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(nn)), dim3(kBlock), 0, s, nn,
                           (const double*)h->f64.ainv, V.ainv);
    }
    HIP_CHECK(hipStreamSynchronize(s));
    V.dbg_in = dalloc<T>(h, maxn, s);
    V.dbg_in2 = dalloc<T>(h, maxn, s);
    V.built = true;
}

// Matrix bytes of one pass over a level in the tile format: values, 16-bit
// dictionary positions, the tiles' dictionaries, descriptors (16 B) and spans
// (8 B), and the row pointer.
static uint64_t matrix_bytes(const DevLevelIdx& I, bool down, uint64_t s) {
    const uint64_t dict = (uint64_t)(down ? I.down_dlen : I.up_dlen);
    const uint64_t nt = (uint64_t)(down ? I.n_down : I.n_up);
    return (uint64_t)I.nnz * (2 + s) + 4 * dict + 24 * nt + 4 * ((uint64_t)I.n + 1);
}

static uint64_t vcycle_bytes(const pamg_hierarchy* h, int s) {
    // sum over l < L of the two matrix passes + (10 n_l + 2 n_{l+1}) s, plus the coarse solve
    uint64_t B = 0;
    for (int l = 0; l < h->L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        const uint64_t n = I.n, nc = h->idx[l + 1].n;
        B += matrix_bytes(I, true, s) + matrix_bytes(I, false, s) + (10 * n + 2 * nc) * s;
    }
    const uint64_t nL = h->idx[h->L].n;
    B += (nL * nL + 2 * nL) * s;
    return B;
}

// The same cycle with plain CSR matrices (int32 columns and row pointers).
static uint64_t csr_vcycle_bytes(const pamg_hierarchy* h, uint64_t s) {
    uint64_t B = 0;
    for (int l = 0; l < h->L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        const uint64_t n = I.n, nc = h->idx[l + 1].n;
        B += 2 * ((uint64_t)I.nnz * (4 + s) + 4 * (n + 1)) + (10 * n + 2 * nc) * s;
    }
    const uint64_t nL = h->idx[h->L].n;
    B += (nL * nL + 2 * nL) * s;
    return B;
}

// The device levels of the hierarchy: levels below db->m (if any) from the
// device build, the others uploaded from `lay` (level db->m + j is lay[j]);
// then the solver's vectors and the level summary.
void upload_hierarchy(pamg_hierarchy* h, const std::vector<LayoutLevel>& lay, bool build_f32, hipStream_t s,
                      const DeviceBuild* db) {
    const int m = db ? db->m : 0;
    const int nl = m + (int)lay.size();
    h->L = nl - 1;
    h->idx.resize(nl);
    for (int l = 0; l < m; ++l) {
        DevLevelIdx& I = h->idx[l];
        const DevLevelOut& D = db->dev[l];
        I.n = D.n;
        I.nnz = D.nnz;
        I.nc = D.nc;
        I.items = D.items;
        I.rp = D.rp;
        I.ci = D.ci;
        I.perm = D.perm;
        I.iperm = D.iperm;
        I.aggptr = D.aggptr;
        I.max_agg = D.max_agg;
        I.up_tiles = reinterpret_cast<const int4*>(D.up_tiles);
        I.n_up = D.n_up;
        I.down_tiles = reinterpret_cast<const int4*>(D.down_tiles);
        I.n_down = D.n_down;
        auto dict = [&](const DevDict& d, const int2*& span, const int*& col, const uint16_t*& loc, int& dmax,
                        long long& dlen) {
            span = reinterpret_cast<const int2*>(d.span ? d.span : dalloc<int>(h, 2, s));
            col = d.col ? d.col : dalloc<int>(h, 1, s);
            loc = d.loc ? d.loc : dalloc<uint16_t>(h, 1, s);
            dmax = std::max(1, d.max_len);
            dlen = d.len;
        };
        dict(D.up_dict, I.up_span, I.up_col, I.up_loc, I.up_dmax, I.up_dlen);
        dict(D.down_dict, I.down_span, I.down_col, I.down_loc, I.down_dmax, I.down_dlen);
        if (h->smoother == PAMG_SMOOTHER_HYBRID_GS) {
            I.gs_df = D.gs_df;
            I.gs_db = D.gs_db;
            I.gs_maxd = D.gs_maxd;
            I.gs_fresh = reinterpret_cast<const int2*>(D.gs_fresh);
            I.gs_nblk = D.gs_nblk;
        }
    }
    for (int l = m; l < nl; ++l) {
        DevLevelIdx& I = h->idx[l];
        const LayoutLevel& Ly = lay[l - m];
        I.n = (int)Ly.dinv.size();
        I.nnz = (long long)Ly.ci.size();
        I.nc = (l + 1 < nl) ? (int)lay[l + 1 - m].dinv.size() : 0;
        I.items = Ly.items;
        I.rp = upload<int>(h, Ly.rp, s);
        I.ci = upload<int>(h, Ly.ci, s);
        I.perm = upload<int>(h, Ly.perm, s);
        I.iperm = upload<int>(h, Ly.iperm, s);
        I.up_tiles = reinterpret_cast<const int4*>(upload<int>(h, Ly.up_tiles, s));
        I.n_up = (int)Ly.up_tiles.size() / 4;
        I.up_span = reinterpret_cast<const int2*>(upload<int>(h, Ly.up_dict.span, s));
        I.up_col = upload<int>(h, Ly.up_dict.col, s);
        I.up_loc = upload<uint16_t>(h, Ly.up_dict.local, s);
        I.up_dmax = std::max(1, (int)Ly.up_dict.max_len);
        I.up_dlen = (long long)Ly.up_dict.col.size();
        if (l + 1 < nl) {
            I.aggptr = upload<int>(h, Ly.aggptr, s);
            for (size_t c = 0; c + 1 < Ly.aggptr.size(); ++c)
                I.max_agg = std::max(I.max_agg, Ly.aggptr[c + 1] - Ly.aggptr[c]);
            I.down_tiles = reinterpret_cast<const int4*>(upload<int>(h, Ly.down_tiles, s));
            I.n_down = (int)Ly.down_tiles.size() / 4;
            I.down_span = reinterpret_cast<const int2*>(upload<int>(h, Ly.down_dict.span, s));
            I.down_col = upload<int>(h, Ly.down_dict.col, s);
            I.down_loc = upload<uint16_t>(h, Ly.down_dict.local, s);
            I.down_dmax = std::max(1, (int)Ly.down_dict.max_len);
            I.down_dlen = (long long)Ly.down_dict.col.size();
            if (h->smoothed_p) {
                const auto tiled = [&](const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                                       const TiledRows& T) {
                    DevTiled D;
                    D.rp = upload<int>(h, rp, s);
                    D.ci = upload<int>(h, ci, s);
                    D.tiles = reinterpret_cast<const int4*>(upload<int>(h, T.tiles, s));
                    D.ntiles = (int)T.tiles.size() / 4;
                    D.items = T.items;
                    D.span = reinterpret_cast<const int2*>(upload<int>(h, T.dict.span, s));
                    D.col = upload<int>(h, T.dict.col, s);
                    D.loc = upload<uint16_t>(h, T.dict.local, s);
                    D.dmax = std::max(1, (int)T.dict.max_len);
                    return D;
                };
                I.sa_p = tiled(Ly.sa_prp, Ly.sa_pci, Ly.sa_ptile);
                I.sa_t = tiled(Ly.sa_trp, Ly.sa_tci, Ly.sa_ttile);
                I.sa_nnz = (long long)Ly.sa_pci.size();
            }
            if (h->smoother == PAMG_SMOOTHER_HYBRID_GS) {
                I.gs_df = upload<uint8_t>(h, Ly.gs.depth_f, s);
                I.gs_db = upload<uint8_t>(h, Ly.gs.depth_b, s);
                I.gs_maxd = upload<int>(h, Ly.gs.maxd, s);
                I.gs_fresh = reinterpret_cast<const int2*>(upload<int>(h, Ly.gs.fresh, s));
                I.gs_nblk = (int)Ly.gs.maxd.size() / 2;
            }
        }
    }
    upload_values<double>(h, h->f64, lay, db, s);
    if (build_f32) upload_values<float>(h, h->f32, lay, db, s);
    const int n0 = h->idx[0].n;
    int maxn = 0;
    for (auto& I : h->idx) maxn = std::max(maxn, I.n);
    h->x = dalloc<double>(h, n0, s);
    h->r = dalloc<double>(h, n0, s);
    h->z = dalloc<double>(h, n0, s);
    h->p[0] = dalloc<double>(h, n0, s);
    h->p[1] = dalloc<double>(h, n0, s);
    h->q = dalloc<double>(h, n0, s);
    h->b = dalloc<double>(h, n0, s);
    h->dbg0 = dalloc<double>(h, maxn, s);
    h->dbg1 = dalloc<double>(h, maxn, s);
    h->dbg2 = dalloc<double>(h, maxn, s);
    if (build_f32) {
        h->r32 = dalloc<float>(h, n0, s);
        h->z32 = dalloc<float>(h, n0, s);
    }
    h->partial = dalloc<double>(h, 2 * kMaxGrid, s);
    h->partial_b = dalloc<double>(h, 2 * kMaxGrid, s);
    h->zero_flag = dalloc<int>(h, 1, s);
    h->st = dalloc<SolveState>(h, 1, s);
    HIP_CHECK(hipMemsetAsync(h->zero_flag, 0, sizeof(int), s));
    HIP_CHECK(hipMemsetAsync(h->st, 0, sizeof(SolveState), s));
    for (double* v : {h->x, h->r, h->z, h->p[0], h->p[1], h->q, h->b, h->dbg0, h->dbg1, h->dbg2})
        HIP_CHECK(hipMemsetAsync(v, 0, sizeof(double) * (v == h->dbg0 || v == h->dbg1 || v == h->dbg2 ? maxn : n0), s));
    HIP_CHECK(hipHostMalloc((void**)&h->st_host, sizeof(SolveState), hipHostMallocDefault));
    HIP_CHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_CHECK(hipStreamSynchronize(s));
    h->info.levels = nl;
    double tot = 0;
    for (int l = 0; l < nl && l < PAMG_MAX_LEVELS; ++l) {
        h->info.n[l] = h->idx[l].n;
        h->info.nnz[l] = h->idx[l].nnz;
        h->info.pairs[l] = h->host.lev[l].pairs;
        tot += (double)h->idx[l].nnz;
    }
    h->info.operator_complexity = tot / (double)h->idx[0].nnz;
    h->info.vcycle_bytes_f64 = vcycle_bytes(h, 8);
    h->info.vcycle_bytes_f32 = build_f32 ? vcycle_bytes(h, 4) : 0;
    h->info.csr_vcycle_bytes_f64 = csr_vcycle_bytes(h, 8);
    h->info.csr_vcycle_bytes_f32 = build_f32 ? csr_vcycle_bytes(h, 4) : 0;
    h->info.spmv_bytes = matrix_bytes(h->idx[0], false, 8) + 2 * 8 * (uint64_t)n0;
}

void destroy_hierarchy(pamg_hierarchy* h) {
    if (h->host_only) {
        if (h->ctx) h->ctx->users.fetch_sub(1);
        delete h;
        return;
    }
    (void)hipDeviceSynchronize();
    h->batch[0].reset();
    h->batch[1].reset();
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            if (h->graph[a][b]) (void)hipGraphExecDestroy(h->graph[a][b]);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    ctx_free_all(h->ctx, h->allocs);
    if (h->st_host) (void)hipHostFree(h->st_host);
    h->ctx->users.fetch_sub(1);
    delete h;
}

// ---------------------------------------------------------------- launchers

#define LAUNCH(kernel, grid, shmem, stream, ...)                                           \
    do {                                                                                   \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), shmem, stream, __VA_ARGS__); \
    } while (0)

// Call f with std::integral_constant<int, items> for the level's tile capacity.
template <typename F>
static void with_items(int items, F&& f) {
    switch (items) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default: f(std::integral_constant<int, 16>{}); break;
    }
}

template <typename T, typename RT>
static void launch_down(const DevLevelIdx& I, const T* vd, const RT* r, const T* p, T* rc, const int* done,
                        hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_down<IT, T, RT, RT>), tile_grid(I.n_down), (tile_lds_bytes<IT, T>(I.down_dmax)), s, (const int*)I.rp,
               (const int*)I.ci, vd, r, r, p, (const int*)I.aggptr, I.down_tiles, I.n_down, I.down_span, I.down_col,
               I.down_loc, rc, done);
    });
}

// Residual of a smoothed z and its restriction: rc = P^T (r - A z).
template <typename T, typename RT>
static void launch_resid_restrict(const DevLevelIdx& I, const T* v, const RT* r, const T* z, const T* p, T* rc,
                                  const int* done, hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_down<IT, T, RT, T>), tile_grid(I.n_down), (tile_lds_bytes<IT, T>(I.down_dmax)), s, (const int*)I.rp,
               (const int*)I.ci, v, r, z, p, (const int*)I.aggptr, I.down_tiles, I.n_down, I.down_span, I.down_col,
               I.down_loc, rc, done);
    });
}

// F: the finer level (l - 1) prolongated into, or nullptr at level 0 (OUT).
template <typename T, typename RT, typename RTF, bool OUT, typename ZO = double>
static void launch_up(const DevLevelIdx& I, const T* v, const T* zp, const RT* r, const T* dinv, const DevLevelIdx* F,
                      const RTF* r_f, const T* dinv_f, const T* p_f, T* zp_f,
                      typename std::common_type<ZO>::type* z_out, const double* dv,
                      double* partial, const int* done, hipStream_t s) {
    const int* aggptr_f = F ? (const int*)F->aggptr : nullptr;
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        if constexpr (OUT) {
            LAUNCH((k_up<IT, T, RT, RTF, kUpOut, ZO>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s, (const int*)I.rp,
                   (const int*)I.ci, v, zp, r, dinv, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc, aggptr_f,
                   r_f, dinv_f, p_f, zp_f, z_out, dv, partial, done);
        } else if (F->max_agg <= 2) {
            LAUNCH((k_up<IT, T, RT, RTF, kUpPair>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s, (const int*)I.rp,
                   (const int*)I.ci, v, zp, r, dinv, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc, aggptr_f,
                   r_f, dinv_f, p_f, zp_f, z_out, dv, partial, done);
        } else {
            LAUNCH((k_up<IT, T, RT, RTF, kUpWide>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s, (const int*)I.rp,
                   (const int*)I.ci, v, zp, r, dinv, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc, aggptr_f,
                   r_f, dinv_f, p_f, zp_f, z_out, dv, partial, done);
        }
    });
}

template <typename T, typename XT>
static void launch_spmv(const DevLevelIdx& I, const T* v, const XT* x, const double* b, double* y, double* partial,
                        hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_spmv<IT, T, XT, double>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s, (const int*)I.rp,
               (const int*)I.ci, v, x, b, (const T*)nullptr, y, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc,
               partial, (const int*)nullptr);
    });
}

// y = b - A x through the row tiles, any vector types; no partials.
template <typename T, typename XT, typename YT, typename BT>
static void launch_resid(const DevLevelIdx& I, const T* v, const XT* x, const BT* b, YT* y, hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_spmv<IT, T, XT, YT, BT>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s, (const int*)I.rp,
               (const int*)I.ci, v, x, b, (const T*)nullptr, y, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc,
               (double*)nullptr, (const int*)nullptr);
    });
}

// The l1-Jacobi step from x on a level: y = x + D^-1 (b - A x), through the
// level's row tiles (t = b - A x rounded to T first).
template <typename T, typename BT>
static void launch_smooth(const DevLevelIdx& I, const T* v, const T* x, const BT* b, const T* dinv, T* y,
                          const int* done, hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_spmv<IT, T, T, T, BT, kSpmvSmooth>), tile_grid(I.n_up), (tile_lds_bytes<IT, T>(I.up_dmax)), s,
               (const int*)I.rp, (const int*)I.ci, v, x, b, dinv, y, I.up_tiles, I.n_up, I.up_span, I.up_col,
               I.up_loc, (double*)nullptr, done);
    });
}

// y = z + M x with a tiled matrix M (the prolongated correction z + P e).
template <typename T>
static void launch_tiled_add(const DevTiled& M, const T* v, const T* x, const T* z, T* y, const int* done,
                             hipStream_t s) {
    with_items(M.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_spmv<IT, T, T, T, T, kSpmvAdd>), tile_grid(M.ntiles), (tile_lds_bytes<IT, T>(M.dmax)), s, M.rp, M.ci,
               v, x, z, (const T*)nullptr, y, M.tiles, M.ntiles, M.span, M.col, M.loc, (double*)nullptr, done);
    });
}

// Products with a tiled matrix M (the smoothed prolongator's P or P^T):
// y = M x, or with d: y_i = d_i b_i + (M x)_i.
template <typename T, typename BT>
static void launch_tiled(const DevTiled& M, const T* v, const T* x, const BT* b, const T* d, T* y, const int* done,
                         hipStream_t s) {
    with_items(M.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        if (d)
            LAUNCH((k_spmv<IT, T, T, T, BT, kSpmvProlong>), tile_grid(M.ntiles), (tile_lds_bytes<IT, T>(M.dmax)), s, M.rp,
                   M.ci, v, x, b, d, y, M.tiles, M.ntiles, M.span, M.col, M.loc, (double*)nullptr, done);
        else
            LAUNCH((k_spmv<IT, T, T, T, BT>), tile_grid(M.ntiles), (tile_lds_bytes<IT, T>(M.dmax)), s, M.rp, M.ci,
                   v, x, (const BT*)nullptr, (const T*)nullptr, y, M.tiles, M.ntiles, M.span, M.col, M.loc,
                   (double*)nullptr, done);
    });
}

template <typename ZT>
static void launch_krylov(const DevLevelIdx& I, const double* v, const ZT* z, const double* p_old, double* p_new,
                          double* q, const double* r, const SolveState* st, double* partial, const int* done,
                          hipStream_t s) {
    with_items(I.items, [&](auto it) {
        constexpr int IT = decltype(it)::value;
        LAUNCH((k_krylov_pq<IT, ZT>), tile_grid(I.n_up), (tile_lds_bytes<IT, double>(I.up_dmax)), s, (const int*)I.rp,
               (const int*)I.ci, v, z, p_old, p_new, q, r, I.up_tiles, I.n_up, I.up_span, I.up_col, I.up_loc, st,
               partial, done);
    });
}

template <typename T, typename RT, typename RTF, bool OUT>
static void launch_coarse(int nL, const T* ainv, const RT* r, const int* aggptr_f, const RTF* r_f, const T* dinv_f,
                          const T* p_f, T* zp_f, double* z_out, const double* dv, double* partial, const int* done,
                          hipStream_t s) {
    if (nL > kCoarseRowsMin) {
        hipLaunchKernelGGL((k_coarse_rows<T, RT, RTF, OUT>), dim3(coarse_rows_grid(nL)), dim3(kBlock), 0, s, nL, ainv,
                           r, aggptr_f, r_f, dinv_f, p_f, zp_f, z_out, dv, partial, done);
        return;
    }
    const int G = coarse_groups(nL);
    const size_t lds = (size_t)(1 + G) * nL * sizeof(T);
    hipLaunchKernelGGL((k_coarse<T, RT, RTF, OUT>), dim3(1), dim3(kCoarseThreads), lds, s, nL, G, ainv, r, aggptr_f,
                       r_f, dinv_f, p_f, zp_f, z_out, dv, partial, done);
}

// number of partials the coarsest level leaves when it writes z (single level)
static int coarse_partials(int nL) { return nL > kCoarseRowsMin ? coarse_rows_grid(nL) : 1; }

// ---------------------------------------------------------------- schedule

// One hybrid Gauss-Seidel sweep at level l from x_old into x_new (zero: from
// x_old = 0, the first pre-smoothing sweep, which needs no residual pass).
template <int MAXB, typename T, typename RT, int RB>
static void launch_hgs_rb(pamg_hierarchy* h, DevVals<T>& V, int l, const RT* r, const T* x_old, T* x_new,
                          bool backward, bool zero, const int* done, hipStream_t s) {
    const DevLevelIdx& I = h->idx[l];
    const T winv = (T)(1.0 / h->omega);
    const dim3 g(I.gs_nblk), blk(MAXB);
    if (zero) {
        hipLaunchKernelGGL((k_hgs<MAXB, T, RT, false, true, RB>), g, blk, 0, s, I.n, h->gs_block, (const int*)I.ci,
                           (const T*)V.v[l], I.gs_fresh, (const T*)V.gsa[l], I.gs_df, I.gs_maxd, r,
                           (const T*)nullptr, x_new, winv, done);
        return;
    }
    // t = r - A x_old through the row tiles
    launch_resid<T, T, T, RT>(I, V.v[l], x_old, r, V.gst[l], s);
    if (backward)
        hipLaunchKernelGGL((k_hgs<MAXB, T, T, true, false, RB>), g, blk, 0, s, I.n, h->gs_block, (const int*)I.ci,
                           (const T*)V.v[l], I.gs_fresh, (const T*)V.gsa[l], I.gs_db, I.gs_maxd, (const T*)V.gst[l],
                           x_old, x_new, winv, done);
    else
        hipLaunchKernelGGL((k_hgs<MAXB, T, T, false, false, RB>), g, blk, 0, s, I.n, h->gs_block, (const int*)I.ci,
                           (const T*)V.v[l], I.gs_fresh, (const T*)V.gsa[l], I.gs_df, I.gs_maxd, (const T*)V.gst[l],
                           x_old, x_new, winv, done);
}

// One sweep.  A level whose rows average kGsWideRow entries or more
// (smoothed coarse levels) loads the in-block entries past the registers
// kGsWideBatch at a time instead of kGsBatch, at the price of registers (two
// waves per SIMD): with blocks of 256 rows (many in-block entries per row),
// or with one-wave blocks when the level's waves fit the chip in one round.
template <int MAXB, typename T, typename RT>
static void launch_hgs(pamg_hierarchy* h, DevVals<T>& V, int l, const RT* r, const T* x_old, T* x_new, bool backward,
                       bool zero, const int* done, hipStream_t s) {
    const DevLevelIdx& I = h->idx[l];
    constexpr long long kWideWaves = 256LL * 4 * 2;  // CUs x SIMDs x waves per SIMD of the wide form
    const bool long_rows = I.nnz >= (long long)kGsWideRow * I.n;
    if (long_rows && (MAXB > kGsSmallBlock || (long long)I.gs_nblk * (MAXB / 64) <= kWideWaves))
        launch_hgs_rb<MAXB, T, RT, kGsWideBatch>(h, V, l, r, x_old, x_new, backward, zero, done, s);
    else
        launch_hgs_rb<MAXB, T, RT, kGsBatch>(h, V, l, r, x_old, x_new, backward, zero, done, s);
}

// `sweeps` hybrid Gauss-Seidel sweeps at level l on A_l x = r: forward from
// x = 0 (pre-smoothing) or backward from x (post-smoothing).  Ping-pongs
// between x and the level's second buffer; returns where the result is.
// Blocks of at most 64 rows run one wave per workgroup.
template <typename T, typename RT>
static T* enqueue_hgs(pamg_hierarchy* h, DevVals<T>& V, int l, const RT* r, T* x, bool backward, const int* done,
                      hipStream_t s) {
    T* a = x;
    T* b = (x == V.zt[l]) ? V.zp[l] : V.zt[l];
    for (int k = 0; k < h->sweeps; ++k) {
        const bool zero = !backward && k == 0;
        if (h->gs_block <= kGsSmallBlock)
            launch_hgs<kGsSmallBlock, T, RT>(h, V, l, r, a, b, backward, zero, done, s);
        else
            launch_hgs<kGsMaxBlock, T, RT>(h, V, l, r, a, b, backward, zero, done, s);
        std::swap(a, b);
    }
    return a;
}

// V-cycle with the hybrid Gauss-Seidel smoother (L >= 1): per level `sweeps`
// forward sweeps from zero, the residual and its restriction (tile kernel;
// with smoothed prolongators the residual, then P^T t through P^T's tiles),
// then after the coarse solve the prolongated correction (z + P e through
// P's tiles when smoothed) and `sweeps` backward sweeps.  Returns the number
// of z . dv partials.
template <typename T>
static int enqueue_vcycle_gs(pamg_hierarchy* h, DevVals<T>& V, const double* r0, double* z_out, const double* dv,
                             const int* done, hipStream_t s) {
    const int L = h->L;
    std::vector<T*> z(L + 1, nullptr);
    for (int l = 0; l < L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        if (l == 0)
            z[0] = enqueue_hgs<T, double>(h, V, 0, r0, V.zp[0], false, done, s);
        else
            z[l] = enqueue_hgs<T, T>(h, V, l, (const T*)V.r[l], V.zp[l], false, done, s);
        if (h->smoothed_p) {
            // t = r - A z (row tiles), then r_{l+1} = P^T t (tiles of P^T)
            if (l == 0)
                launch_resid<T, T, T, double>(I, V.v[0], (const T*)z[0], r0, V.gst[0], s);
            else
                launch_resid<T, T, T, T>(I, V.v[l], (const T*)z[l], (const T*)V.r[l], V.gst[l], s);
            launch_tiled<T, T>(I.sa_t, (const T*)V.sa_tv[l], (const T*)V.gst[l], (const T*)nullptr,
                               (const T*)nullptr, V.r[l + 1], done, s);
        } else if (l == 0) {
            launch_resid_restrict<T, double>(I, V.v[0], r0, z[0], V.p[0], V.r[1], done, s);
        } else {
            launch_resid_restrict<T, T>(I, V.v[l], V.r[l], z[l], V.p[l], V.r[l + 1], done, s);
        }
    }
    const int nL = h->idx[L].n;
    LAUNCH((k_gs_coarse<T, T>), coarse_rows_grid(nL), 0, s, nL, (const T*)V.ainv, (const T*)V.r[L], V.zc, done);
    z[L] = V.zc;
    for (int l = L - 1; l >= 0; --l) {
        const DevLevelIdx& I = h->idx[l];
        const int nc = h->idx[l + 1].n;
        if (h->smoothed_p) {
            // z + P e (tiles of P) into the level's other iterate buffer
            T* zn = z[l] == V.zp[l] ? V.zt[l] : V.zp[l];
            launch_tiled_add<T>(I.sa_p, (const T*)V.sa_pv[l], (const T*)z[l + 1], (const T*)z[l], zn, done, s);
            z[l] = zn;
        } else {
            LAUNCH((k_gs_prolong<T>), vec_grid(nc), 0, s, nc, (const int*)I.aggptr, (const T*)V.p[l],
                   (const T*)z[l + 1], z[l], done);
        }
        if (l == 0)
            z[0] = enqueue_hgs<T, double>(h, V, 0, r0, z[0], true, done, s);
        else
            z[l] = enqueue_hgs<T, T>(h, V, l, (const T*)V.r[l], z[l], true, done, s);
    }
    const int n0 = h->idx[0].n, g = vec_grid(n0);
    LAUNCH((k_gs_out<T>), g, 0, s, n0, (const T*)z[0], z_out, dv, h->partial, done);
    return g;
}

// V-cycle with smoothed prolongators (L >= 1; Sec. 3.1, P = (I - w D^-1 A) P^):
// per level the residual of the l1-Jacobi pre-smoothing from zero and its
// restriction P^T t; after the coarse solve the prolongation D^-1 r + P e
// and the post-smoothing.  P is no longer piecewise constant, so the
// restriction and the prolongation are products with P^T and P, each in the
// row-tile layout of a level's matrix (tiles and column dictionaries built
// for them at setup).
template <typename T>
static int enqueue_vcycle_sa(pamg_hierarchy* h, DevVals<T>& V, const double* r0, double* z_out, const double* dv,
                             const int* done, hipStream_t s) {
    const int L = h->L;
    for (int l = 0; l < L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        // t = r - (A D^-1) r through the row tiles (column-scaled values),
        // then r_{l+1} = P^T t through the tiles of P^T
        if (l == 0)
            launch_resid<T, double, T, double>(I, V.vd[0], r0, r0, V.zt[0], s);
        else
            launch_resid<T, T, T, T>(I, V.vd[l], (const T*)V.r[l], (const T*)V.r[l], V.zt[l], s);
        launch_tiled<T, T>(I.sa_t, (const T*)V.sa_tv[l], (const T*)V.zt[l], (const T*)nullptr, (const T*)nullptr,
                           V.r[l + 1], done, s);
    }
    const int nL = h->idx[L].n;
    LAUNCH((k_gs_coarse<T, T>), coarse_rows_grid(nL), 0, s, nL, (const T*)V.ainv, (const T*)V.r[L], V.zc, done);
    const T* e = V.zc;
    for (int l = L - 1; l >= 0; --l) {
        const DevLevelIdx& I = h->idx[l];
        // zp = D^-1 r + P e (tiles of P), then the post-smoothing
        // z = zp + D^-1 (r - A zp): into zt[l] on the levels below (the
        // residual there is no longer needed), at level 0 the output z with
        // the partials of z . dv (the level-0 up-sweep kernel)
        if (l == 0) {
            launch_tiled<T, double>(I.sa_p, (const T*)V.sa_pv[0], e, r0, (const T*)V.dinv[0], V.zp[0], done, s);
        } else {
            launch_tiled<T, T>(I.sa_p, (const T*)V.sa_pv[l], e, (const T*)V.r[l], (const T*)V.dinv[l], V.zp[l], done, s);
            launch_smooth<T, T>(I, V.v[l], (const T*)V.zp[l], (const T*)V.r[l], (const T*)V.dinv[l], V.zt[l], done, s);
            e = V.zt[l];
        }
    }
    const DevLevelIdx& I0 = h->idx[0];
    launch_up<T, double, double, true>(I0, V.v[0], V.zp[0], r0, V.dinv[0], nullptr, (const double*)nullptr, nullptr,
                                       nullptr, nullptr, z_out, dv, h->partial, done, s);
    return tile_grid(I0.n_up);
}

// The l1-Jacobi cycle with tentative prolongators; r0 of type R0 (the FP64
// residual, or its FP32 rounding for the FP32 cycle, whose kernels round
// every level-0 residual value they read to FP32 anyway).
template <typename T, typename R0, typename ZO = double>
static int enqueue_vcycle_plain(pamg_hierarchy* h, DevVals<T>& V, const R0* r0, ZO* z_out, const double* dv,
                                const int* done, hipStream_t s) {
    const int L = h->L;
    for (int l = 0; l < L; ++l) {
        const DevLevelIdx& I = h->idx[l];
        if (l == 0)
            launch_down<T, R0>(I, V.vd[0], r0, V.p[0], V.r[1], done, s);
        else
            launch_down<T, T>(I, V.vd[l], V.r[l], V.p[l], V.r[l + 1], done, s);
    }
    const int nL = h->idx[L].n;
    if constexpr (std::is_same<ZO, double>::value) {
        if (L == 0) {
            launch_coarse<T, R0, R0, true>(nL, V.ainv, r0, nullptr, (const R0*)nullptr, nullptr, nullptr, nullptr,
                                           z_out, dv, h->partial, done, s);
            return coarse_partials(nL);
        }
    }
    const DevLevelIdx& F = h->idx[L - 1];
    if (L - 1 == 0)
        launch_coarse<T, T, R0, false>(nL, V.ainv, V.r[L], F.aggptr, r0, V.dinv[0], V.p[0], V.zp[0], nullptr,
                                       nullptr, nullptr, done, s);
    else
        launch_coarse<T, T, T, false>(nL, V.ainv, V.r[L], F.aggptr, V.r[L - 1], V.dinv[L - 1], V.p[L - 1],
                                      V.zp[L - 1], nullptr, nullptr, nullptr, done, s);
    for (int l = L - 1; l >= 1; --l) {
        const DevLevelIdx& I = h->idx[l];
        const DevLevelIdx& Fi = h->idx[l - 1];
        if (l - 1 == 0)
            launch_up<T, T, R0, false>(I, V.v[l], V.zp[l], V.r[l], V.dinv[l], &Fi, r0, V.dinv[0], V.p[0],
                                       V.zp[0], nullptr, nullptr, nullptr, done, s);
        else
            launch_up<T, T, T, false>(I, V.v[l], V.zp[l], V.r[l], V.dinv[l], &Fi, V.r[l - 1], V.dinv[l - 1],
                                      V.p[l - 1], V.zp[l - 1], nullptr, nullptr, nullptr, done, s);
    }
    const DevLevelIdx& I0 = h->idx[0];
    launch_up<T, R0, R0, true, ZO>(I0, V.v[0], V.zp[0], r0, V.dinv[0], nullptr, (const R0*)nullptr, nullptr, nullptr,
                                   nullptr, z_out, dv, h->partial, done, s);
    return tile_grid(I0.n_up);
}

// z_out = B r0 on level 0 (r0, z_out FP64, hierarchical order); the level-0
// up-sweep also writes the partials of z . dv.  Returns the number of partials.
// The FP32 cycle first rounds r0 to FP32 once (r32): its level-0 kernels then
// gather 4-byte values, with the same results.
// z32_out (FP32 cycle with tentative prolongators and l1-Jacobi, L >= 1
// only; else null): z written there in FP32, exactly, instead of z_out.
template <typename T>
static int enqueue_vcycle(pamg_hierarchy* h, DevVals<T>& V, const double* r0, double* z_out, const double* dv,
                          const int* done, hipStream_t s, float* z32_out = nullptr) {
    const int L = h->L;
    if (h->smoother == PAMG_SMOOTHER_HYBRID_GS && L > 0) return enqueue_vcycle_gs<T>(h, V, r0, z_out, dv, done, s);
    if (h->smoothed_p && L > 0) return enqueue_vcycle_sa<T>(h, V, r0, z_out, dv, done, s);
    if constexpr (std::is_same<T, float>::value) {
        if (h->r32) {
            const long long n0 = h->idx[0].n;
            hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_grid(n0)), dim3(kBlock), 0, s, n0, r0, h->r32);
            if (z32_out && L > 0)
                return enqueue_vcycle_plain<float, float, float>(h, V, (const float*)h->r32, z32_out, dv, done, s);
            return enqueue_vcycle_plain<float, float>(h, V, (const float*)h->r32, z_out, dv, done, s);
        }
    }
    return enqueue_vcycle_plain<T, double>(h, V, r0, z_out, dv, done, s);
}

// Whether the FP32 cycle hands z to the Krylov pass in FP32 (z32).
template <typename T>
static bool cycle_z32(const pamg_hierarchy* h) {
    return std::is_same<T, float>::value && h->z32 && h->r32 && h->L > 0 &&
           h->smoother == PAMG_SMOOTHER_L1_JACOBI && !h->smoothed_p;
}

template <typename T>
static void enqueue_iteration(pamg_hierarchy* h, DevVals<T>& V, int krylov, int parity, hipStream_t s) {
    const int* done = &h->st->done;
    const double* dv = (krylov == PAMG_KRYLOV_CG) ? h->r : h->q;
    const bool z32 = cycle_z32<T>(h);
    const int cnt = enqueue_vcycle<T>(h, V, h->r, h->z, dv, done, s, z32 ? h->z32 : nullptr);
    LAUNCH(k_fin_beta, 1, 0, s, h->st, (const double*)h->partial, cnt);
    const DevLevelIdx& I = h->idx[0];
    if (z32)
        launch_krylov<float>(I, h->f64.v[0], h->z32, h->p[parity], h->p[1 - parity], h->q, h->r, h->st, h->partial,
                             done, s);
    else
        launch_krylov<double>(I, h->f64.v[0], h->z, h->p[parity], h->p[1 - parity], h->q, h->r, h->st, h->partial,
                              done, s);
    LAUNCH(k_fin_alpha, 1, 0, s, h->st, (const double*)h->partial, tile_grid(I.n_up));
    const int gv = vec_grid(I.n);
    LAUNCH(k_krylov_update, gv, 0, s, I.n, h->x, h->r, (const double*)h->p[1 - parity], (const double*)h->q,
           (const SolveState*)h->st, h->partial, done);
    LAUNCH(k_fin_norm, 1, 0, s, h->st, (const double*)h->partial, gv);
}

template <typename T>
static void enqueue_block(pamg_hierarchy* h, DevVals<T>& V, int krylov, int k, hipStream_t s) {
    for (int j = 0; j < k; ++j) enqueue_iteration<T>(h, V, krylov, j & 1, s);
}

template <typename T>
static hipGraphExec_t get_graph(pamg_hierarchy* h, DevVals<T>& V, int prec, int krylov, int k) {
    hipGraphExec_t& ex = h->graph[prec][krylov];
    if (ex && h->graph_k[prec][krylov] == k) return ex;
    if (ex) {
        HIP_CHECK(hipGraphExecDestroy(ex));
        ex = nullptr;
    }
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_block<T>(h, V, krylov, k, h->cap_stream);
    HIP_CHECK(hipStreamEndCapture(h->cap_stream, &g));
    HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    HIP_CHECK(hipGraphDestroy(g));
    h->graph_k[prec][krylov] = k;
    return ex;
}

static void read_state_async(pamg_hierarchy* h, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(h->st_host, h->st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
}

static void read_state(pamg_hierarchy* h, hipStream_t s) {
    read_state_async(h, s);
    HIP_CHECK(hipStreamSynchronize(s));
}

// ||b - A x|| / ||b|| for the hierarchical-order x, b; uses dbg0 as scratch.
static double true_relres(pamg_hierarchy* h, hipStream_t s) {
    const DevLevelIdx& I = h->idx[0];
    const int g = tile_grid(I.n_up);
    launch_spmv<double, double>(I, h->f64.v[0], h->x, h->b, h->dbg0, h->partial_b, s);
    double part[kMaxGrid];        // g <= kMaxGrid; no heap allocation on the solve path
    HIP_CHECK(hipMemcpyAsync(part, h->partial_b, sizeof(double) * g, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    double rr = 0.0;
    for (int i = 0; i < g; ++i) rr += part[i];
    return std::sqrt(rr) / h->st_host->bnorm;
}

// Start of a solve: the recurrence state, b in hierarchical order, x (x0 or
// zero) and r = b - A x.  The host copy of the state is the staging buffer,
// so the stream must have passed any earlier copy through it.
static void begin_solve(pamg_hierarchy* h, const double* b_user, const double* x0_user, double tol, int maxit,
                        int fixed_iters, int krylov, hipStream_t s) {
    const DevLevelIdx& I0 = h->idx[0];
    const int n = I0.n;
    const int gv = vec_grid(n);
    SolveState init{};
    init.tol = tol;
    init.maxit = maxit;
    init.fixed_iters = fixed_iters;
    init.krylov = krylov;
    *h->st_host = init;
    HIP_CHECK(hipMemcpyAsync(h->st, h->st_host, sizeof(SolveState), hipMemcpyHostToDevice, s));
    LAUNCH((k_gather<double, double>), gv, 0, s, n, (const int*)I0.iperm, b_user, h->b);
    LAUNCH(k_norm2, gv, 0, s, n, (const double*)h->b, (double*)nullptr, h->partial_b);
    if (x0_user) {
        LAUNCH((k_gather<double, double>), gv, 0, s, n, (const int*)I0.iperm, x0_user, h->x);
        launch_spmv<double, double>(I0, h->f64.v[0], h->x, h->b, h->r, h->partial, s);
        LAUNCH(k_fin_init, 1, 0, s, h->st, (const double*)h->partial_b, gv, (const double*)h->partial,
               tile_grid(I0.n_up));
    } else {
        LAUNCH(k_fill, gv, 0, s, (long long)n, h->x, 0.0);
        LAUNCH(k_norm2, gv, 0, s, n, (const double*)h->b, h->r, h->partial);
        LAUNCH(k_fin_init, 1, 0, s, h->st, (const double*)h->partial_b, gv, (const double*)h->partial, gv);
    }
}

// k iterations (a replay of `ex` when given), then the state copy to the host.
template <typename T>
static void run_block(pamg_hierarchy* h, DevVals<T>& V, int krylov, int k, hipGraphExec_t ex, hipStream_t s) {
    if (ex)
        HIP_CHECK(hipGraphLaunch(ex, s));
    else
        enqueue_block<T>(h, V, krylov, k, s);
    read_state_async(h, s);
}

// The recurrence restarted from the true residual r = b - A x (the FP32
// preconditioner's recurrence residual can drift from it); then the state copy.
static void restart_solve(pamg_hierarchy* h, hipStream_t s) {
    const DevLevelIdx& I0 = h->idx[0];
    launch_spmv<double, double>(I0, h->f64.v[0], h->x, h->b, h->r, h->partial, s);
    LAUNCH(k_fin_init, 1, 0, s, h->st, (const double*)h->partial_b, 0, (const double*)h->partial,
           tile_grid(I0.n_up));
    read_state_async(h, s);
}

// x in the caller's numbering (zero for a zero right-hand side); the host
// copy of the state must be current.
static void end_solve(pamg_hierarchy* h, double* x_user, hipStream_t s) {
    const DevLevelIdx& I0 = h->idx[0];
    const int n = I0.n;
    const int gv = vec_grid(n);
    if (h->st_host->done == 2) LAUNCH(k_fill, gv, 0, s, (long long)n, h->x, 0.0);
    LAUNCH((k_gather<double, double>), gv, 0, s, n, (const int*)I0.perm, (const double*)h->x, x_user);
}

template <typename T>
static void solve_impl(pamg_hierarchy* h, DevVals<T>& V, int prec, const double* b_user, double* x_user,
                       const pamg_solve_opts& o, hipStream_t s, pamg_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    const int krylov = o.krylov == PAMG_KRYLOV_CG ? PAMG_KRYLOV_CG : PAMG_KRYLOV_FCG;
    // wait for any earlier use of the pinned staging buffer
    HIP_CHECK(hipStreamSynchronize(s));
    begin_solve(h, b_user, o.use_x0 ? x_user : nullptr, o.tol, o.maxit, o.fixed_iters, krylov, s);
    int k = o.check_every > 0 ? o.check_every : 4;
    if (k & 1) ++k;
    hipGraphExec_t ex = o.use_graph ? get_graph<T>(h, V, prec, krylov, k) : nullptr;
    int restarts = 0;
    double relres_true = -1.0;
    read_state(h, s);
    for (;;) {
        while (!h->st_host->done) {
            run_block<T>(h, V, krylov, k, ex, s);
            HIP_CHECK(hipStreamSynchronize(s));
        }
        if (h->st_host->done == 2) break;   // zero right-hand side
        const bool want_true = o.true_residual || prec == PAMG_PREC_F32;
        if (!want_true || h->st_host->status != PAMG_OK || o.fixed_iters > 0) break;
        relres_true = true_relres(h, s);
        if (relres_true <= o.tol || prec != PAMG_PREC_F32 || restarts >= 10 || h->st_host->iter >= o.maxit) break;
        ++restarts;
        restart_solve(h, s);
        HIP_CHECK(hipStreamSynchronize(s));
        relres_true = -1.0;
    }
    end_solve(h, x_user, s);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->status = h->st_host->status;
        info->iterations = h->st_host->iter;
        info->restarts = restarts;
        info->relres = h->st_host->bnorm > 0 ? h->st_host->rnorm / h->st_host->bnorm : 0.0;
        info->relres_true = relres_true;
        info->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
}

// ---------------------------------------------------------------- no-allocation solve
// pamg_solve for callers that cannot allocate: the solve state and the
// reduction partials live in `scratch`, a static device array (one copy per
// GPU, held until the process ends), instead of the hierarchy's buffers, and
// the iterations are launched directly (instantiating a graph allocates).
// In host code `scratch` names a host-side stand-in: its device address on
// each GPU comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels and copies.
constexpr size_t kScratchStateOff = 0;                  // SolveState
constexpr size_t kScratchFlagOff = 256;                 // an int that stays 0
constexpr size_t kScratchPartials = 2 * (size_t)kMaxGrid;
constexpr size_t kScratchPartOff = 512;                 // partials (kScratchPartials doubles)
constexpr size_t kScratchPartBOff = kScratchPartOff + kScratchPartials * sizeof(double);
constexpr size_t kScratchBytes = kScratchPartBOff + kScratchPartials * sizeof(double);
static_assert(sizeof(SolveState) <= kScratchFlagOff, "solve state exceeds its scratch slot");
static_assert(kScratchBytes == PAMG_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (taken on the first call there).
static unsigned char* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error(PAMG_E_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        HIP_CHECK(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error(PAMG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<unsigned char*>(p);
    }
    return g_scratch_dev[device];
}

// The hierarchy's state and partial buffers pointed at the scratch for the
// duration of one call (the hierarchy's lock is held), restored after.
struct ScratchView {
    pamg_hierarchy* h;
    SolveState* st;
    double *partial, *partial_b;
    int* zero_flag;
    ScratchView(pamg_hierarchy* hh, unsigned char* base)
        : h(hh), st(hh->st), partial(hh->partial), partial_b(hh->partial_b), zero_flag(hh->zero_flag) {
        h->st = reinterpret_cast<SolveState*>(base + kScratchStateOff);
        h->zero_flag = reinterpret_cast<int*>(base + kScratchFlagOff);
        h->partial = reinterpret_cast<double*>(base + kScratchPartOff);
        h->partial_b = reinterpret_cast<double*>(base + kScratchPartBOff);
    }
    ~ScratchView() {
        h->st = st;
        h->partial = partial;
        h->partial_b = partial_b;
        h->zero_flag = zero_flag;
    }
};

// Partials the solve's reductions write into one buffer (both hold
// kScratchPartials): the Krylov pass two per workgroup, the level-0 up-sweep
// or the single-level coarse product, the vector kernels.
static size_t solve_partials(const pamg_hierarchy* h) {
    const DevLevelIdx& I0 = h->idx[0];
    size_t need = 2 * (size_t)tile_grid(I0.n_up);
    need = std::max(need, (size_t)vec_grid(I0.n));
    if (h->L == 0) need = std::max(need, (size_t)coarse_partials(h->idx[0].n));
    return need;
}

int solve_noalloc(pamg_hierarchy* h, const double* b, double* x, pamg_solve_opts o, hipStream_t s,
                  pamg_solve_info* info) {
    require_device(h);
    std::lock_guard<std::mutex> lk(h->mu);
    unsigned char* base = scratch_address(h->device);
    HIP_CHECK(hipSetDevice(h->device));
    const size_t need = solve_partials(h);
    if (need > kScratchPartials)
        throw Error(PAMG_E_INVALID, "the hierarchy's reductions need " + std::to_string(need) +
                                        " partials; the static scratch holds " + std::to_string(kScratchPartials));
    if (o.precision == PAMG_PREC_F32 && !h->f32.built)
        throw Error(PAMG_E_INVALID, "FP32 hierarchy not built (set params.build_f32)");
    ScratchView view(h, base);
    // the array keeps the last call's contents: state and flag start from zero
    LAUNCH(k_fill, 1, 0, s, (long long)(kScratchPartOff / sizeof(double)), reinterpret_cast<double*>(base), 0.0);
    o.use_graph = 0;
    pamg_solve_info tmp{};
    if (!info) info = &tmp;
    if (o.precision == PAMG_PREC_F32)
        solve_impl<float>(h, h->f32, 1, b, x, o, s, info);
    else
        solve_impl<double>(h, h->f64, 0, b, x, o, s, info);
    return info->status;
}

void require_device(const pamg_hierarchy* h) {
    if (h->host_only) throw Error(PAMG_E_INVALID, "hierarchy was built with host_only=1");
}

int solve(pamg_hierarchy* h, const double* b, double* x, const pamg_solve_opts& o, hipStream_t s,
          pamg_solve_info* info) {
    require_device(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    pamg_solve_info tmp{};
    if (!info) info = &tmp;
    if (o.precision == PAMG_PREC_F32) {
        if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built (set params.build_f32)");
        solve_impl<float>(h, h->f32, 1, b, x, o, s, info);
    } else {
        solve_impl<double>(h, h->f64, 0, b, x, o, s, info);
    }
    return info->status;
}

// ---------------------------------------------------------------- stepped solve
// The serving loop drives a single-right-hand-side FCG solve step by step on
// its own stream, with the arithmetic of solve() (x0 = 0): the caller orders
// the steps and waits for the stream before reading single_state.

void single_begin(pamg_hierarchy* h, const double* b, double tol, int maxit, hipStream_t s) {
    require_device(h);
    begin_solve(h, b, nullptr, tol, maxit, 0, PAMG_KRYLOV_FCG, s);
}

void single_block(pamg_hierarchy* h, int prec, int k, bool use_graph, hipStream_t s) {
    if (k & 1) ++k;
    if (prec == PAMG_PREC_F32) {
        if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built (set params.build_f32)");
        run_block<float>(h, h->f32, PAMG_KRYLOV_FCG, k,
                         use_graph ? get_graph<float>(h, h->f32, 1, PAMG_KRYLOV_FCG, k) : nullptr, s);
    } else {
        run_block<double>(h, h->f64, PAMG_KRYLOV_FCG, k,
                          use_graph ? get_graph<double>(h, h->f64, 0, PAMG_KRYLOV_FCG, k) : nullptr, s);
    }
}

void single_prepare_graph(pamg_hierarchy* h, int prec, int k) {
    if (k & 1) ++k;
    if (prec == PAMG_PREC_F32)
        (void)get_graph<float>(h, h->f32, 1, PAMG_KRYLOV_FCG, k);
    else
        (void)get_graph<double>(h, h->f64, 0, PAMG_KRYLOV_FCG, k);
}

const SolveState& single_state(const pamg_hierarchy* h) { return *h->st_host; }
double single_true_relres(pamg_hierarchy* h, hipStream_t s) { return true_relres(h, s); }
void single_restart(pamg_hierarchy* h, hipStream_t s) { restart_solve(h, s); }

void single_end(pamg_hierarchy* h, double* x, hipStream_t s) {
    end_solve(h, x, s);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

// Algorithmic bytes of one iteration: the V-cycle, the FP64 Krylov product
// and twelve level-0 vector passes.
uint64_t single_iteration_bytes(const pamg_hierarchy* h, int prec) {
    const uint64_t n0 = (uint64_t)h->idx[0].n;
    return vcycle_bytes(h, prec == PAMG_PREC_F32 ? 4 : 8) + matrix_bytes(h->idx[0], false, 8) + 12 * n0 * 8;
}

// ---------------------------------------------------------------- debug ops

template <typename T>
static void debug_impl(pamg_hierarchy* h, DevVals<T>& V, int op, int l, const double* in0, const double* in1,
                       double* out, hipStream_t s) {
    const int* nodone = h->zero_flag;
    const DevLevelIdx& I = h->idx[l];
    const int gv = vec_grid(I.n);
    switch (op) {
        case PAMG_OP_SPMV: {
            LAUNCH((k_gather<double, T>), gv, 0, s, I.n, (const int*)I.iperm, in0, V.dbg_in);
            launch_spmv<T, T>(I, V.v[l], V.dbg_in, nullptr, h->dbg1, nullptr, s);
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.perm, (const double*)h->dbg1, out);
            break;
        }
        case PAMG_OP_DOWN: {
            if (l >= h->L) throw Error(PAMG_E_INVALID, "DOWN needs level < L");
            const DevLevelIdx& C = h->idx[l + 1];
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
            LAUNCH((k_gather<double, T>), gv, 0, s, I.n, (const int*)I.iperm, in0, V.dbg_in);
            if (l == 0)
                launch_down<T, double>(I, V.vd[0], h->dbg0, V.p[0], V.dbg_in2, nodone, s);
            else
                launch_down<T, T>(I, V.vd[l], V.dbg_in, V.p[l], V.dbg_in2, nodone, s);
            LAUNCH((k_gather<T, double>), vec_grid(C.n), 0, s, C.n, (const int*)C.perm, (const T*)V.dbg_in2, out);
            break;
        }
        case PAMG_OP_UP: {
            // out = in1 + D^-1 (in0 - A in1): the post-smoothing step
            if (l >= h->L) throw Error(PAMG_E_INVALID, "UP needs level < L");
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
            LAUNCH((k_gather<double, T>), gv, 0, s, I.n, (const int*)I.iperm, in1, V.dbg_in);
            launch_up<T, double, double, true>(I, V.v[l], V.dbg_in, h->dbg0, V.dinv[l], nullptr,
                                               (const double*)nullptr, nullptr, nullptr, nullptr, h->dbg1, h->dbg0,
                                               h->partial, nodone, s);
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.perm, (const double*)h->dbg1, out);
            break;
        }
        case PAMG_OP_PROLONG: {
            // out = D^-1 in0 + P in1
            if (l >= h->L) throw Error(PAMG_E_INVALID, "PROLONG needs level < L");
            const DevLevelIdx& C = h->idx[l + 1];
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
            LAUNCH((k_gather<double, T>), vec_grid(C.n), 0, s, C.n, (const int*)C.iperm, in1, V.dbg_in);
            LAUNCH((k_prolong<T>), vec_grid(C.n), 0, s, C.n, (const T*)V.dbg_in, (const int*)I.aggptr,
                   (const double*)h->dbg0, (const T*)V.dinv[l], (const T*)V.p[l], V.dbg_in2);
            LAUNCH((k_gather<T, double>), gv, 0, s, I.n, (const int*)I.perm, (const T*)V.dbg_in2, out);
            break;
        }
        case PAMG_OP_COARSE: {
            if (l != h->L) throw Error(PAMG_E_INVALID, "COARSE needs level == L");
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
            launch_coarse<T, double, double, true>(I.n, V.ainv, h->dbg0, nullptr, (const double*)nullptr, nullptr,
                                                   nullptr, nullptr, h->dbg1, h->dbg0, h->partial, nodone, s);
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.perm, (const double*)h->dbg1, out);
            break;
        }
        case PAMG_OP_SMOOTH: {
            // hybrid GS sweeps: forward from zero on r = in0, or backward from x = in1
            if (h->smoother != PAMG_SMOOTHER_HYBRID_GS || l >= h->L)
                throw Error(PAMG_E_INVALID, "SMOOTH needs a hybrid Gauss-Seidel hierarchy and level < L");
            const bool back = in1 != nullptr;
            if (back) LAUNCH((k_gather<double, T>), gv, 0, s, I.n, (const int*)I.iperm, in1, V.zp[l]);
            T* res;
            if (l == 0) {
                LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
                res = enqueue_hgs<T, double>(h, V, 0, (const double*)h->dbg0, V.zp[0], back, nodone, s);
            } else {
                LAUNCH((k_gather<double, T>), gv, 0, s, I.n, (const int*)I.iperm, in0, V.dbg_in);
                res = enqueue_hgs<T, T>(h, V, l, (const T*)V.dbg_in, V.zp[l], back, nodone, s);
            }
            LAUNCH((k_gather<T, double>), gv, 0, s, I.n, (const int*)I.perm, (const T*)res, out);
            break;
        }
        case PAMG_OP_VCYCLE: {
            if (l != 0) throw Error(PAMG_E_INVALID, "VCYCLE is applied at level 0");
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.iperm, in0, h->dbg0);
            enqueue_vcycle<T>(h, V, h->dbg0, h->dbg1, h->dbg0, nodone, s);
            LAUNCH((k_gather<double, double>), gv, 0, s, I.n, (const int*)I.perm, (const double*)h->dbg1, out);
            break;
        }
        default:
            throw Error(PAMG_E_INVALID, "unknown operator");
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

int debug_apply(pamg_hierarchy* h, int op, int level, int prec, const double* in0, const double* in1, double* out,
                hipStream_t s) {
    require_device(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    if (level < 0 || level > h->L) throw Error(PAMG_E_INVALID, "level out of range");
    if (prec == PAMG_PREC_F32) {
        if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built");
        debug_impl<float>(h, h->f32, op, level, in0, in1, out, s);
    } else {
        debug_impl<double>(h, h->f64, op, level, in0, in1, out, s);
    }
    return PAMG_OK;
}

// ---------------------------------------------------------------- timing

template <typename F>
static double time_launches(F&& launch, int reps, hipStream_t s) {
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    for (int w = 0; w < 2; ++w) launch();
    HIP_CHECK(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) launch();
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    HIP_CHECK(hipGetLastError());
    float a = 0;
    HIP_CHECK(hipEventElapsedTime(&a, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)a / reps;
}

template <typename T>
static void time_impl(pamg_hierarchy* h, DevVals<T>& V, const double* r, int reps, hipStream_t s, double* vms,
                      double* sms) {
    const DevLevelIdx& I = h->idx[0];
    LAUNCH((k_gather<double, double>), vec_grid(I.n), 0, s, I.n, (const int*)I.iperm, r, h->dbg0);
    *vms = time_launches([&]() { enqueue_vcycle<T>(h, V, h->dbg0, h->dbg1, h->dbg0, h->zero_flag, s); }, reps, s);
    *sms = time_launches([&]() { launch_spmv<double, double>(I, h->f64.v[0], h->dbg1, nullptr, h->dbg2, nullptr, s); },
                         reps, s);
}

int time_kernels(pamg_hierarchy* h, int prec, const double* r, int reps, hipStream_t s, double* vms, double* sms) {
    require_device(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    if (reps < 1) throw Error(PAMG_E_INVALID, "reps must be >= 1");
    if (prec == PAMG_PREC_F32) {
        if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built");
        time_impl<float>(h, h->f32, r, reps, s, vms, sms);
    } else {
        time_impl<double>(h, h->f64, r, reps, s, vms, sms);
    }
    return PAMG_OK;
}

template <typename T>
static void time_op_impl(pamg_hierarchy* h, DevVals<T>& V, int op, int l, int reps, hipStream_t s, double* ms,
                         uint64_t* bytes) {
    const DevLevelIdx& I = h->idx[l];
    const int* nodone = h->zero_flag;
    const uint64_t n = I.n, nnz = I.nnz, sz = sizeof(T);
    const uint64_t M = matrix_bytes(I, op == PAMG_OP_DOWN, sz);
    (void)nnz;
    std::function<void()> launch;
    if (op == PAMG_OP_DOWN) {
        if (l >= h->L) throw Error(PAMG_E_INVALID, "DOWN needs level < L");
        const uint64_t nc = h->idx[l + 1].n;
        // scaled matrix, own r/p (r in FP64 at level 0), aggptr, coarse output
        *bytes = M + n * (l == 0 ? 8 : sz) + n * sz + 4 * (nc + 1) + nc * sz;
        if (l == 0)
            launch = [=]() { launch_down<T, double>(I, V.vd[0], h->r, V.p[0], V.r[1], nodone, s); };
        else
            launch = [=]() { launch_down<T, T>(I, V.vd[l], V.r[l], V.p[l], V.r[l + 1], nodone, s); };
    } else if (op == PAMG_OP_UP) {
        if (l >= h->L) throw Error(PAMG_E_INVALID, "UP needs level < L");
        if (l == 0) {
            // matrix, own zp/dinv (T), r and dv (FP64), z out (FP64)
            *bytes = M + 2 * n * sz + 3 * n * 8;
            launch = [=]() {
                launch_up<T, double, double, true>(I, V.v[0], V.zp[0], h->r, V.dinv[0], nullptr,
                                                   (const double*)nullptr, nullptr, nullptr, nullptr, h->z, h->q,
                                                   h->partial, nodone, s);
            };
        } else {
            const DevLevelIdx& F = h->idx[l - 1];
            const uint64_t nf = F.n;
            // matrix, own zp/r/dinv, fine aggptr, fine r/dinv/p reads and zp write
            *bytes = M + 3 * n * sz + 4 * (n + 1) + nf * ((l - 1 == 0 ? 8 : sz) + 3 * sz);
            if (l - 1 == 0)
                launch = [=]() {
                    launch_up<T, T, double, false>(I, V.v[l], V.zp[l], V.r[l], V.dinv[l], &F, h->r, V.dinv[0],
                                                   V.p[0], V.zp[0], nullptr, nullptr, nullptr, nodone, s);
                };
            else
                launch = [=]() {
                    launch_up<T, T, T, false>(I, V.v[l], V.zp[l], V.r[l], V.dinv[l], &F, V.r[l - 1],
                                              V.dinv[l - 1], V.p[l - 1], V.zp[l - 1], nullptr, nullptr, nullptr,
                                              nodone, s);
                };
        }
    } else if (op == PAMG_OP_SPMV) {
        *bytes = M + n * sz + n * 8;
        launch = [=]() { launch_spmv<T, T>(I, V.v[l], V.dbg_in, nullptr, h->dbg1, nullptr, s); };
    } else if (op == PAMG_OP_KRYLOV) {
        if (l != 0) throw Error(PAMG_E_INVALID, "KRYLOV runs on level 0");
        const uint64_t M8 = matrix_bytes(I, false, 8);
        // matrix (FP64), z, p_old, q_old, r reads; p_new, q writes
        *bytes = M8 + 6 * n * 8;
        launch = [=]() {
            launch_krylov<double>(I, h->f64.v[0], h->z, h->p[0], h->p[1], h->q, h->r, h->st, h->partial, nodone, s);
        };
    } else if (op == PAMG_OP_SMOOTH) {
        // one backward hybrid Gauss-Seidel sweep: CSR (int32 columns), own r,
        // x_old, 1/a_ii, depth, x_new; per block its largest depths
        if (h->smoother != PAMG_SMOOTHER_HYBRID_GS || l >= h->L)
            throw Error(PAMG_E_INVALID, "SMOOTH needs a hybrid Gauss-Seidel hierarchy and level < L");
        *bytes = I.nnz * (4 + sz) + 4 * (n + 1) + n * ((l == 0 ? 8 : sz) + 3 * sz + 1) + 8 * (uint64_t)I.gs_nblk;
        DevVals<T>* Vp = &V;
        const bool small = h->gs_block <= kGsSmallBlock;
        if (l == 0)
            launch = [=]() {
                if (small)
                    launch_hgs<kGsSmallBlock, T, double>(h, *Vp, 0, (const double*)h->r, Vp->zp[0], Vp->zt[0], true,
                                                         false, nodone, s);
                else
                    launch_hgs<kGsMaxBlock, T, double>(h, *Vp, 0, (const double*)h->r, Vp->zp[0], Vp->zt[0], true,
                                                       false, nodone, s);
            };
        else
            launch = [=]() {
                if (small)
                    launch_hgs<kGsSmallBlock, T, T>(h, *Vp, l, (const T*)Vp->r[l], Vp->zp[l], Vp->zt[l], true, false,
                                                    nodone, s);
                else
                    launch_hgs<kGsMaxBlock, T, T>(h, *Vp, l, (const T*)Vp->r[l], Vp->zp[l], Vp->zt[l], true, false,
                                                  nodone, s);
            };
    } else {
        throw Error(PAMG_E_INVALID, "op must be DOWN, UP, SPMV, KRYLOV or SMOOTH");
    }
    *ms = time_launches(launch, reps, s);
}

int time_op(pamg_hierarchy* h, int op, int level, int prec, int reps, hipStream_t s, double* ms, uint64_t* bytes) {
    require_device(h);
    std::lock_guard<std::mutex> lk(h->mu);
    HIP_CHECK(hipSetDevice(h->device));
    if (reps < 1) throw Error(PAMG_E_INVALID, "reps must be >= 1");
    if (level < 0 || level > h->L) throw Error(PAMG_E_INVALID, "level out of range");
    if (prec == PAMG_PREC_F32) {
        if (!h->f32.built) throw Error(PAMG_E_INVALID, "FP32 hierarchy not built");
        if (op == PAMG_OP_KRYLOV) throw Error(PAMG_E_INVALID, "KRYLOV is FP64 only");
        time_op_impl<float>(h, h->f32, op, level, reps, s, ms, bytes);
    } else {
        time_op_impl<double>(h, h->f64, op, level, reps, s, ms, bytes);
    }
    return PAMG_OK;
}

pamg_hierarchy* new_hierarchy(bool host_only, pamg_context* ctx) {
    if (!host_only && !ctx) {
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        ctx = default_context(dev);
    }
    if (!host_only) HIP_CHECK(hipSetDevice(ctx->device));
    pamg_hierarchy* h = new pamg_hierarchy();
    h->host_only = host_only;
    h->ctx = ctx;
    if (ctx) {
        h->device = ctx->device;
        ctx->users.fetch_add(1);
    }
    return h;
}

}  // namespace pamg

// ============================================================================
// C ABI
// ============================================================================

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace pamg {
void set_last_error(const std::string& m) { g_last_error = m; }
}

namespace pamg {

void check_params(const pamg_params& prm) {
    if (prm.max_coarse < 1 || prm.max_levels < 1 || prm.max_levels > PAMG_MAX_LEVELS || prm.max_dense < 1 ||
        prm.max_dense > kMaxDense || !(prm.min_ratio == prm.min_ratio) || prm.agg_steps < 1 || prm.agg_steps > kMaxAggSteps)
        throw Error(PAMG_E_INVALID, "bad params (need max_coarse >= 1, 1 <= max_levels <= 64, "
                                    "1 <= max_dense <= 8192, min_ratio not NaN, 1 <= agg_steps <= 4)");
    if (prm.smoother == PAMG_SMOOTHER_L1_JACOBI) {
        if (prm.sweeps != 0 && prm.sweeps != 1)
            throw Error(PAMG_E_INVALID, "the l1-Jacobi smoother runs one sweep per side (sweeps 0 or 1)");
    } else if (prm.smoother == PAMG_SMOOTHER_HYBRID_GS) {
        if (prm.sweeps < 0 || prm.sweeps > 16 || prm.gs_block < 0 || prm.gs_block > 256 ||
            !(prm.omega >= 0.0) || std::isinf(prm.omega))
            throw Error(PAMG_E_INVALID, "bad hybrid Gauss-Seidel params (need 0 <= sweeps <= 16, "
                                        "0 <= gs_block <= 256, finite omega >= 0; 0 = default)");
    } else {
        throw Error(PAMG_E_INVALID, "unknown smoother");
    }
    if (prm.smooth_prolongator != 0 && prm.smooth_prolongator != 1)
        throw Error(PAMG_E_INVALID, "smooth_prolongator must be 0 or 1");
    if (prm.device_setup != 0 && prm.device_setup != 1) throw Error(PAMG_E_INVALID, "device_setup must be 0 or 1");
    if (prm.device_min_rows < 0) throw Error(PAMG_E_INVALID, "device_min_rows must be >= 0");
}

std::unique_ptr<HostBuild> host_build(const pamg_csr& A, const pamg_params& prm) {
    check_params(prm);
    set_num_threads(prm.num_threads > 0 ? prm.num_threads : 0);
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<HostBuild> b(new HostBuild());
    b->prm = prm;
    validate_csr(A, prm.check_symmetry != 0);
    b->H = build_hierarchy(A, prm);
    b->lay = build_layout(b->H);
    if (prm.smoother == PAMG_SMOOTHER_HYBRID_GS) {
        const int nb = prm.gs_block > 0 ? prm.gs_block : 256;
        for (size_t l = 0; l + 1 < b->lay.size(); ++l) b->lay[l].gs = gs_schedule(b->lay[l], nb);
    }
    if (prm.smooth_prolongator)
        for (size_t l = 0; l + 1 < b->lay.size(); ++l) sa_layout(b->H.lev[l].P, b->lay[l], b->lay[l + 1], b->lay[l]);
    b->host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return b;
}

int coarsest_n(const HostBuild& b) { return b.H.lev.back().A.n; }

pamg_hierarchy* finish_build(std::unique_ptr<HostBuild> b, hipStream_t stream, pamg_context* ctx) {
    auto t0 = std::chrono::steady_clock::now();
    pamg_hierarchy* h = new_hierarchy(b->prm.host_only != 0, ctx);
    h->smoother = b->prm.smoother;
    h->smoothed_p = b->prm.smooth_prolongator != 0;
    if (h->smoother == PAMG_SMOOTHER_HYBRID_GS) {
        h->sweeps = b->prm.sweeps > 0 ? b->prm.sweeps : 4;
        h->gs_block = b->prm.gs_block > 0 ? b->prm.gs_block : 256;
        h->omega = b->prm.omega > 0.0 ? b->prm.omega : 1.5;
    }
    for (size_t l = 0; l < b->lay.size() && l < (size_t)PAMG_MAX_LEVELS; ++l) h->info.tile_items[l] = b->lay[l].items;
    try {
        h->host = std::move(b->H);
        if (b->prm.host_only) {
            const int nl = (int)h->host.lev.size();
            h->L = nl - 1;
            h->info.levels = nl;
            double tot = 0;
            for (int l = 0; l < nl; ++l) {
                h->info.n[l] = h->host.lev[l].A.n;
                h->info.nnz[l] = h->host.lev[l].A.nnz();
                h->info.pairs[l] = h->host.lev[l].pairs;
                tot += (double)h->info.nnz[l];
            }
            h->info.operator_complexity = tot / (double)h->info.nnz[0];
        } else {
            upload_hierarchy(h, b->lay, b->prm.build_f32 != 0, stream, nullptr);
        }
    } catch (...) {
        destroy_hierarchy(h);
        throw;
    }
    const double dev_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    h->info.setup_ms = b->host_ms + dev_ms;
    return h;
}

pamg_hierarchy* device_setup_build(const pamg_csr& A, const pamg_params& prm, hipStream_t stream,
                                   pamg_context* ctx) {
    auto t0 = std::chrono::steady_clock::now();
    set_num_threads(prm.num_threads > 0 ? prm.num_threads : 0);
    validate_csr_header(A);   // the rows are checked on the device (or by the host build)
    pamg_hierarchy* h = new_hierarchy(false, ctx);
    try {
        std::unique_ptr<DeviceBuild> db = device_build(h, A, prm, stream);
        if (!db) {
            destroy_hierarchy(h);
            return nullptr;
        }
        const int m = db->m;
        h->host.lev.resize(m);
        for (int l = 0; l < m; ++l) {
            h->host.lev[l].A.n = db->dev[l].n;
            h->host.lev[l].pairs = db->dev[l].pairs;
        }
        for (HostLevel& hl : db->host.lev) h->host.lev.push_back(std::move(hl));
        h->lazy_levels = m;
        h->prm = prm;
        const int nl = m + (int)db->host_lay.size();
        h->smoother = prm.smoother;
        if (h->smoother == PAMG_SMOOTHER_HYBRID_GS) {
            h->sweeps = prm.sweeps > 0 ? prm.sweeps : 4;
            h->gs_block = prm.gs_block > 0 ? prm.gs_block : 256;
            h->omega = prm.omega > 0.0 ? prm.omega : 1.5;
            // the Gauss-Seidel schedule of every level but the coarsest: on
            // the device for the device-built levels, on the host for the rest
            for (int l = 0; l < m && l + 1 < nl; ++l) device_gs_schedule(h, db->dev[l], h->gs_block, stream);
            for (int l = m; l + 1 < nl; ++l) db->host_lay[l - m].gs = gs_schedule(db->host_lay[l - m], h->gs_block);
        }
        for (int l = 0; l < nl && l < PAMG_MAX_LEVELS; ++l)
            h->info.tile_items[l] = l < m ? db->dev[l].items : db->host_lay[l - m].items;
        upload_hierarchy(h, db->host_lay, prm.build_f32 != 0, stream, db.get());
        h->info.device_levels = m;
    } catch (...) {
        destroy_hierarchy(h);
        throw;
    }
    h->info.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return h;
}

void ensure_host_levels(pamg_hierarchy* h) {
    std::lock_guard<std::mutex> lk(h->host_mu);
    if (h->lazy_levels == 0) return;
    HIP_CHECK(hipSetDevice(h->device));
    HIP_CHECK(hipDeviceSynchronize());
    auto get = [](auto& out, const auto* d, size_t count) {
        out.resize(count);
        if (count) HIP_CHECK(hipMemcpy(out.data(), d, count * sizeof(out[0]), hipMemcpyDeviceToHost));
    };
    // with composed aggregates the pairwise chain between kept levels exists
    // only during the build: rebuild the whole host hierarchy (bitwise the
    // same) from the canonical level-0 matrix
    const bool composed = h->prm.agg_steps > 1;
    const int upto = composed ? 1 : h->lazy_levels;
    for (int l = 0; l < upto; ++l) {
        const DevLevelIdx& I = h->idx[l];
        const int n = I.n, nc = I.nc;
        std::vector<int32_t> rp, ci, perm, iperm, aggptr, ciperm;
        std::vector<double> v, dinv, p;
        get(rp, I.rp, (size_t)n + 1);
        get(ci, I.ci, (size_t)I.nnz);
        get(v, h->f64.v[l], (size_t)I.nnz);
        get(perm, I.perm, (size_t)n);
        get(iperm, I.iperm, (size_t)n);
        get(dinv, h->f64.dinv[l], (size_t)n);
        get(p, h->f64.p[l], (size_t)n);
        get(aggptr, I.aggptr, (size_t)nc + 1);
        get(ciperm, h->idx[l + 1].iperm, (size_t)nc);
        HostLevel& H = h->host.lev[l];
        H.A.n = n;
        H.A.rp.assign(n + 1, 0);
        for (int32_t i = 0; i < n; ++i) H.A.rp[i + 1] = H.A.rp[i] + (rp[perm[i] + 1] - rp[perm[i]]);
        H.A.ci.resize(I.nnz);
        H.A.v.resize(I.nnz);
        H.dinv.resize(n);
        H.p.resize(n);
        H.agg.resize(n);
        parallel_ranges(n, [&](int, int64_t b, int64_t e) {
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t i = b; i < e; ++i) {
                const int32_t ip = perm[i];
                row.clear();
                for (int32_t k = rp[ip]; k < rp[ip + 1]; ++k) row.emplace_back(iperm[ci[k]], v[k]);
                std::sort(row.begin(), row.end(), [](const std::pair<int32_t, double>& x,
                                                     const std::pair<int32_t, double>& y) { return x.first < y.first; });
                const int32_t o = H.A.rp[i];
                for (size_t u = 0; u < row.size(); ++u) {
                    H.A.ci[o + u] = row[u].first;
                    H.A.v[o + u] = row[u].second;
                }
                H.dinv[i] = dinv[ip];
                H.p[i] = p[ip];
            }
        });
        for (int32_t Ip = 0; Ip < nc; ++Ip)
            for (int32_t ip = aggptr[Ip]; ip < aggptr[Ip + 1]; ++ip) H.agg[iperm[ip]] = ciperm[Ip];
    }
    if (composed) {
        const HostCSR& A0 = h->host.lev[0].A;
        const pamg_csr c{A0.n, A0.nnz(), A0.rp.data(), A0.ci.data(), A0.v.data()};
        HostHierarchy full = build_hierarchy(c, h->prm);
        h->host = std::move(full);
    }
    h->lazy_levels = 0;
}

}  // namespace pamg

extern "C" {

const char* pamg_last_error(void) { return g_last_error.c_str(); }

int pamg_params_default(pamg_params* p) {
    if (!p) return PAMG_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->max_coarse = 200;
    p->max_levels = 50;
    p->max_dense = pamg::kMaxDense;
    p->min_ratio = 1.5;
    p->agg_steps = 1;
    p->match_all_edges = 0;
    p->build_f32 = 0;
    p->num_threads = 0;
    p->check_symmetry = 0;
    p->device_setup = 1;
    p->device_min_rows = 0;
    return PAMG_OK;
}

int pamg_solve_opts_default(pamg_solve_opts* o) {
    if (!o) return PAMG_E_INVALID;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6;
    o->maxit = 1000;
    o->krylov = PAMG_KRYLOV_FCG;
    o->precision = PAMG_PREC_F64;
    o->check_every = 4;
    o->use_graph = 1;
    return PAMG_OK;
}

int pamg_setup(pamg_context* ctx, const pamg_csr* A, const pamg_params* params, void* stream, pamg_hierarchy** out) {
    return pamg::guarded([&]() -> int {
        if (!A || !out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        *out = nullptr;
        pamg_params prm;
        if (params) prm = *params; else pamg_params_default(&prm);
        pamg::check_params(prm);
        if (pamg::device_setup_applies(prm)) {
            *out = pamg::device_setup_build(*A, prm, (hipStream_t)stream, ctx);
            if (*out) return PAMG_OK;
        }
        std::unique_ptr<pamg::HostBuild> hb = pamg::host_build(*A, prm);
        *out = pamg::finish_build(std::move(hb), (hipStream_t)stream, ctx);
        return PAMG_OK;
    });
}

int pamg_hierarchy_destroy(pamg_hierarchy* h) {
    return pamg::guarded([&]() -> int {
        if (h) pamg::destroy_hierarchy(h);
        return PAMG_OK;
    });
}

int pamg_hierarchy_info(const pamg_hierarchy* h, pamg_hier_info* out) {
    if (!h || !out) { g_last_error = "null argument"; return PAMG_E_INVALID; }
    *out = h->info;
    return PAMG_OK;
}

int pamg_hierarchy_aggregates(const pamg_hierarchy* h, int32_t level, int32_t* agg) {
    return pamg::guarded([&]() -> int {
        if (!h || !agg) throw pamg::Error(PAMG_E_INVALID, "null argument");
        if (level < 0 || level >= h->L) throw pamg::Error(PAMG_E_INVALID, "level must be in [0, levels-2]");
        pamg::ensure_host_levels(const_cast<pamg_hierarchy*>(h));
        const auto& a = h->host.lev[level].agg;
        std::memcpy(agg, a.data(), a.size() * sizeof(int32_t));
        return PAMG_OK;
    });
}

int pamg_hierarchy_level_csr(const pamg_hierarchy* h, int32_t level, int32_t* rp, int32_t* ci, double* v) {
    return pamg::guarded([&]() -> int {
        if (!h || !rp || !ci || !v) throw pamg::Error(PAMG_E_INVALID, "null argument");
        if (level < 0 || level > h->L) throw pamg::Error(PAMG_E_INVALID, "level out of range");
        pamg::ensure_host_levels(const_cast<pamg_hierarchy*>(h));
        const auto& A = h->host.lev[level].A;
        std::memcpy(rp, A.rp.data(), A.rp.size() * sizeof(int32_t));
        std::memcpy(ci, A.ci.data(), A.ci.size() * sizeof(int32_t));
        if (h->values_updated)
            pamg::updated_level_values(h, level, v);
        else
            std::memcpy(v, A.v.data(), A.v.size() * sizeof(double));
        return PAMG_OK;
    });
}

int pamg_solve(pamg_hierarchy* h, const double* b, double* x, const pamg_solve_opts* opts, void* stream,
               pamg_solve_info* info) {
    return pamg::guarded([&]() -> int {
        if (!h || !b || !x) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg_solve_opts o;
        if (opts) o = *opts; else pamg_solve_opts_default(&o);
        if (!(o.tol >= 0.0) || o.maxit < 1 || o.fixed_iters < 0)
            throw pamg::Error(PAMG_E_INVALID, "bad solve options (need tol >= 0, maxit >= 1)");
        return pamg::solve(h, b, x, o, (hipStream_t)stream, info);
    });
}

int pamg_solve_noalloc(pamg_hierarchy* h, const double* b, double* x, const pamg_solve_opts* opts, void* stream,
                       pamg_solve_info* info) {
    return pamg::guarded([&]() -> int {
        if (!h || !b || !x) throw pamg::Error(PAMG_E_INVALID, "null argument");
        pamg_solve_opts o;
        if (opts) o = *opts; else pamg_solve_opts_default(&o);
        if (!(o.tol >= 0.0) || o.maxit < 1 || o.fixed_iters < 0)
            throw pamg::Error(PAMG_E_INVALID, "bad solve options (need tol >= 0, maxit >= 1)");
        return pamg::solve_noalloc(h, b, x, o, (hipStream_t)stream, info);
    });
}

int pamg_debug_apply(pamg_hierarchy* h, int32_t op, int32_t level, int32_t precision, const double* in0,
                     const double* in1, double* out, void* stream) {
    return pamg::guarded([&]() -> int {
        if (!h || !in0 || !out) throw pamg::Error(PAMG_E_INVALID, "null argument");
        if ((op == PAMG_OP_UP || op == PAMG_OP_PROLONG) && !in1) throw pamg::Error(PAMG_E_INVALID, "in1 required");
        return pamg::debug_apply(h, op, level, precision, in0, in1, out, (hipStream_t)stream);
    });
}

int pamg_time_kernels(pamg_hierarchy* h, int32_t precision, const double* r, int32_t reps, void* stream,
                      double* vms, double* sms) {
    return pamg::guarded([&]() -> int {
        if (!h || !r || !vms || !sms) throw pamg::Error(PAMG_E_INVALID, "null argument");
        return pamg::time_kernels(h, precision, r, reps, (hipStream_t)stream, vms, sms);
    });
}

int pamg_time_op(pamg_hierarchy* h, int32_t op, int32_t level, int32_t precision, int32_t reps, void* stream,
                 double* ms, uint64_t* bytes) {
    return pamg::guarded([&]() -> int {
        if (!h || !ms || !bytes) throw pamg::Error(PAMG_E_INVALID, "null argument");
        return pamg::time_op(h, op, level, precision, reps, (hipStream_t)stream, ms, bytes);
    });
}

}  // extern "C"
