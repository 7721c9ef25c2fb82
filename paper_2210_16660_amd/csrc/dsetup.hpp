// Device construction of the large levels of the hierarchy (dsetup.hip).
#pragma once

#include "hier.hpp"

namespace pamg {

// Levels with at most this many rows (or the dense or coarsening limit, if
// larger) are built on the host.
constexpr int kDeviceMinRows = 65536;

// Column dictionaries of a level's tiles (TileDict on the device).
struct DevDict {
    int* span = nullptr;        // 2 per tile: first entry, length
    int* col = nullptr;
    uint16_t* loc = nullptr;    // per matrix entry
    long long len = 0;
    int max_len = 0;
};

// One device-built level in hierarchical numbering (LayoutLevel on the
// device); its arrays belong to the hierarchy's allocation list.
struct DevLevelOut {
    int n = 0, nc = 0, pairs = 0, items = 8, n_up = 0, n_down = 0, max_agg = 0;
    long long nnz = 0;
    int *rp = nullptr, *ci = nullptr, *perm = nullptr, *iperm = nullptr, *aggptr = nullptr;
    int *up_tiles = nullptr, *down_tiles = nullptr;
    double *v = nullptr, *vd = nullptr, *dinv = nullptr, *p = nullptr;
    DevDict up_dict, down_dict;
    // hybrid Gauss-Seidel schedule (GsLevel on the device; device_gs_schedule)
    uint8_t *gs_df = nullptr, *gs_db = nullptr;
    int *gs_maxd = nullptr, *gs_fresh = nullptr;
    double* gs_ainv = nullptr;
    int gs_nblk = 0;
};

struct DeviceBuild {
    int m = 0;                          // (kept) levels 0..m-1 built on the device
    std::vector<DevLevelOut> dev;
    HostHierarchy host;                 // levels m..L, built on the host from level m
    std::vector<LayoutLevel> host_lay;  // their layouts
};

// The hybrid Gauss-Seidel schedule of a device-built level with blocks of nb
// rows: the host's gs_schedule, row by row and block by block, on the
// device (depths, in-block entry ranges, 1 / a_ii); arrays allocated on h.
// A non-positive diagonal gives PAMG_E_NOT_SPD, as on the host.
void device_gs_schedule(pamg_hierarchy* h, DevLevelOut& D, int nb, hipStream_t s);

// The configurations the device construction covers: pairwise aggregates
// or their composition, tentative prolongators, the l1-Jacobi or the hybrid
// Gauss-Seidel smoother, weight-eligible edges.
bool device_setup_applies(const pamg_params& prm);

// Build the hierarchy of A (validated host CSR) with its large levels on the
// device; device arrays are allocated on h.  Null: nothing to build on the
// device (a small or asymmetric-pattern input, or long rows): the host build
// applies.
std::unique_ptr<DeviceBuild> device_build(pamg_hierarchy* h, const pamg_csr& A, const pamg_params& prm,
                                          hipStream_t s);

}  // namespace pamg
