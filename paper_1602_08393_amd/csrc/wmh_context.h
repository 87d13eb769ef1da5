// Private to libwmh: the context object and the host helpers shared by the C-ABI entry points
// (wmh_host.cpp) and the serving loop (wmh_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/wmh.h"
#include "wmh_internal.h"

namespace wmh {

constexpr uint32_t kMaxDims = 1u << 26;
constexpr uint32_t kMaxK = 1u << 24;
constexpr uint64_t kStreamBudgetBytes = 1ull << 30;  // shared position stream, at most 1 GiB

struct GraphKey {
    const void *row_ptr = nullptr, *col = nullptr, *val = nullptr;
    void *sig = nullptr;
    uint64_t n_rows = 0, nnz = 0, seed = 0;
    uint32_t k = 0, R = 0, J = 0, depth = 0, waves = 0, grid = 0;
    bool narrow = false, packed = false;
    uint64_t bounds_epoch = 0;
    bool operator==(const GraphKey &o) const
    {
        return row_ptr == o.row_ptr && col == o.col && val == o.val && sig == o.sig &&
               n_rows == o.n_rows && nnz == o.nnz && seed == o.seed && k == o.k && R == o.R &&
               J == o.J && depth == o.depth && waves == o.waves && grid == o.grid &&
               narrow == o.narrow && packed == o.packed && bounds_epoch == o.bounds_epoch;
    }
};

}  // namespace wmh

struct wmh_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int cu_count = 0;
    // bounds
    bool has_bounds = false;
    uint64_t bounds_epoch = 0;
    uint32_t dims = 0;
    uint64_t total = 0;
    uint64_t threshold = 0;
    uint32_t shift = 0;
    uint64_t n_buckets = 0;
    uint32_t max_bound = 0;
    std::vector<uint32_t> h_bound;  // host copy of m, for host-side checks
    uint64_t *d_prefix = nullptr;
    uint32_t *d_bucket = nullptr;
    uint32_t *d_bound = nullptr;
    // per-call scratch
    wmh::CheckWords *d_check = nullptr;
    wmh::CheckWords *h_check = nullptr;  // pinned
    uint32_t *d_tile_counter = nullptr;
    void *d_stream = nullptr;
    size_t stream_bytes = 0;
    // graph of the batched launch
    hipGraphExec_t graph_exec = nullptr;
    wmh::GraphKey graph_key;
    // profiling events: [0] before the stream build, [1] before the walk, [2] after the walk
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool profiled = false;
    bool profiled_stream = false;
    int servers = 0;  // live serving loops using this context's bounds
    std::string last_error;
};

namespace wmh {

wmh_status fail(wmh_ctx *ctx, wmh_status st, const char *fmt, ...);
wmh_status device_fail(wmh_ctx *ctx, hipError_t e, const char *what);
Bounds bounds_view(const wmh_ctx *ctx);
// Tile plan of the batched walk; false when no dense plan fits in LDS.
bool plan_batched(const wmh_ctx *ctx, uint32_t k, uint64_t min_green, const wmh_opts &o,
                  BatchedPlan *plan);
// Host-side check of CSR rows against the context's bounds (same rules as the device check).
wmh_status check_rows_host(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                           const uint32_t *val, uint64_t n_rows, uint64_t nnz,
                           uint64_t *min_green);

}  // namespace wmh
