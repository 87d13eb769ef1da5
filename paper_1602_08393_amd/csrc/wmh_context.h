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
constexpr uint32_t kCoarseCodeBits = 15;  // default (and largest) resolution of coarse codes
constexpr uint64_t kStreamBudgetBytes = 1ull << 30;  // shared position stream, at most 1 GiB

// What the content of the shared position stream depends on.
struct StreamKey {
    uint64_t seed = 0;
    uint32_t k = 0, depth = 0, scale = 0;
    bool packed = false;
    uint64_t bounds_epoch = 0;
    uint32_t coarse_bits = 0;  // offsets replaced by their coarse codes of this many bits
    bool operator==(const StreamKey &o) const
    {
        return seed == o.seed && k == o.k && depth == o.depth && scale == o.scale &&
               packed == o.packed && bounds_epoch == o.bounds_epoch &&
               coarse_bits == o.coarse_bits;
    }
};

struct GraphKey {
    const void *row_ptr = nullptr, *col = nullptr, *val = nullptr;
    void *sig = nullptr;
    uint64_t n_rows = 0, nnz = 0, seed = 0;
    uint32_t k = 0, R = 0, K = 0, J = 0, depth = 0, waves = 0, grid = 0, groups = 0;
    bool narrow = false, packed = false, independent_rows = false, ballot = false;
    uint32_t coarse_bits = 0;  // 0: exact dense rows
    const void *row_class = nullptr;  // row filter of a split walk (nullptr: every row)
    uint32_t keep = 0;
    uint64_t bounds_epoch = 0;
    // the component index's rows kernel (the walk fields above then stay 0)
    bool indexed = false;
    const void *index_keys = nullptr, *index_steps = nullptr, *index_offsets = nullptr;
    uint32_t ix_batch = 0, ix_claim = 0;
    bool operator==(const GraphKey &o) const
    {
        return row_ptr == o.row_ptr && col == o.col && val == o.val && sig == o.sig &&
               row_class == o.row_class && keep == o.keep && indexed == o.indexed &&
               index_keys == o.index_keys && index_steps == o.index_steps &&
               index_offsets == o.index_offsets && ix_batch == o.ix_batch &&
               ix_claim == o.ix_claim &&
               n_rows == o.n_rows && nnz == o.nnz && seed == o.seed && k == o.k && R == o.R &&
               K == o.K &&
               J == o.J && depth == o.depth && waves == o.waves && grid == o.grid &&
               groups == o.groups &&
               narrow == o.narrow && packed == o.packed && coarse_bits == o.coarse_bits &&
               independent_rows == o.independent_rows && ballot == o.ballot &&
               bounds_epoch == o.bounds_epoch;
    }
};

// Row statistics gathered by the validation pass (device) or the host check, for the planner.
struct RowStats {
    bool known = false;
    uint64_t nonempty = 0;       // rows with sum(x) > 0
    uint64_t min_green = ~0ull;  // smallest sum(x) over non-empty rows
    uint64_t walk_steps = 0;     // sum over non-empty rows of min(M / sum(x), 65535)
    uint64_t index_keys = 0;     // sum over non-empty rows of the index keys read per hash
    bool keys_known = false;     // index_keys was estimated
    // row split (per-row classes written to the context's row_class buffer)
    bool split_known = false;
    uint64_t walk_rows = 0, walk_min_green = ~0ull, walk_class_steps = 0;
    uint64_t index_rows = 0, index_nnz = 0, index_class_keys = 0;
};

// A component index owned by a context or a serving loop, rebuilt when its key changes.
struct OwnedIndex {
    IndexBuffers buf;
    uint64_t cap_entries = 0;
    uint32_t cap_dims = 0;
    bool valid = false;
    uint64_t seed = 0, epoch = 0;
    uint32_t k = 0;
    hipEvent_t used = nullptr;  // recorded after each read, awaited before a rebuild
};

constexpr uint64_t kIndexBudgetBytes = 4ull << 30;  // each key order of the index, at most 4 GiB

enum class Path { kPlain, kBatched, kIndexed, kSplit, kPlainShared };

// Autotuned batched plans, per (D, value width, k, step class); step class = floor(log2) of
// the mean capped step count of the tuned rows.
struct TuneKey {
    uint32_t dims = 0;
    bool narrow = false;
    uint32_t k = 0;
    int32_t steps_class = -1;
    bool operator==(const TuneKey &o) const
    {
        return dims == o.dims && narrow == o.narrow && k == o.k && steps_class == o.steps_class;
    }
};

struct TuneEntry {
    TuneKey key;
    uint32_t R = 0, J = 0, W = 0, K = 0, G = 1;  // G: hash groups of the ballot walk
    int32_t V = 1;  // wmh_opts.values: 1 exact dense rows, 2 coarse codes
    int32_t walk = 1;  // wmh_opts.walk: 1 shared windows, 2 independent rows, 3 ballot walk
    float ms = 0.f;
};

// An autotuned plan of the component index's rows kernel, for rows the planner sends there.
struct IndexTuneEntry {
    TuneKey key;
    IndexPlan plan;
    float ms = 0.f;
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
    // per block of kBoundBlock components: the smallest bound, then (after all minima) the
    // rounded mean bound; for the validation pass when m does not fit in LDS (nullptr when D
    // is small enough for m itself, or too large for the table)
    uint32_t *d_bound_blocks = nullptr;
    // per-call scratch
    wmh::CheckWords *d_check = nullptr;
    wmh::CheckWords *h_check = nullptr;  // pinned
    uint8_t *d_row_class = nullptr;      // row split: one class byte per row
    uint64_t row_class_cap = 0;
    unsigned long long *d_tile_counter = nullptr;
    unsigned long long *d_row_counter = nullptr;  // rows claimed by the index rows kernel
    unsigned long long *d_codec = nullptr;  // codec counters: saturated values, maximum
    unsigned long long *h_codec = nullptr;  // pinned copy
    void *d_stream = nullptr;
    size_t stream_bytes = 0;
    // the shared position stream is kept between calls: it depends only on (seed, k, depth,
    // entry layout, bounds); stream_ready is recorded after its build
    bool stream_valid = false;
    wmh::StreamKey stream_key{};
    hipEvent_t stream_ready = nullptr;
    // graph of the batched launch
    hipGraphExec_t graph_exec = nullptr;
    wmh::GraphKey graph_key;
    // profiling events: [0] before the stream build, [1] before the walk, [2] after the walk
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool profiled = false;
    bool profiled_stream = false;
    wmh::OwnedIndex index;  // component index of the last indexed call
    int32_t last_mode = 0;  // path of the last successful wmh_hash (wmh_mode)
    wmh::BatchedPlan last_plan{};  // its batched plan (when batched)
    std::vector<wmh::TuneEntry> tuned;  // autotuner results
    std::vector<wmh::IndexTuneEntry> tuned_index;
    wmh::IndexPlan last_index_plan{};  // index rows plan of the last indexed call
    int servers = 0;  // live serving loops using this context's bounds
    std::string last_error;
};

namespace wmh {

wmh_status fail(wmh_ctx *ctx, wmh_status st, const char *fmt, ...);
// Status of a validation-pass error code (the low four bits of CheckWords::first_error).
wmh_status check_status(uint32_t code);
wmh_status device_fail(wmh_ctx *ctx, hipError_t e, const char *what);
Bounds bounds_view(const wmh_ctx *ctx);
// Tile plan of the batched walk; false when no dense plan fits in LDS.  Options left at 0
// take the autotuned plan for (ctx, k, stats) when there is one and use_tuned is set.
bool plan_batched(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o,
                  BatchedPlan *plan, bool use_tuned = true);
TuneKey tune_key(const wmh_ctx *ctx, uint32_t k, const RowStats &stats);
// Validation pass on the device: checks the rows (when check) and fills *stats; waits.
// want_keys: also estimate index_keys (only the path choice in auto mode reads it);
// want_split (with want_keys): also class every row for a row split (ctx->d_row_class).
// words: device words the pass writes (nullptr: the context's own).
wmh_status gather_stats(wmh_ctx *ctx, const Rows &rows, uint32_t k, hipStream_t s, bool check,
                        bool want_keys, RowStats *stats, bool want_split = false,
                        CheckWords *words = nullptr);
// Whether an index for k hashes is allowed (k and memory limits).
bool index_fits(uint32_t k);
// Makes `ix` the index of (ctx's bounds, seed, k), building it on `stream` when stale.
// With record_error false the context's error text is left alone (calls from the serving
// loop's worker thread).
wmh_status ensure_index(wmh_ctx *ctx, OwnedIndex *ix, uint64_t seed, uint32_t k,
                        hipStream_t stream, bool record_error = true);
void free_index(OwnedIndex *ix);
// The planner's choice for `mode` (AUTO compares estimated costs; see wmh_mode).  split_ok: a
// batched plan fits for the rows a split would walk (stats.split_known needed).
Path choose_path(const wmh_ctx *ctx, int mode, bool batched_ok, bool index_ready, uint32_t k,
                 uint64_t n_rows, uint64_t nnz, const RowStats &stats, bool split_ok = false);
// The statistics of the rows a split walks, as plan_batched reads them.
RowStats walk_class_stats(const RowStats &stats);
// Plan of the index rows kernel: the options' (waves_per_block, index_batch, index_claim)
// when any is set, else the autotuned plan of the rows' key (or the same (D, width, k) at the
// nearest step class within two), else the launcher's defaults.  False when the options do
// not fit.
bool plan_index(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o,
                IndexPlan *plan);

// The static device scratch of wmh_hash_noalloc (wmh_noalloc.hip): looks up its address on
// `device`, which must be current, once per device; later calls return the first result.
hipError_t static_scratch_init(int device);

}  // namespace wmh
