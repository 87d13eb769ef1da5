// Host side of libwmh: the C-ABI declared in include/wmh.h.
//
// wmh_set_bounds does the paper's one-time preprocessing (Sec. 3.1; Algorithm 4): prefix sums
// of the bounds and a lookup structure from positions to components.  Algorithm 4 stores one
// entry per integer of [0, M), which is infeasible here (M reaches 2^40), so the lookup is a
// uniform bucket table: bucket b covers positions [b << shift, (b+1) << shift) and stores the
// component owning its first position; with about two buckets per dimension the search inside
// a bucket is O(1) expected.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

namespace wmh {

wmh_status fail(wmh_ctx *ctx, wmh_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return st;
}

wmh_status device_fail(wmh_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? WMH_E_NOMEM : WMH_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

const char *check_name(uint32_t code)
{
    switch (code) {
    case kCheckRowPtr: return "row_ptr decreasing or beyond nnz";
    case kCheckColumn: return "column index >= D";
    case kCheckUnsorted: return "columns not strictly increasing";
    case kCheckBound: return "value above its bound m_i";
    default: return "?";
    }
}

wmh_status check_status(uint32_t code)
{
    switch (code) {
    case kCheckRowPtr: return WMH_E_ROW_PTR;
    case kCheckColumn: return WMH_E_COL_RANGE;
    case kCheckUnsorted: return WMH_E_UNSORTED;
    case kCheckBound: return WMH_E_BOUND;
    default: return WMH_E_DEVICE;
    }
}

Bounds bounds_view(const wmh_ctx *ctx)
{
    Bounds b;
    b.prefix = ctx->d_prefix;
    b.bucket = ctx->d_bucket;
    b.bound = ctx->d_bound;
    b.total = ctx->total;
    b.threshold = ctx->threshold;
    b.shift = ctx->shift;
    b.dims = ctx->dims;
    return b;
}

// Tile plan of the batched walk.  Returns false when no dense plan fits in LDS.
TuneKey tune_key(const wmh_ctx *ctx, uint32_t k, const RowStats &stats)
{
    TuneKey key;
    key.dims = ctx->dims;
    key.narrow = ctx->max_bound <= 0xFFFFu;
    key.k = k;
    if (stats.known && stats.nonempty) {
        const double mean = (double)stats.walk_steps / (double)stats.nonempty;
        key.steps_class = mean >= 1.0 ? (int32_t)std::floor(std::log2(mean)) : 0;
    }
    return key;
}

static bool plan_rows(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o,
                      bool coarse, BatchedPlan *plan);

bool plan_batched(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o_in,
                  BatchedPlan *plan, bool use_tuned)
{
    wmh_opts o = o_in;
    if (use_tuned && stats.known && !o.rows_per_block && !o.hashes_per_tile &&
        !o.waves_per_block && !o.walk && !o.steps_per_lane) {
        // the plan tuned for this key, else for the same (D, width, k) at the nearest step class
        // within two (a factor of four in mean steps), e.g. the walk rows of a row split
        const TuneKey key = tune_key(ctx, k, stats);
        const TuneEntry *pick = nullptr;
        int best = 3;
        for (const TuneEntry &e : ctx->tuned) {
            if (e.key.dims != key.dims || e.key.narrow != key.narrow || e.key.k != key.k) continue;
            const int d = std::abs(e.key.steps_class - key.steps_class);
            if (d < best) {
                best = d;
                pick = &e;
            }
        }
        if (pick) {
            o.rows_per_block = pick->R;
            o.hashes_per_tile = pick->J;
            o.waves_per_block = pick->W;
            o.walk = pick->walk;
            o.steps_per_lane = pick->K;
            o.hash_groups = pick->G;
            if (!o.values) o.values = pick->V;
        }
    }
    if (o.values < 0 || o.values > 2) return false;
    // Dense rows as coarse codes: when asked for, or by default when some bound does not fit
    // 16 bits (half the LDS and stream bytes of exact 32-bit rows), if the plan takes them.
    if (o.values == 2) return plan_rows(ctx, k, stats, o, true, plan);
    if (o.values == 0 && ctx->max_bound > 0xFFFFu && o.walk != 2 &&
        plan_rows(ctx, k, stats, o, true, plan))
        return true;
    return plan_rows(ctx, k, stats, o, false, plan);
}

// The plan of plan_batched with exact or coarse dense rows.
static bool plan_rows(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o,
                      bool coarse, BatchedPlan *plan)
{
    const uint64_t min_green = stats.known ? stats.min_green : ~0ull;
    BatchedPlan p{};
    p.coarse = coarse;
    if (o.coarse_bits > kCoarseCodeBits) return false;
    p.coarse_bits = o.coarse_bits ? o.coarse_bits : kCoarseCodeBits;
    p.narrow = coarse || ctx->max_bound <= 0xFFFFu;
    p.waves_per_block = o.waves_per_block ? std::min<uint32_t>(o.waves_per_block, 16u) : 8u;
    p.hashes_per_tile = o.hashes_per_tile ? std::min(o.hashes_per_tile, k) : std::min(k, 1024u);
    const size_t elem = p.narrow ? 2 : 4;
    const size_t lds_target = 48 * 1024;  // keep several workgroups resident per CU
    if (o.walk < 0 || o.walk > 3) return false;
    uint32_t R = o.rows_per_block;
    int32_t walk = o.walk;
    if (R == 0) {
        R = 4;
        while (R > 1 && (size_t)ctx->dims * R * elem > lds_target) R >>= 1;
        if (walk == 2) R = 4;
        if (walk == 3) R = 1;
        // one row per block: the ballot walk (measured faster than one-row shared windows on
        // every workload here)
        if (walk == 0 && R == 1 && !o.steps_per_lane) walk = 3;
    }
    if (R != 1 && R != 2 && R != 4 && R != 8 && R != 16) return false;
    if (walk == 2 && R != 4) return false;
    if (walk == 3 && R != 1) return false;
    // steps per lane: R (a window of 64 steps per row), or 4 for R < 4 (windows of 256 or 128)
    const uint32_t K = o.steps_per_lane ? o.steps_per_lane : R;
    if (K != R && !(K == 4 && R < 4)) return false;
    if (walk == 2 && K != 4) return false;
    if (walk == 3 && K != 1) return false;
    p.rows_per_block = R;
    p.steps_per_lane = K;
    p.independent_rows = walk == 2;
    p.ballot = walk == 3;
    // hash groups (ballot walk): G blocks of ceil(k / G) ids, G lowered until none is empty
    if (o.hash_groups > kMaxHashGroups || (o.hash_groups > 1 && !p.ballot)) return false;
    uint32_t G = o.hash_groups ? o.hash_groups : 1;
    while (G > 1 && (uint64_t)(G - 1) * ((k + G - 1) / G) >= k) --G;
    p.hash_groups = G;
    if (G > 1) p.hashes_per_tile = (k + G - 1) / G;
    if (batched_lds_bytes(ctx->dims, p) > kMaxDynamicLds) return false;
    p.packed = p.narrow && (uint64_t)ctx->dims * p.scale() <= 65536u;
    if (coarse && (!p.packed || p.independent_rows || R > 4)) return false;
    // shared stream depth: cover eight mean step counts of the sparsest row, in whole cycles of
    // three windows (the walk's prefetch ring) that stay below the cap
    const uint32_t cycle = p.cycle();  // 3 x (64, 128 or 256) steps
    const uint32_t max_depth = 65535u / cycle * cycle;
    auto round_up = [&](double steps) {
        const double w = std::ceil(steps / cycle) * cycle;
        return (uint32_t)std::max<double>(cycle, std::min<double>(max_depth, w));
    };
    uint32_t depth;
    if (o.stream_depth == UINT32_MAX) {
        depth = p.independent_rows ? cycle : 0;  // the independent-rows walk reads the stream
    } else if (o.stream_depth) {
        depth = round_up((double)o.stream_depth);
    } else if (min_green != ~0ull && min_green != 0) {
        const double mean_steps = (double)ctx->total / (double)min_green;
        depth = round_up(std::min(65536.0, 8.0 * mean_steps + 64.0));
    } else {
        depth = 4096 / cycle * cycle;
    }
    const uint64_t entry = p.packed ? 4 : 8;
    while (depth > cycle && (uint64_t)depth * k * entry > kStreamBudgetBytes) depth -= cycle;
    // the planner's stream stays within the budget: with so many hash ids that one cycle does
    // not fit, every step is drawn in-lane (the independent-rows walk reads the stream)
    if (o.stream_depth == 0 && !p.independent_rows &&
        (uint64_t)depth * k * entry > kStreamBudgetBytes)
        depth = 0;
    p.stream_depth = depth;
    *plan = p;
    return true;
}

bool plan_index(const wmh_ctx *ctx, uint32_t k, const RowStats &stats, const wmh_opts &o,
                IndexPlan *plan)
{
    IndexPlan p;
    if (o.waves_per_block || o.index_batch || o.index_claim) {
        p.waves = o.waves_per_block;
        p.batch = o.index_batch;
        p.claim = o.index_claim;
    } else if (stats.known) {
        const TuneKey key = tune_key(ctx, k, stats);
        int best = 3;
        for (const IndexTuneEntry &e : ctx->tuned_index) {
            if (e.key.dims != key.dims || e.key.narrow != key.narrow || e.key.k != key.k) continue;
            const int d = std::abs(e.key.steps_class - key.steps_class);
            if (d < best) {
                best = d;
                p = e.plan;
            }
        }
    }
    if (index_rows_waves(k, p.waves) == 0 || (p.batch && p.batch != 8 && p.batch != 16) ||
        p.claim > 2)
        return false;
    *plan = p;
    return true;
}

// Relative costs in units of one membership test of the batched walk (measured on MI355X:
// the walk runs about 1.7e12 tests/s; the other figures are per item of the named kind).
namespace {
constexpr double kCostPlainDenseStep = 12.0;   // a step of the plain walk, dense row in LDS
constexpr double kCostPlainSparseStep = 24.0;  // a step of the plain walk, binary search in HBM
constexpr double kCostPerRowHash = 2.0;        // writing one signature value (either order)
constexpr double kCostIndexEntry = 64.0;       // building one index key (two draws, sort)
constexpr double kCostIndexNnz = 64.0;         // a nonzero's list lookup (dependent loads)
constexpr double kCostIndexKey = 20.0;         // one green key read and its LDS minimum
}  // namespace

wmh_status gather_stats(wmh_ctx *ctx, const Rows &rows, uint32_t k, hipStream_t s, bool check,
                        bool want_keys, RowStats *stats, bool want_split, CheckWords *words)
{
    if (!words) words = ctx->d_check;
    RowSplit split;
    want_split = want_split && want_keys;
    if (want_split) {
        if (ctx->row_class_cap < rows.n_rows) {
            if (ctx->d_row_class) hipFree(ctx->d_row_class);
            ctx->d_row_class = nullptr;
            ctx->row_class_cap = 0;  // a captured split walk keys on the buffer's address
            const hipError_t ae = hipMalloc(&ctx->d_row_class, std::max<uint64_t>(rows.n_rows, 1));
            if (ae != hipSuccess) return device_fail(ctx, ae, "row class buffer");
            ctx->row_class_cap = rows.n_rows;
        }
        split.row_class = ctx->d_row_class;
        split.k = k;
        split.key_cost = (float)kCostIndexKey;
        split.nnz_cost = (float)kCostIndexNnz;
    }
    hipError_t e = launch_check_init(words, s);
    if (e == hipSuccess)
        e = launch_validate(rows, ctx->d_bound, ctx->dims, ctx->total, k, want_keys, words, s,
                            want_split ? &split : nullptr, ctx->d_bound_blocks);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_check, words, sizeof(CheckWords), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(ctx, e, "validation pass");
    const CheckWords v = *ctx->h_check;
    if (check && v.first_error != ~0ull) {
        const uint64_t row = v.first_error >> 4;
        const uint32_t code = (uint32_t)(v.first_error & 15u);
        return fail(ctx, check_status(code), "row %llu: %s", (unsigned long long)row,
                    check_name(code));
    }
    stats->known = true;
    stats->nonempty = rows.n_rows - std::min<uint64_t>(rows.n_rows, v.n_empty);
    stats->min_green = v.min_green;
    stats->walk_steps = v.walk_steps;
    stats->index_keys = v.index_keys;
    stats->keys_known = want_keys;
    stats->split_known = want_split;
    if (want_split) {
        stats->walk_rows = v.walk_rows;
        stats->walk_min_green = v.walk_min_green;
        stats->walk_class_steps = v.walk_class_steps;
        stats->index_rows = v.index_rows;
        stats->index_nnz = v.index_nnz;
        stats->index_class_keys = v.index_class_keys;
    }
    return WMH_OK;
}

RowStats walk_class_stats(const RowStats &stats)
{
    RowStats w;
    w.known = stats.known;
    w.nonempty = stats.walk_rows;  // empty rows included: a bound for the mean step count
    w.min_green = stats.walk_min_green;
    w.walk_steps = stats.walk_class_steps;
    return w;
}

bool index_fits(uint32_t k)
{
    return k >= 1 && k <= kIndexMaxK && index_entry_count(k) * sizeof(uint64_t) <= kIndexBudgetBytes;
}

void free_index(OwnedIndex *ix)
{
    if (ix->buf.entries) (void)hipFree(ix->buf.entries);
    if (ix->buf.by_step) (void)hipFree(ix->buf.by_step);
    if (ix->buf.offsets) (void)hipFree(ix->buf.offsets);
    if (ix->buf.cursor) (void)hipFree(ix->buf.cursor);
    if (ix->buf.block_sums) (void)hipFree(ix->buf.block_sums);
    if (ix->used) (void)hipEventDestroy(ix->used);
    *ix = OwnedIndex{};
}

wmh_status ensure_index(wmh_ctx *ctx, OwnedIndex *ix, uint64_t seed, uint32_t k,
                        hipStream_t stream, bool record_error)
{
    if (ix->valid && ix->seed == seed && ix->k == k && ix->epoch == ctx->bounds_epoch)
        return WMH_OK;
    wmh_ctx *err = record_error ? ctx : nullptr;
    if (!index_fits(k))
        return fail(err, WMH_E_ARG, "the component index needs k <= %u", kIndexMaxK);
    ix->valid = false;
    hipError_t e = hipSuccess;
    if (!ix->used) e = hipEventCreateWithFlags(&ix->used, hipEventDisableTiming);
    else e = hipStreamWaitEvent(stream, ix->used, 0);  // earlier readers, on any stream
    if (e != hipSuccess) return device_fail(err, e, "index event");
    // lists start on 128-byte lines when the padding fits the budget
    const uint32_t align =
        index_padded_count(k, ctx->dims, kIndexListAlign) * sizeof(uint64_t) <= kIndexBudgetBytes
            ? kIndexListAlign
            : 1u;
    const uint64_t n = index_padded_count(k, ctx->dims, align);
    if (n > ix->cap_entries) {
        for (uint64_t **p : {&ix->buf.entries, &ix->buf.by_step}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        ix->cap_entries = 0;
        const size_t bytes = (n + kIndexPadKeys) * sizeof(uint64_t);
        e = hipMalloc(&ix->buf.entries, bytes);
        if (e == hipSuccess) e = hipMalloc(&ix->buf.by_step, bytes);
        if (e != hipSuccess) return device_fail(err, e, "index entries");
        ix->cap_entries = n;
    }
    if (ctx->dims > ix->cap_dims || !ix->buf.offsets) {
        for (uint32_t **p : {&ix->buf.offsets, &ix->buf.cursor, &ix->buf.block_sums}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        ix->cap_dims = 0;
        const size_t words = (size_t)ctx->dims + 1;
        e = hipMalloc(&ix->buf.offsets, words * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&ix->buf.cursor, words * sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMalloc(&ix->buf.block_sums, index_scan_blocks(ctx->dims) * sizeof(uint32_t));
        if (e != hipSuccess) return device_fail(err, e, "index offsets");
        ix->cap_dims = ctx->dims;
    }
    ix->buf.align = align;
    e = launch_index_build(bounds_view(ctx), seed, k, ix->buf, stream);
    if (e != hipSuccess) return device_fail(err, e, "index build");
    ix->valid = true;
    ix->seed = seed;
    ix->k = k;
    ix->epoch = ctx->bounds_epoch;
    return WMH_OK;
}

Path choose_path(const wmh_ctx *ctx, int mode, bool batched_ok, bool index_ready, uint32_t k,
                 uint64_t n_rows, uint64_t nnz, const RowStats &stats, bool split_ok)
{
    if (mode == WMH_MODE_PLAIN) return Path::kPlain;
    if (mode == WMH_MODE_BATCHED) return Path::kBatched;
    if (mode == WMH_MODE_INDEXED) return Path::kIndexed;
    if (mode == WMH_MODE_SPLIT) return Path::kSplit;
    if (mode == WMH_MODE_PLAIN_SHARED) return Path::kPlainShared;
    const Path walk_path = batched_ok ? Path::kBatched : Path::kPlain;
    if (!stats.known || !stats.keys_known || !index_fits(k)) return walk_path;
    const bool narrow = ctx->max_bound <= 0xFFFFu;
    const bool dense = (size_t)4 * ctx->dims * (narrow ? 2 : 4) <= 64 * 1024;
    const double step = batched_ok ? 1.0 : (dense ? kCostPlainDenseStep : kCostPlainSparseStep);
    const double walk = (double)k * ((double)stats.walk_steps * step + kCostPerRowHash * n_rows);
    const double build = index_ready ? 0.0 : (double)index_entry_count(k) * kCostIndexEntry;
    const double index = build + (double)nnz * kCostIndexNnz +
                         (double)k * ((double)stats.index_keys * kCostIndexKey +
                                      kCostPerRowHash * n_rows);
    const Path best = index < walk ? Path::kIndexed : walk_path;
    if (!split_ok || !stats.split_known || stats.walk_rows == 0 || stats.index_rows == 0)
        return best;
    // each row on its cheaper path: the batched walk for one class, the index for the other
    const double split =
        (double)k * ((double)stats.walk_class_steps + kCostPerRowHash * stats.walk_rows) + build +
        (double)stats.index_nnz * kCostIndexNnz +
        (double)k * ((double)stats.index_class_keys * kCostIndexKey +
                     kCostPerRowHash * stats.index_rows);
    return split < std::min(walk, index) ? Path::kSplit : best;
}

}  // namespace wmh

namespace {

#define WMH_HIP(ctx, call)                                      \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return device_fail(ctx, e_, #call); \
    } while (0)

void release_bounds(wmh_ctx *ctx)
{
    if (ctx->d_prefix) hipFree(ctx->d_prefix);
    if (ctx->d_bucket) hipFree(ctx->d_bucket);
    if (ctx->d_bound) hipFree(ctx->d_bound);
    if (ctx->d_bound_blocks) hipFree(ctx->d_bound_blocks);
    ctx->d_prefix = nullptr;
    ctx->d_bucket = nullptr;
    ctx->d_bound = nullptr;
    ctx->d_bound_blocks = nullptr;
    ctx->has_bounds = false;
}

void drop_graph(wmh_ctx *ctx)
{
    if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    ctx->graph_key = GraphKey{};
}

hipStream_t pick_stream(wmh_ctx *ctx, void *stream)
{
    return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
}

wmh_status ensure_stream_capacity(wmh_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->stream_bytes) return WMH_OK;
    if (ctx->d_stream) hipFree(ctx->d_stream);
    ctx->d_stream = nullptr;
    ctx->stream_bytes = 0;
    ctx->stream_valid = false;
    drop_graph(ctx);
    WMH_HIP(ctx, hipMalloc(&ctx->d_stream, bytes));
    ctx->stream_bytes = bytes;
    return WMH_OK;
}

}  // namespace

extern "C" {

void wmh_opts_init(wmh_opts *opts)
{
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->mode = WMH_MODE_AUTO;
    opts->batch_rows = 8192;
    opts->validate = 1;
    opts->use_graph = 1;
    opts->sync = 1;
}

const char *wmh_status_string(wmh_status status)
{
    switch (status) {
    case WMH_OK: return "WMH_OK";
    case WMH_E_ARG: return "WMH_E_ARG";
    case WMH_E_NO_BOUNDS: return "WMH_E_NO_BOUNDS";
    case WMH_E_COL_RANGE: return "WMH_E_COL_RANGE";
    case WMH_E_UNSORTED: return "WMH_E_UNSORTED";
    case WMH_E_BOUND: return "WMH_E_BOUND";
    case WMH_E_OVERFLOW: return "WMH_E_OVERFLOW";
    case WMH_E_NOMEM: return "WMH_E_NOMEM";
    case WMH_E_DEVICE: return "WMH_E_DEVICE";
    case WMH_E_ROW_PTR: return "WMH_E_ROW_PTR";
    }
    return "WMH_E_UNKNOWN";
}

const char *wmh_last_error(const wmh_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

wmh_status wmh_create(int device, wmh_ctx **out)
{
    if (!out) return WMH_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return WMH_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return WMH_E_DEVICE;
    wmh_ctx *ctx = new (std::nothrow) wmh_ctx();
    if (!ctx) return WMH_E_NOMEM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&ctx->d_check, sizeof(CheckWords)) != hipSuccess ||
        hipHostMalloc(&ctx->h_check, sizeof(CheckWords), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&ctx->d_tile_counter, kMaxHashGroups * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx->d_row_counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx->d_codec, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(&ctx->h_codec, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&ctx->ev[0]) != hipSuccess || hipEventCreate(&ctx->ev[1]) != hipSuccess ||
        hipEventCreate(&ctx->ev[2]) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->stream_ready, hipEventDisableTiming) != hipSuccess) {
        wmh_destroy(ctx);
        return WMH_E_DEVICE;
    }
    ctx->cu_count = prop.multiProcessorCount;
    // the address of the no-allocation entry point's static scratch on this device; a failure
    // here is reported by that entry point, not by the context
    (void)static_scratch_init(device);
    *out = ctx;
    return WMH_OK;
}

void wmh_destroy(wmh_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    drop_graph(ctx);
    release_bounds(ctx);
    free_index(&ctx->index);
    if (ctx->d_stream) hipFree(ctx->d_stream);
    if (ctx->d_check) hipFree(ctx->d_check);
    if (ctx->d_row_class) hipFree(ctx->d_row_class);
    if (ctx->h_check) hipHostFree(ctx->h_check);
    if (ctx->d_tile_counter) hipFree(ctx->d_tile_counter);
    if (ctx->d_row_counter) hipFree(ctx->d_row_counter);
    if (ctx->d_codec) hipFree(ctx->d_codec);
    if (ctx->h_codec) hipHostFree(ctx->h_codec);
    for (hipEvent_t &e : ctx->ev)
        if (e) hipEventDestroy(e);
    if (ctx->stream_ready) hipEventDestroy(ctx->stream_ready);
    if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
    if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

wmh_status wmh_bounds_tables(const uint32_t *m, uint32_t D, uint64_t *prefix, uint32_t *bucket,
                             uint32_t *shift_out, uint64_t *n_buckets_out, uint64_t *threshold_out)
{
    if (!m || D == 0 || D > kMaxDims) return WMH_E_ARG;
    uint64_t total = 0;
    for (uint32_t i = 0; i < D; ++i) total += m[i];
    if (total == 0) return WMH_E_OVERFLOW;
    // about two buckets per dimension: at most 2 * 2^ceil(log2 D), at least 4
    uint64_t target = 2;
    while (target < (uint64_t)D) target <<= 1;
    target <<= 1;
    uint32_t shift = 0;
    while ((((total - 1) >> shift) + 1) > target) ++shift;
    const uint64_t n_buckets = ((total - 1) >> shift) + 1;
    if (shift_out) *shift_out = shift;
    if (n_buckets_out) *n_buckets_out = n_buckets;
    if (threshold_out) *threshold_out = (0ull - total) % total;  // 2^64 mod M
    if (prefix) {
        prefix[0] = 0;
        for (uint32_t i = 0; i < D; ++i) prefix[i + 1] = prefix[i] + m[i];
    }
    if (bucket) {
        // two pointers over the prefix sums, computed again here so `prefix` may be NULL
        uint64_t start_next = m[0];  // P[c + 1]
        uint32_t c = 0;
        for (uint64_t bkt = 0; bkt <= n_buckets; ++bkt) {
            const uint64_t q = bkt << shift;
            while (c + 1 < D && start_next <= q) {
                ++c;
                start_next += m[c];
            }
            bucket[bkt] = c;
        }
    }
    return WMH_OK;
}

wmh_status wmh_set_bounds(wmh_ctx *ctx, const uint32_t *m, uint32_t D)
{
    if (!ctx) return WMH_E_ARG;
    if (!m || D == 0 || D > kMaxDims) return fail(ctx, WMH_E_ARG, "D must be in [1, 2^26]");
    if (ctx->servers > 0)
        return fail(ctx, WMH_E_ARG, "a serving loop is using this context's bounds");
    if (ctx->has_bounds && ctx->dims == D &&
        std::memcmp(ctx->h_bound.data(), m, (size_t)D * sizeof(uint32_t)) == 0) {
        ctx->last_error.clear();  // the same bounds: tables, graph and index stay valid
        return WMH_OK;
    }
    WMH_HIP(ctx, hipSetDevice(ctx->device));
    uint32_t shift = 0;
    uint64_t n_buckets = 0, threshold = 0;
    wmh_status st = wmh_bounds_tables(m, D, nullptr, nullptr, &shift, &n_buckets, &threshold);
    if (st == WMH_E_OVERFLOW) return fail(ctx, st, "the bounds sum to 0");
    if (st != WMH_OK) return fail(ctx, st, "invalid bounds");
    std::vector<uint64_t> prefix((size_t)D + 1);
    std::vector<uint32_t> bucket(n_buckets + 1);
    wmh_bounds_tables(m, D, prefix.data(), bucket.data(), nullptr, nullptr, nullptr);
    const uint64_t total = prefix[D];
    uint32_t max_bound = 0;
    for (uint32_t i = 0; i < D; ++i) max_bound = std::max(max_bound, m[i]);

    drop_graph(ctx);
    release_bounds(ctx);
    WMH_HIP(ctx, hipMalloc(&ctx->d_prefix, prefix.size() * sizeof(uint64_t)));
    WMH_HIP(ctx, hipMalloc(&ctx->d_bucket, bucket.size() * sizeof(uint32_t)));
    WMH_HIP(ctx, hipMalloc(&ctx->d_bound, (size_t)D * sizeof(uint32_t)));
    WMH_HIP(ctx, hipMemcpy(ctx->d_prefix, prefix.data(), prefix.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice));
    WMH_HIP(ctx, hipMemcpy(ctx->d_bucket, bucket.data(), bucket.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice));
    WMH_HIP(ctx, hipMemcpy(ctx->d_bound, m, (size_t)D * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (bound_blocks_wanted(D)) {
        // per block of kBoundBlock components: the smallest bound, then the rounded mean
        const uint32_t nb = (D + kBoundBlock - 1) / kBoundBlock;
        std::vector<uint32_t> blocks(2 * (size_t)nb);
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t lo = b * kBoundBlock, hi = std::min(D, lo + kBoundBlock);
            uint32_t mn = m[lo];
            uint64_t sum = 0;
            for (uint32_t i = lo; i < hi; ++i) {
                mn = std::min(mn, m[i]);
                sum += m[i];
            }
            blocks[b] = mn;
            blocks[nb + b] = (uint32_t)((sum + (hi - lo) / 2) / (hi - lo));
        }
        WMH_HIP(ctx, hipMalloc(&ctx->d_bound_blocks, blocks.size() * sizeof(uint32_t)));
        WMH_HIP(ctx, hipMemcpy(ctx->d_bound_blocks, blocks.data(), blocks.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice));
    }
    ctx->dims = D;
    ctx->total = total;
    ctx->threshold = threshold;
    ctx->shift = shift;
    ctx->n_buckets = n_buckets;
    ctx->max_bound = max_bound;
    ctx->h_bound.assign(m, m + D);
    ctx->has_bounds = true;
    ctx->bounds_epoch++;
    ctx->last_error.clear();
    return WMH_OK;
}

wmh_status wmh_bounds_info(const wmh_ctx *ctx, uint32_t *D, uint64_t *M, uint32_t *shift,
                           uint64_t *n_buckets)
{
    if (!ctx) return WMH_E_ARG;
    if (!ctx->has_bounds) return WMH_E_NO_BOUNDS;
    if (D) *D = ctx->dims;
    if (M) *M = ctx->total;
    if (shift) *shift = ctx->shift;
    if (n_buckets) *n_buckets = ctx->n_buckets;
    return WMH_OK;
}

wmh_status wmh_hash(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                    const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k,
                    uint64_t seed, uint16_t *sig, void *stream, const wmh_opts *opts)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (!ctx->has_bounds) return fail(ctx, WMH_E_NO_BOUNDS, "wmh_set_bounds was not called");
    if (k == 0 || k > kMaxK) return fail(ctx, WMH_E_ARG, "k must be in [1, 2^24]");
    if (n_rows == 0) return WMH_OK;
    if (!row_ptr || !sig || (nnz && (!col || !val)))
        return fail(ctx, WMH_E_ARG, "null buffer");
    if (n_rows > (1ull << 40) || nnz > (1ull << 40))
        return fail(ctx, WMH_E_ARG, "sizes out of range");
    wmh_opts o;
    if (opts) o = *opts;
    else wmh_opts_init(&o);
    if (o.mode < WMH_MODE_AUTO || o.mode > WMH_MODE_PLAIN_SHARED)
        return fail(ctx, WMH_E_ARG, "unknown mode %d", o.mode);
    if ((o.mode == WMH_MODE_INDEXED || o.mode == WMH_MODE_SPLIT) && !index_fits(k))
        return fail(ctx, WMH_E_ARG, "the component index needs k <= %u", kIndexMaxK);
    WMH_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    const Rows rows{row_ptr, col, val, n_rows, nnz};
    const Bounds b = bounds_view(ctx);

    RowStats stats;
    const bool profile = o.profile != 0;
    ctx->profiled = false;
    const bool split_mode = o.mode == WMH_MODE_SPLIT;
    if (o.validate || o.mode == WMH_MODE_AUTO || split_mode) {
        const bool want_keys = (o.mode == WMH_MODE_AUTO || split_mode) && index_fits(k);
        // the row classes of a split (not with the independent-rows walk, which has no filter)
        const bool want_split = want_keys && o.walk != 2;
        const wmh_status st =
            gather_stats(ctx, rows, k, s, o.validate != 0, want_keys, &stats, want_split);
        if (st != WMH_OK) return st;
    }

    BatchedPlan plan{};
    const bool batched_ok = (o.mode == WMH_MODE_AUTO || o.mode == WMH_MODE_BATCHED ||
                             o.mode == WMH_MODE_PLAIN_SHARED) &&
                            plan_batched(ctx, k, stats, o, &plan);
    if ((o.mode == WMH_MODE_BATCHED || o.mode == WMH_MODE_PLAIN_SHARED) && !batched_ok)
        return fail(ctx, WMH_E_ARG, "no batched plan fits for D=%u with these options", ctx->dims);
    // a split walks one class with a plan sized for that class alone
    BatchedPlan split_plan{};
    const bool split_ok = stats.split_known && stats.walk_rows && stats.index_rows &&
                          plan_batched(ctx, k, walk_class_stats(stats), o, &split_plan) &&
                          !split_plan.independent_rows;
    const bool index_ready = ctx->index.valid && ctx->index.seed == seed && ctx->index.k == k &&
                             ctx->index.epoch == ctx->bounds_epoch;
    Path path = choose_path(ctx, o.mode, batched_ok, index_ready, k, n_rows, nnz, stats, split_ok);
    if (path == Path::kSplit && !split_ok) {
        // a forced split whose rows all fall on one side runs that side alone
        if (stats.index_rows == 0 && plan_batched(ctx, k, stats, o, &plan) && !plan.independent_rows)
            path = Path::kBatched;
        else if (stats.walk_rows == 0)
            path = Path::kIndexed;
        else
            return fail(ctx, WMH_E_ARG, "no batched plan fits for the walk rows of a split");
    }

    if (path == Path::kIndexed) {
        IndexPlan ip;
        if (!plan_index(ctx, k, stats, o, &ip))
            return fail(ctx, WMH_E_ARG, "index rows plan does not fit (waves %u, batch %u, "
                        "claim %u, k %u)", o.waves_per_block, o.index_batch, o.index_claim, k);
        if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[0], s));
        const wmh_status st = ensure_index(ctx, &ctx->index, seed, k, s);
        if (st != WMH_OK) return st;
        const uint32_t grid =
            (uint32_t)ctx->cu_count * (uint32_t)index_rows_blocks_per_cu(k, ip.waves);
        if (o.use_graph) {
            // the steady state (counter reset and rows kernel) replayed as a graph
            GraphKey key;
            key.row_ptr = row_ptr; key.col = col; key.val = val; key.sig = sig;
            key.n_rows = n_rows; key.nnz = nnz; key.seed = seed; key.k = k;
            key.waves = ip.waves; key.grid = grid; key.bounds_epoch = ctx->bounds_epoch;
            key.indexed = true;
            key.index_keys = ctx->index.buf.entries;
            key.index_steps = ctx->index.buf.by_step;
            key.index_offsets = ctx->index.buf.offsets;
            key.ix_batch = ip.batch;
            key.ix_claim = ip.claim;
            if (!(ctx->graph_exec && ctx->graph_key == key)) {
                drop_graph(ctx);
                hipGraph_t graph = nullptr;
                WMH_HIP(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = launch_index_rows(rows, ctx->index.buf, b, k, sig,
                                                 ctx->d_row_counter, grid, ctx->capture_stream, ip);
                hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &graph);
                if (e != hipSuccess) {
                    if (graph) hipGraphDestroy(graph);
                    return device_fail(ctx, e, "index rows launch (capture)");
                }
                if (e2 != hipSuccess) return device_fail(ctx, e2, "hipStreamEndCapture");
                e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    ctx->graph_exec = nullptr;
                    return device_fail(ctx, e, "hipGraphInstantiate");
                }
                ctx->graph_key = key;
            }
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[1], s));
            WMH_HIP(ctx, hipGraphLaunch(ctx->graph_exec, s));
        } else {
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[1], s));
            WMH_HIP(ctx, launch_index_rows(rows, ctx->index.buf, b, k, sig, ctx->d_row_counter,
                                           grid, s, ip));
        }
        if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[2], s));
        ctx->last_index_plan = ip;
        WMH_HIP(ctx, hipEventRecord(ctx->index.used, s));
        ctx->profiled = profile;
        ctx->profiled_stream = profile && !index_ready;
        ctx->last_mode = WMH_MODE_INDEXED;
        if (o.sync) WMH_HIP(ctx, hipStreamSynchronize(s));
        return WMH_OK;
    }

    if (path == Path::kPlain) {
        const bool narrow = ctx->max_bound <= 0xFFFFu;
        const bool dense = (size_t)4 * ctx->dims * (narrow ? 2 : 4) <= 64 * 1024;
        const uint64_t step = o.batch_rows ? o.batch_rows : 8192;
        if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[1], s));
        for (uint64_t r0 = 0; r0 < n_rows; r0 += step) {
            const uint64_t r1 = std::min(n_rows, r0 + step);
            WMH_HIP(ctx, launch_plain(b, rows, r0, r1, k, seed, sig, narrow, dense, s));
        }
        if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[2], s));
        ctx->profiled = profile;
        ctx->profiled_stream = false;
        ctx->last_mode = WMH_MODE_PLAIN;
        ctx->last_plan = BatchedPlan{};
        if (o.sync) WMH_HIP(ctx, hipStreamSynchronize(s));
        return WMH_OK;
    }

    // The batched walk of `wrows` (every row, or the walk class of a split) under plan `pl`:
    // one persistent launch (graph-captured with use_graph), or with `per_batch` one launch
    // per batch of batch_rows rows, a workgroup per tile and no tile counter.
    auto run_batched = [&](const Rows &wrows, const BatchedPlan &pl,
                           bool per_batch = false) -> wmh_status {
        {
            wmh_status st = ensure_stream_capacity(ctx, pl.stream_bytes(k));
            if (st != WMH_OK) return st;
        }
        const int per_cu = std::max(1, batched_blocks_per_cu(ctx->dims, pl));
        const uint64_t n_blocks = (n_rows + pl.rows_per_block - 1) / pl.rows_per_block;
        const uint64_t n_tiles =
            n_blocks * ((k + pl.hashes_per_tile - 1) / pl.hashes_per_tile);
        const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)ctx->cu_count * per_cu, n_tiles);

        GraphKey key;
        key.row_ptr = row_ptr; key.col = col; key.val = val; key.sig = sig;
        key.n_rows = n_rows; key.nnz = nnz; key.seed = seed; key.k = k;
        key.R = pl.rows_per_block; key.J = pl.hashes_per_tile; key.depth = pl.stream_depth;
        key.K = pl.steps_per_lane;
        key.waves = pl.waves_per_block; key.grid = grid; key.narrow = pl.narrow;
        key.packed = pl.packed;
        key.coarse_bits = pl.coarse ? pl.coarse_bits : 0u;
        key.independent_rows = pl.independent_rows;
        key.ballot = pl.ballot;
        key.groups = pl.hash_groups;
        key.row_class = wrows.row_class;
        key.keep = wrows.keep;
        key.bounds_epoch = ctx->bounds_epoch;

        // The shared position stream (cached position stream): built once per (seed, k,
        // depth, entry layout, bounds) and kept for later calls, which wait for its build.
        bool stream_built = false;
        if (pl.stream_depth) {
            const StreamKey skey{seed, k, pl.stream_depth, pl.scale(), pl.packed,
                                 ctx->bounds_epoch, pl.coarse ? pl.coarse_bits : 0u};
            if (!(ctx->stream_valid && ctx->stream_key == skey)) {
                ctx->stream_valid = false;
                if (profile && !o.use_graph) WMH_HIP(ctx, hipEventRecord(ctx->ev[0], s));
                WMH_HIP(ctx, launch_stream_build(b, seed, k, pl.stream_depth, pl.packed,
                                                 pl.scale(), pl.coarse ? pl.coarse_bits : 0u,
                                                 ctx->d_stream, s));
                WMH_HIP(ctx, hipEventRecord(ctx->stream_ready, s));
                ctx->stream_key = skey;
                ctx->stream_valid = true;
                stream_built = true;
            } else {
                WMH_HIP(ctx, hipStreamWaitEvent(s, ctx->stream_ready, 0));
            }
        }

        if (per_batch) {
            // the same kernels and plan, scheduled plainly: one launch per batch of rows, one
            // workgroup per (row block, hash block) tile, no counter and no graph
            const uint64_t step = o.batch_rows ? o.batch_rows : 8192;
            const uint64_t hash_tiles = (k + pl.hashes_per_tile - 1) / pl.hashes_per_tile;
            BatchedPlan one = pl;  // static tiles: (row block, hash block) over one index
            one.hash_groups = 1;
            if (((step + pl.rows_per_block - 1) / pl.rows_per_block) * hash_tiles > UINT32_MAX)
                return fail(ctx, WMH_E_ARG, "a batch of %llu rows has too many tiles for one launch",
                            (unsigned long long)step);
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[1], s));
            for (uint64_t r0 = 0; r0 < n_rows; r0 += step) {
                Rows batch = wrows;
                batch.row_ptr = wrows.row_ptr + r0;
                batch.n_rows = std::min(n_rows, r0 + step) - r0;
                const uint64_t tiles =
                    (batch.n_rows + pl.rows_per_block - 1) / pl.rows_per_block * hash_tiles;
                WMH_HIP(ctx, launch_batched(b, batch, k, seed, sig + r0 * k, one, ctx->d_stream,
                                            nullptr, (uint32_t)tiles, s));
            }
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[2], s));
            ctx->profiled_stream = profile && stream_built;
            return WMH_OK;
        }

        // events around the walk only on direct launches; a graph is timed as a whole
        auto enqueue = [&](hipStream_t q, bool events) -> hipError_t {
            hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->d_tile_counter), 0u,
                                           2 * kMaxHashGroups, q);
            if (e != hipSuccess) return e;
            if (events && (e = hipEventRecord(ctx->ev[1], q)) != hipSuccess) return e;
            e = launch_batched(b, wrows, k, seed, sig, pl, ctx->d_stream, ctx->d_tile_counter,
                               grid, q);
            if (e != hipSuccess) return e;
            if (events) e = hipEventRecord(ctx->ev[2], q);
            return e;
        };

        if (o.use_graph) {
            if (!(ctx->graph_exec && ctx->graph_key == key)) {
                drop_graph(ctx);
                hipGraph_t graph = nullptr;
                WMH_HIP(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
                hipError_t e = enqueue(ctx->capture_stream, false);
                hipError_t e2 = hipStreamEndCapture(ctx->capture_stream, &graph);
                if (e != hipSuccess) {
                    if (graph) hipGraphDestroy(graph);
                    return device_fail(ctx, e, "batched launch (capture)");
                }
                if (e2 != hipSuccess) return device_fail(ctx, e2, "hipStreamEndCapture");
                e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    ctx->graph_exec = nullptr;
                    return device_fail(ctx, e, "hipGraphInstantiate");
                }
                ctx->graph_key = key;
            }
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[1], s));
            WMH_HIP(ctx, hipGraphLaunch(ctx->graph_exec, s));
            if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[2], s));
            ctx->profiled_stream = false;
        } else {
            hipError_t e = enqueue(s, profile);
            if (e != hipSuccess) return device_fail(ctx, e, "batched launch");
            ctx->profiled_stream = profile && stream_built;
        }
        return WMH_OK;
    };

    if (path == Path::kSplit) {
        // the index first (built once per bounds, seed and k), then the walk rows, then the
        // index rows; each kernel leaves the other class's signatures untouched
        {
            const wmh_status st = ensure_index(ctx, &ctx->index, seed, k, s);
            if (st != WMH_OK) return st;
        }
        Rows walk_rows = rows, index_rows = rows;
        walk_rows.row_class = index_rows.row_class = ctx->d_row_class;
        walk_rows.keep = 0;
        index_rows.keep = 1;
        const wmh_status st = run_batched(walk_rows, split_plan);
        if (st != WMH_OK) return st;
        const uint32_t grid = (uint32_t)ctx->cu_count * (uint32_t)index_rows_blocks_per_cu(k);
        WMH_HIP(ctx, launch_index_rows(index_rows, ctx->index.buf, b, k, sig, ctx->d_row_counter, grid, s));
        if (profile) WMH_HIP(ctx, hipEventRecord(ctx->ev[2], s));  // walk_ms spans both
        WMH_HIP(ctx, hipEventRecord(ctx->index.used, s));
        ctx->profiled = profile;
        ctx->last_mode = WMH_MODE_SPLIT;
        ctx->last_plan = split_plan;
        if (o.sync) WMH_HIP(ctx, hipStreamSynchronize(s));
        return WMH_OK;
    }

    const bool per_batch = path == Path::kPlainShared;
    const wmh_status st = run_batched(rows, plan, per_batch);
    if (st != WMH_OK) return st;
    ctx->profiled = profile;
    ctx->last_mode = per_batch ? WMH_MODE_PLAIN_SHARED : WMH_MODE_BATCHED;
    ctx->last_plan = plan;
    if (o.sync) WMH_HIP(ctx, hipStreamSynchronize(s));
    return WMH_OK;
}

wmh_status wmh_last_mode(const wmh_ctx *ctx, int32_t *mode)
{
    if (!ctx || !mode) return WMH_E_ARG;
    *mode = ctx->last_mode;
    return WMH_OK;
}

wmh_status wmh_last_plan(const wmh_ctx *ctx, wmh_opts *plan)
{
    if (!ctx || !plan) return WMH_E_ARG;
    wmh_opts_init(plan);
    plan->mode = ctx->last_mode;
    plan->rows_per_block = ctx->last_plan.rows_per_block;
    plan->hashes_per_tile = ctx->last_plan.hashes_per_tile;
    plan->stream_depth = ctx->last_plan.stream_depth;
    plan->steps_per_lane = ctx->last_plan.steps_per_lane;
    plan->waves_per_block = ctx->last_plan.waves_per_block;
    plan->hash_groups = ctx->last_plan.hash_groups;
    plan->values = ctx->last_plan.rows_per_block ? (ctx->last_plan.coarse ? 2 : 1) : 0;
    plan->coarse_bits = ctx->last_plan.coarse ? ctx->last_plan.coarse_bits : 0;
    if (ctx->last_mode == WMH_MODE_INDEXED) {
        plan->rows_per_block = plan->hashes_per_tile = plan->stream_depth = 0;
        plan->steps_per_lane = 0;
        plan->hash_groups = 0;
        plan->values = 0;
        plan->coarse_bits = 0;
        plan->waves_per_block = ctx->last_index_plan.waves;
        plan->index_batch = ctx->last_index_plan.batch;
        plan->index_claim = ctx->last_index_plan.claim;
        plan->walk = 0;
        return WMH_OK;
    }
    plan->walk = ctx->last_mode != WMH_MODE_BATCHED && ctx->last_mode != WMH_MODE_SPLIT &&
                         ctx->last_mode != WMH_MODE_PLAIN_SHARED
                     ? 0
                 : ctx->last_plan.ballot           ? 3
                 : ctx->last_plan.independent_rows ? 2
                                                   : 1;
    return WMH_OK;
}

wmh_status wmh_last_kernel_ms(wmh_ctx *ctx, float *walk_ms, float *stream_ms)
{
    if (!ctx) return WMH_E_ARG;
    if (!ctx->profiled) return fail(ctx, WMH_E_ARG, "no profiled wmh_hash call");
    WMH_HIP(ctx, hipEventSynchronize(ctx->ev[2]));
    float w = 0.f, st = 0.f;
    WMH_HIP(ctx, hipEventElapsedTime(&w, ctx->ev[1], ctx->ev[2]));
    if (ctx->profiled_stream) WMH_HIP(ctx, hipEventElapsedTime(&st, ctx->ev[0], ctx->ev[1]));
    if (walk_ms) *walk_ms = w;
    if (stream_ms) *stream_ms = st;
    return WMH_OK;
}

wmh_status wmh_draws(wmh_ctx *ctx, uint64_t seed, uint32_t j0, uint32_t n_hashes, uint32_t depth,
                     uint64_t *pos, uint32_t *comp, uint64_t *off, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (!ctx->has_bounds) return fail(ctx, WMH_E_NO_BOUNDS, "wmh_set_bounds was not called");
    if (depth == 0 || depth > 65536u || n_hashes == 0 || (uint64_t)j0 + n_hashes > (1ull << 32))
        return fail(ctx, WMH_E_ARG, "depth must be in [1, 65536], n_hashes >= 1");
    if ((uint64_t)n_hashes * depth > (1ull << 34)) return fail(ctx, WMH_E_ARG, "too many draws");
    WMH_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    WMH_HIP(ctx, launch_draws(bounds_view(ctx), seed, j0, n_hashes, depth, pos, comp, off, s));
    WMH_HIP(ctx, hipStreamSynchronize(s));
    return WMH_OK;
}

wmh_status wmh_estimate(wmh_ctx *ctx, const uint16_t *A, const uint16_t *B, uint64_t n_pairs,
                        uint32_t k, uint32_t *count, double *jhat, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (k == 0) return fail(ctx, WMH_E_ARG, "k must be >= 1");
    if (n_pairs == 0) return WMH_OK;
    if (!A || !B || (!count && !jhat)) return fail(ctx, WMH_E_ARG, "null buffer");
    WMH_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    WMH_HIP(ctx, launch_estimate(A, B, n_pairs, k, count, jhat, s));
    WMH_HIP(ctx, hipStreamSynchronize(s));
    return WMH_OK;
}

wmh_status wmh_estimate_pair(const uint16_t *a, const uint16_t *b, uint32_t k, uint32_t *count,
                             double *jhat)
{
    if (!a || !b || k == 0 || (!count && !jhat)) return WMH_E_ARG;
    uint32_t equal = 0;
    for (uint32_t j = 0; j < k; ++j) equal += a[j] == b[j];
    if (count) *count = equal;
    if (jhat) *jhat = (double)equal / (double)k;
    return WMH_OK;
}

wmh_status wmh_collisions(wmh_ctx *ctx, const uint16_t *A, uint64_t NA, const uint16_t *B,
                          uint64_t NB, uint32_t k, uint32_t *counts, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (k == 0) return fail(ctx, WMH_E_ARG, "k must be >= 1");
    if (NA == 0 || NB == 0) return WMH_OK;
    if (!A || !B || !counts) return fail(ctx, WMH_E_ARG, "null buffer");
    if (NA > 65535ull * 64) return fail(ctx, WMH_E_ARG, "NA too large for one call (max 4194240)");
    WMH_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = pick_stream(ctx, stream);
    WMH_HIP(ctx, launch_collisions(A, NA, B, NB, k, counts, s));
    WMH_HIP(ctx, hipStreamSynchronize(s));
    return WMH_OK;
}

}  // extern "C"
