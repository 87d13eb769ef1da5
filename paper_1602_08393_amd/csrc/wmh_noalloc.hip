// wmh_hash_noalloc: the batched walk of wmh_hash for callers that cannot allocate device memory
// during a call (code under graph capture, tight serving loops, harnesses that forbid it).
//
// Every scratch buffer the walk needs -- the tile counter, the validation pass's words and the
// shared position stream -- lives in one static device array, `scratch`, of
// WMH_NOALLOC_SCRATCH_BYTES.  Each device holds its own copy until the process ends.  In host
// code the array's name only stands for the device symbol, so its device address is looked up
// once per device, with that device current, when a context is created on it (wmh_create calls
// static_scratch_init); the kernels receive that address, never the name.
//
// Every call on one device shares the array and finds the previous call's contents: the tile
// counter is cleared by a fill kernel, the validation words are initialised by their own kernel
// and the stream is rebuilt on every call.  Calls that overlap on one device race on the array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

namespace wmh {

namespace {

constexpr size_t kScratchBytes = (size_t)WMH_NOALLOC_SCRATCH_BYTES;
// byte offsets of the three buffers inside the array
constexpr size_t kTileCounterAt = 0;
constexpr size_t kCheckWordsAt = 256;
constexpr size_t kStreamAt = 512;
static_assert(sizeof(CheckWords) <= kStreamAt - kCheckWordsAt, "validation words overlap");
static_assert(kMaxHashGroups * sizeof(unsigned long long) <= kCheckWordsAt - kTileCounterAt,
              "tile counters overlap");

constexpr int kMaxDevices = 64;
std::mutex g_lookup;
bool g_looked_up[kMaxDevices];
hipError_t g_status[kMaxDevices];
unsigned char *g_address[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_lookup);
    if (!g_looked_up[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_status[device] = e;
        g_address[device] = e == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
        g_looked_up[device] = true;
    }
    return g_status[device];
}

namespace {

// Device address of the array on `device` (looked up by static_scratch_init), or nullptr.
unsigned char *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_lookup);
    return g_looked_up[device] ? g_address[device] : nullptr;
}

}  // namespace

}  // namespace wmh

using namespace wmh;

#define WMH_NA_HIP(ctx, call)                                     \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return device_fail(ctx, e_, #call); \
    } while (0)

extern "C" wmh_status wmh_hash_noalloc(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                                       const uint32_t *val, uint64_t n_rows, uint64_t nnz,
                                       uint32_t k, uint64_t seed, uint16_t *sig, void *stream,
                                       const wmh_opts *opts)
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
    if (o.mode != WMH_MODE_AUTO && o.mode != WMH_MODE_BATCHED)
        return fail(ctx, WMH_E_ARG, "wmh_hash_noalloc runs the batched walk only (mode %d)", o.mode);
    WMH_NA_HIP(ctx, hipSetDevice(ctx->device));
    {
        const hipError_t e = static_scratch_init(ctx->device);
        if (e != hipSuccess) return device_fail(ctx, e, "static scratch lookup");
    }
    unsigned char *base = scratch_address(ctx->device);
    if (!base) return fail(ctx, WMH_E_DEVICE, "no static scratch on device %d", ctx->device);
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    const Rows rows{row_ptr, col, val, n_rows, nnz};
    const Bounds b = bounds_view(ctx);
    auto *words = reinterpret_cast<CheckWords *>(base + kCheckWordsAt);
    auto *counter = reinterpret_cast<unsigned long long *>(base + kTileCounterAt);
    void *entries = base + kStreamAt;

    RowStats stats;
    if (o.validate) {
        const wmh_status st = gather_stats(ctx, rows, k, s, true, false, &stats, false, words);
        if (st != WMH_OK) return st;
    }
    BatchedPlan plan{};
    if (!plan_batched(ctx, k, stats, o, &plan))
        return fail(ctx, WMH_E_ARG, "no batched plan fits for D=%u with these options", ctx->dims);

    // The stream must fit the array.  A depth the caller asked for, and the stream of the
    // independent-rows walk (which cannot do without one), are taken as given or rejected; the
    // planner's own depth shrinks to whole cycles that fit (steps past it are drawn in-lane,
    // with the same values).
    const size_t room = kScratchBytes - kStreamAt;
    if (plan.stream_bytes(k) > room) {
        const bool depth_given = o.stream_depth != 0 && o.stream_depth != UINT32_MAX;
        if (depth_given || plan.independent_rows)
            return fail(ctx, WMH_E_ARG,
                        "a shared stream of %zu bytes (depth %u, k %u) exceeds the %zu bytes of "
                        "static scratch",
                        plan.stream_bytes(k), plan.stream_depth, k, room);
        const size_t entry = plan.packed ? 4u : 8u;
        const size_t fit = room / entry;  // entries: depth * k + one spare cycle
        const size_t depth = fit > plan.cycle() ? (fit - plan.cycle()) / k : 0;
        plan.stream_depth = (uint32_t)(std::min<size_t>(depth, plan.stream_depth) / plan.cycle() *
                                       plan.cycle());
    }

    const int per_cu = std::max(1, batched_blocks_per_cu(ctx->dims, plan));
    const uint64_t n_blocks = (n_rows + plan.rows_per_block - 1) / plan.rows_per_block;
    const uint64_t n_tiles = n_blocks * ((k + plan.hashes_per_tile - 1) / plan.hashes_per_tile);
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)ctx->cu_count * per_cu, n_tiles);

    const bool profile = o.profile != 0;
    ctx->profiled = false;
    if (plan.stream_depth)
        WMH_NA_HIP(ctx, launch_stream_build(b, seed, k, plan.stream_depth, plan.packed,
                                            plan.scale(), plan.coarse ? plan.coarse_bits : 0u,
                                            entries, s));
    WMH_NA_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(counter), 0u,
                                    2 * kMaxHashGroups, s));
    if (profile) WMH_NA_HIP(ctx, hipEventRecord(ctx->ev[1], s));
    WMH_NA_HIP(ctx, launch_batched(b, rows, k, seed, sig, plan, entries, counter, grid, s));
    if (profile) WMH_NA_HIP(ctx, hipEventRecord(ctx->ev[2], s));
    ctx->profiled = profile;
    ctx->profiled_stream = false;
    ctx->last_mode = WMH_MODE_BATCHED;
    ctx->last_plan = plan;
    if (o.sync) WMH_NA_HIP(ctx, hipStreamSynchronize(s));
    return WMH_OK;
}
