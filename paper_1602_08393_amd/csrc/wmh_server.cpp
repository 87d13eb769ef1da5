// Serving loop of libwmh: continuous batching of hash requests on one device.
//
// Requests are queued by any host thread and admitted, in arrival order, by one worker thread
// whenever a slot (a HIP stream with its own buffers) is free and the admitted device bytes
// stay within the budget.  Consecutive queued requests whose rows add up to at most
// group_rows are admitted together into one slot as a group: their rows are laid end to end
// and go through one validation pass, one walk or index launch and one copy out, which small
// requests would otherwise each pay for.  An admitted group runs in two phases on its slot's
// stream: its rows are copied in and checked by the device validation pass (which also
// gathers the planner's statistics); once the check words are back, the worker either
// completes the group (a group whose rows fail the check completes the request holding the
// first bad row with the error and queues the others again, alone) or launches the chosen
// path and the copy out.  Requests overlap on the device and
// the worker never blocks on one.  The bounds tables and the shared position stream are built
// once and stay device-resident.  Every request computes the same function as wmh_hash on its
// rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

namespace {

// The largest number of intervals holding one instant (intervals closed on the left, open on
// the right), and with `overlap_s` the total seconds during which at least two of them do.
uint64_t most_at_once(const std::vector<std::pair<float, float>> &iv, double *overlap_s)
{
    std::vector<std::pair<float, int>> ev;
    ev.reserve(2 * iv.size());
    for (const auto &p : iv) {
        ev.emplace_back(p.first, +1);
        ev.emplace_back(p.second, -1);
    }
    std::sort(ev.begin(), ev.end());  // at equal times ends (-1) come before starts (+1)
    int64_t now = 0, most = 0;
    double two_or_more_ms = 0.0;
    for (size_t i = 0; i < ev.size(); ++i) {
        now += ev[i].second;
        most = std::max(most, now);
        if (now >= 2 && i + 1 < ev.size()) two_or_more_ms += ev[i + 1].first - ev[i].first;
    }
    if (overlap_s) *overlap_s = two_or_more_ms * 1e-3;
    return (uint64_t)most;
}

uint64_t steady_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t id = 0;
    const uint64_t *row_ptr = nullptr;
    const uint32_t *col = nullptr;
    const uint32_t *val = nullptr;
    uint64_t n_rows = 0, nnz = 0;
    uint16_t *sig = nullptr;
    uint64_t arrival_ns = 0, admit_ns = 0, done_ns = 0;
    uint64_t bytes = 0;
    bool retried = false;  // back in the queue after its group failed the check: admitted alone
    bool done = false;
    wmh_status status = WMH_OK;
};

constexpr size_t kMaxGroup = 64;  // requests admitted together into one slot

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t finished = nullptr;
    uint64_t *h_row_ptr = nullptr;  // pinned: a group's row_ptr, requests laid end to end
    uint64_t cap_h_rows = 0;
    uint64_t *d_row_ptr = nullptr;
    uint32_t *d_col = nullptr, *d_val = nullptr;
    uint16_t *d_sig = nullptr;
    uint16_t *h_sig = nullptr;  // pinned staging of the signatures
    uint64_t cap_rows = 0, cap_col = 0, cap_val = 0, cap_sig = 0, cap_h_sig = 0;
    unsigned long long *d_tile_counter = nullptr;
    unsigned long long *d_row_counter = nullptr;
    CheckWords *d_check = nullptr;  // the validation pass's words
    CheckWords *h_check = nullptr;  // pinned copy, read once `checked` has fired
    hipEvent_t checked = nullptr;
    // timing events of the group on the slot: its first copy in, the start of its walk and the
    // end of its copy out (device timestamps, read at completion)
    hipEvent_t t_begin = nullptr, t_compute = nullptr, t_end = nullptr;
    std::vector<Request *> reqs;  // the admitted group, in arrival order (empty: slot free)
    uint64_t rows = 0, nnz = 0;   // the group's rows and nonzeros
    bool computing = false;  // past the check: the walk and the copy out are queued
};

// Grows a slot buffer to hold `want` elements, by at least half its size each time: freeing
// the old buffer waits for the device, so growth must stay rare (wmh_server_reserve sizes the
// buffers up front).
template <typename T>
hipError_t grow_device(T **p, uint64_t *cap, uint64_t want)
{
    if (want <= *cap && *p) return hipSuccess;
    const uint64_t n = std::max<uint64_t>({want, 1, *cap + *cap / 2});
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e == hipSuccess) *cap = n;
    return e;
}

// The slot's buffers for a request of n_rows rows and nnz nonzeros with k hashes per row.
hipError_t grow_slot(Slot &slot, uint64_t n_rows, uint64_t nnz, uint32_t k)
{
    const uint64_t sig_elems = n_rows * (uint64_t)k;
    hipError_t e = grow_device(&slot.d_row_ptr, &slot.cap_rows, n_rows + 1);
    if (e == hipSuccess) e = grow_device(&slot.d_col, &slot.cap_col, nnz);
    if (e == hipSuccess) e = grow_device(&slot.d_val, &slot.cap_val, nnz);
    if (e == hipSuccess) e = grow_device(&slot.d_sig, &slot.cap_sig, sig_elems);
    if (e == hipSuccess && (slot.cap_h_sig < sig_elems || !slot.h_sig)) {
        const uint64_t n = std::max<uint64_t>({sig_elems, 1, slot.cap_h_sig + slot.cap_h_sig / 2});
        if (slot.h_sig) (void)hipHostFree(slot.h_sig);
        slot.h_sig = nullptr;
        slot.cap_h_sig = 0;
        e = hipHostMalloc(reinterpret_cast<void **>(&slot.h_sig), n * sizeof(uint16_t),
                          hipHostMallocDefault);
        if (e == hipSuccess) slot.cap_h_sig = n;
    }
    if (e == hipSuccess && (slot.cap_h_rows < n_rows + 1 || !slot.h_row_ptr)) {
        const uint64_t n = std::max<uint64_t>({n_rows + 1, 2, slot.cap_h_rows + slot.cap_h_rows / 2});
        if (slot.h_row_ptr) (void)hipHostFree(slot.h_row_ptr);
        slot.h_row_ptr = nullptr;
        slot.cap_h_rows = 0;
        e = hipHostMalloc(reinterpret_cast<void **>(&slot.h_row_ptr), n * sizeof(uint64_t),
                          hipHostMallocDefault);
        if (e == hipSuccess) slot.cap_h_rows = n;
    }
    return e;
}

}  // namespace

struct wmh_server {
    wmh_ctx *ctx = nullptr;
    wmh_server_config cfg{};
    std::vector<Slot> slots;
    // walk plan shared by every request
    bool batched = false;
    BatchedPlan plan{};
    uint32_t grid = 0;
    void *d_stream = nullptr;
    // component index for requests whose green fraction is small (built on first use)
    OwnedIndex index;
    uint32_t index_grid = 0;
    // queue and bookkeeping (guarded by mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> requests;
    uint64_t next_id = 1;
    uint64_t inflight_bytes = 0;
    uint32_t inflight = 0;
    bool stopping = false;
    std::thread worker;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, max_queued = 0, peak_bytes = 0;
    uint64_t hashes = 0, loads = 0;
    std::vector<double> latencies_ms;
    uint64_t first_admit_ns = 0, last_done_ns = 0;
    // device intervals of completed groups, in ms after t_ref: [first copy in, end of copy
    // out] and [start of the walk, end of copy out]
    hipEvent_t t_ref = nullptr;
    std::vector<std::pair<float, float>> on_device, computing;

    wmh_status launch_check(Slot &slot);
    wmh_status launch_compute(Slot &slot, uint64_t *bad_row);
    void complete_one(Slot &slot, Request &r, uint64_t row0, wmh_status st);
    void complete(Slot &slot, wmh_status st);
    void release(Slot &slot, Request *culprit, wmh_status st);
    void run();
};

// Phase one: buffers, copy in, validation pass and the copy of its words to the host.  A lone
// request is copied as given; a group's requests are laid end to end, each contributing the
// nonzeros its rows cover (row_ptr[0] up to row_ptr[n_rows]), with its row_ptr rebased on the
// host in pinned memory.
wmh_status wmh_server::launch_check(Slot &slot)
{
    const uint32_t k = cfg.k;
    const bool group = slot.reqs.size() > 1;
    slot.rows = slot.nnz = 0;
    for (const Request *r : slot.reqs) {
        slot.rows += r->n_rows;
        slot.nnz += group ? r->row_ptr[r->n_rows] - r->row_ptr[0] : r->nnz;
    }
    hipError_t e = grow_slot(slot, slot.rows, slot.nnz, k);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? WMH_E_NOMEM : WMH_E_DEVICE;

    hipStream_t s = slot.stream;
    e = hipEventRecord(slot.t_begin, s);
    if (!group) {
        const Request &r = *slot.reqs[0];
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot.d_row_ptr, r.row_ptr, (r.n_rows + 1) * sizeof(uint64_t),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess && r.nnz)
            e = hipMemcpyAsync(slot.d_col, r.col, r.nnz * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && r.nnz)
            e = hipMemcpyAsync(slot.d_val, r.val, r.nnz * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    } else {
        // the slot is free, so no copy still reads its staging buffer
        uint64_t row0 = 0, nz0 = 0;
        for (const Request *r : slot.reqs) {
            const uint64_t lo = r->row_ptr[0], used = r->row_ptr[r->n_rows] - lo;
            for (uint64_t i = 0; i < r->n_rows; ++i)
                slot.h_row_ptr[row0 + i] = r->row_ptr[i] - lo + nz0;
            if (e == hipSuccess && used)
                e = hipMemcpyAsync(slot.d_col + nz0, r->col + lo, used * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess && used)
                e = hipMemcpyAsync(slot.d_val + nz0, r->val + lo, used * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, s);
            row0 += r->n_rows;
            nz0 += used;
        }
        slot.h_row_ptr[row0] = nz0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot.d_row_ptr, slot.h_row_ptr, (row0 + 1) * sizeof(uint64_t),
                               hipMemcpyHostToDevice, s);
    }
    const Rows rows{slot.d_row_ptr, slot.d_col, slot.d_val, slot.rows, slot.nnz};
    // first_error and min_green start at ~0, the counters at 0 (as in wmh_hash's pass); the
    // index-key estimate only when the planner may take the index
    const bool want_keys = cfg.mode == WMH_MODE_AUTO && index_fits(cfg.k);
    if (e == hipSuccess) e = launch_check_init(slot.d_check, s);
    if (e == hipSuccess)
        e = launch_validate(rows, ctx->d_bound, ctx->dims, ctx->total, k, want_keys, slot.d_check, s,
                            nullptr, ctx->d_bound_blocks);
    if (e == hipSuccess)
        e = hipMemcpyAsync(slot.h_check, slot.d_check, sizeof(CheckWords), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(slot.checked, s);
    slot.computing = false;
    return e == hipSuccess ? WMH_OK : WMH_E_DEVICE;
}

// Phase two, once the check words are on the host: the rows' status, then the chosen path and
// the copy out (nothing is launched for rows that failed the check; *bad_row is then the
// group's first bad row).
wmh_status wmh_server::launch_compute(Slot &slot, uint64_t *bad_row)
{
    const CheckWords v = *slot.h_check;
    if (v.first_error != ~0ull) {
        *bad_row = v.first_error >> 4;
        return check_status((uint32_t)(v.first_error & 15u));
    }
    RowStats stats;
    stats.known = true;
    stats.nonempty = slot.rows - std::min<uint64_t>(slot.rows, v.n_empty);
    stats.min_green = v.min_green;
    stats.walk_steps = v.walk_steps;
    stats.index_keys = v.index_keys;
    stats.keys_known = cfg.mode == WMH_MODE_AUTO && index_fits(cfg.k);
    const uint32_t k = cfg.k;
    const uint64_t n_rows = slot.rows;
    const uint64_t sig_elems = n_rows * (uint64_t)k;
    hipStream_t s = slot.stream;
    hipError_t e = hipSuccess;
    const Rows rows{slot.d_row_ptr, slot.d_col, slot.d_val, n_rows, slot.nnz};
    const Bounds b = bounds_view(ctx);
    // the index is built once per loop, so its cost is left out of the comparison
    const Path path = choose_path(ctx, cfg.mode, batched, true, k, n_rows, slot.nnz, stats);
    e = hipEventRecord(slot.t_compute, s);
    if (e == hipSuccess && path == Path::kIndexed) {
        if (!index.valid) {
            // the worker is the only builder; the first indexed request waits for the build so
            // that requests on the other slots' streams find it complete
            const wmh_status st = ensure_index(ctx, &index, cfg.seed, k, s, false);
            if (st != WMH_OK) return st;
            e = hipStreamSynchronize(s);
        }
        if (e == hipSuccess)
            e = launch_index_rows(rows, index.buf, b, k, slot.d_sig, slot.d_row_counter,
                                  index_grid, s);
        if (e == hipSuccess) e = hipEventRecord(index.used, s);
    } else if (e == hipSuccess) {
        if (batched) {
            e = launch_fill_u32(reinterpret_cast<uint32_t *>(slot.d_tile_counter), 0u,
                                2 * kMaxHashGroups, s);
            if (e == hipSuccess)
                e = launch_batched(b, rows, k, cfg.seed, slot.d_sig, plan, d_stream,
                                   slot.d_tile_counter, grid, s);
        } else {
            const bool narrow = ctx->max_bound <= 0xFFFFu;
            const bool dense = (size_t)4 * ctx->dims * (narrow ? 2 : 4) <= 64 * 1024;
            for (uint64_t r0 = 0; r0 < n_rows && e == hipSuccess; r0 += 8192)
                e = launch_plain(b, rows, r0, std::min(n_rows, r0 + 8192), k, cfg.seed,
                                 slot.d_sig, narrow, dense, s);
        }
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(slot.h_sig, slot.d_sig, sig_elems * sizeof(uint16_t),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(slot.t_end, s);
    if (e == hipSuccess) e = hipEventRecord(slot.finished, s);
    slot.computing = true;
    return e == hipSuccess ? WMH_OK : WMH_E_DEVICE;
}

// One request of a slot's group, whose rows start at group row row0.  Called with mu held.
void wmh_server::complete_one(Slot &slot, Request &r, uint64_t row0, wmh_status st)
{
    if (st == WMH_OK)
        std::memcpy(r.sig, slot.h_sig + row0 * (uint64_t)cfg.k,
                    r.n_rows * (uint64_t)cfg.k * sizeof(uint16_t));
    r.done_ns = steady_ns();
    r.status = st;
    r.done = true;
    inflight_bytes -= r.bytes;
    --inflight;
    if (st == WMH_OK) {
        ++completed;
        hashes += r.n_rows * (uint64_t)cfg.k;
        latencies_ms.push_back((double)(r.done_ns - r.arrival_ns) * 1e-6);
        last_done_ns = std::max(last_done_ns, r.done_ns);
    } else if (st == WMH_E_ROW_PTR || st == WMH_E_COL_RANGE || st == WMH_E_UNSORTED ||
               st == WMH_E_BOUND) {
        ++rejected;  // the caller's rows, reported by wmh_server_poll / wait
    } else {
        ++failed;
    }
}

// Every request of the slot's group with status st, and the group's device intervals.  Called
// with mu held.
void wmh_server::complete(Slot &slot, wmh_status st)
{
    if (st == WMH_OK) {
        ++loads;
        // every event of the slot has fired once `finished` has
        float b = 0.f, c = 0.f, d = 0.f;
        if (hipEventElapsedTime(&b, t_ref, slot.t_begin) == hipSuccess &&
            hipEventElapsedTime(&c, t_ref, slot.t_compute) == hipSuccess &&
            hipEventElapsedTime(&d, t_ref, slot.t_end) == hipSuccess) {
            on_device.emplace_back(b, d);
            computing.emplace_back(c, d);
        }
    }
    uint64_t row0 = 0;
    for (Request *r : slot.reqs) {
        complete_one(slot, *r, row0, st);
        row0 += r->n_rows;
    }
    slot.reqs.clear();
    cv_done.notify_all();
}

// A group that cannot go on together: the culprit, if any (the request holding the first bad
// row of a failed check), completes with status st; the others go back to the front of the
// queue in arrival order, marked to be admitted alone (their rows are checked again by
// themselves).  Called with mu held.
void wmh_server::release(Slot &slot, Request *culprit, wmh_status st)
{
    for (size_t i = slot.reqs.size(); i-- > 0;) {
        Request *r = slot.reqs[i];
        if (r == culprit) continue;
        inflight_bytes -= r->bytes;
        --inflight;
        r->retried = true;
        queue.push_front(r);
    }
    if (culprit) complete_one(slot, *culprit, 0, st);
    slot.reqs.clear();
    cv_done.notify_all();
}

void wmh_server::run()
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    const uint64_t group_rows = cfg.group_rows ? cfg.group_rows : 2048;
    while (true) {
        // checked groups go on to their walk; finished ones complete
        for (Slot &slot : slots) {
            if (slot.reqs.empty()) continue;
            const hipError_t q = hipEventQuery(slot.computing ? slot.finished : slot.checked);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                complete(slot, WMH_E_DEVICE);
            } else if (slot.computing) {
                complete(slot, WMH_OK);
            } else {
                uint64_t bad_row = ~0ull;
                lk.unlock();
                const wmh_status st = launch_compute(slot, &bad_row);
                lk.lock();
                if (st == WMH_OK) continue;
                // the request holding the first bad row; every other request of a group is
                // checked again by itself
                Request *culprit = nullptr;
                uint64_t row0 = 0;
                for (Request *r : slot.reqs) {
                    if (bad_row >= row0 && bad_row < row0 + r->n_rows) culprit = r;
                    row0 += r->n_rows;
                }
                if (slot.reqs.size() > 1 && culprit) release(slot, culprit, st);
                else complete(slot, st);
            }
        }
        // admissions, in arrival order: the front request and the queued requests after it
        // while their rows add up to at most group_rows
        while (!queue.empty()) {
            Slot *free_slot = nullptr;
            for (Slot &slot : slots)
                if (slot.reqs.empty()) {
                    free_slot = &slot;
                    break;
                }
            if (!free_slot) break;
            Request *first = queue.front();
            if (inflight > 0 && inflight_bytes + first->bytes > cfg.mem_budget) break;
            queue.pop_front();
            free_slot->reqs.push_back(first);
            uint64_t rows = first->n_rows, bytes = first->bytes;
            // a request retried after its group failed the check goes alone, and joins none
            while (!first->retried && !queue.empty() && free_slot->reqs.size() < kMaxGroup) {
                Request *r = queue.front();
                if (r->retried || rows + r->n_rows > group_rows ||
                    inflight_bytes + bytes + r->bytes > cfg.mem_budget)
                    break;
                queue.pop_front();
                free_slot->reqs.push_back(r);
                rows += r->n_rows;
                bytes += r->bytes;
            }
            const uint64_t now = steady_ns();
            for (Request *r : free_slot->reqs) r->admit_ns = now;
            if (!first_admit_ns) first_admit_ns = now;
            inflight_bytes += bytes;
            inflight += (uint32_t)free_slot->reqs.size();
            peak_bytes = std::max(peak_bytes, inflight_bytes);
            lk.unlock();
            const wmh_status st = launch_check(*free_slot);
            lk.lock();
            // a group whose buffers do not fit is admitted again one request at a time
            if (st == WMH_E_NOMEM && free_slot->reqs.size() > 1) release(*free_slot, nullptr, st);
            else if (st != WMH_OK) complete(*free_slot, st);
        }
        if (stopping && queue.empty() && inflight == 0) break;
        if (inflight > 0) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
        }
    }
}

extern "C" {

uint64_t wmh_server_now_ns(void) { return steady_ns(); }

wmh_status wmh_host_alloc(size_t bytes, void **ptr)
{
    if (!ptr) return WMH_E_ARG;
    *ptr = nullptr;
    if (bytes == 0) return WMH_OK;
    return hipHostMalloc(ptr, bytes, hipHostMallocDefault) == hipSuccess ? WMH_OK : WMH_E_NOMEM;
}

void wmh_host_free(void *ptr)
{
    if (ptr) (void)hipHostFree(ptr);
}

wmh_status wmh_server_create(wmh_ctx *ctx, const wmh_server_config *cfg_in, wmh_server **out)
{
    if (!ctx || !cfg_in || !out) return WMH_E_ARG;
    *out = nullptr;
    if (!ctx->has_bounds) return fail(ctx, WMH_E_NO_BOUNDS, "wmh_set_bounds was not called");
    wmh_server_config cfg = *cfg_in;
    if (cfg.k == 0 || cfg.k > kMaxK) return fail(ctx, WMH_E_ARG, "k must be in [1, 2^24]");
    if (cfg.slots == 0) cfg.slots = 8;
    if (cfg.slots > 64) return fail(ctx, WMH_E_ARG, "slots must be in [1, 64]");
    if (cfg.mem_budget == 0) cfg.mem_budget = 4ull << 30;
    if (cfg.mode < WMH_MODE_AUTO || cfg.mode > WMH_MODE_INDEXED)
        return fail(ctx, WMH_E_ARG, "unknown mode %d", cfg.mode);
    if (cfg.mode == WMH_MODE_INDEXED && !index_fits(cfg.k))
        return fail(ctx, WMH_E_ARG, "the component index needs k <= %u", kIndexMaxK);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");

    wmh_server *srv = new (std::nothrow) wmh_server();
    if (!srv) return WMH_E_NOMEM;
    srv->ctx = ctx;
    srv->cfg = cfg;
    wmh_opts o;
    wmh_opts_init(&o);
    o.stream_depth = cfg.stream_depth ? cfg.stream_depth : 8192;
    srv->batched = (cfg.mode == WMH_MODE_AUTO || cfg.mode == WMH_MODE_BATCHED) &&
                   plan_batched(ctx, cfg.k, RowStats{}, o, &srv->plan);
    srv->index_grid = (uint32_t)ctx->cu_count * (uint32_t)index_rows_blocks_per_cu(cfg.k);
    if (cfg.mode == WMH_MODE_BATCHED && !srv->batched) {
        delete srv;
        return fail(ctx, WMH_E_ARG, "no batched plan fits for D=%u", ctx->dims);
    }
    // the default depth keeps the stream within the planner's budget: with so many hash ids
    // that one cycle of them does not fit, every step is drawn in-lane
    if (srv->batched && !cfg.stream_depth && srv->plan.stream_bytes(cfg.k) > kStreamBudgetBytes)
        srv->plan.stream_depth = 0;
    hipError_t e = hipSuccess;
    if (srv->batched) {
        srv->grid = (uint32_t)(ctx->cu_count * std::max(1, batched_blocks_per_cu(ctx->dims, srv->plan)));
        if (srv->plan.stream_depth) {
            e = hipMalloc(&srv->d_stream, srv->plan.stream_bytes(cfg.k));
            if (e == hipSuccess)
                e = launch_stream_build(bounds_view(ctx), cfg.seed, cfg.k, srv->plan.stream_depth,
                                        srv->plan.packed, srv->plan.scale(),
                                        srv->plan.coarse ? srv->plan.coarse_bits : 0u,
                                        srv->d_stream, ctx->own_stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->own_stream);
        }
    }
    srv->slots.resize(cfg.slots);
    for (Slot &slot : srv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&slot.finished, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipMalloc(&slot.d_tile_counter, kMaxHashGroups * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMalloc(&slot.d_row_counter, sizeof(unsigned long long));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&slot.checked, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreate(&slot.t_begin);
        if (e == hipSuccess) e = hipEventCreate(&slot.t_compute);
        if (e == hipSuccess) e = hipEventCreate(&slot.t_end);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&slot.d_check), sizeof(CheckWords));
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&slot.h_check), sizeof(CheckWords),
                              hipHostMallocDefault);
    }
    // the origin of the device timestamps of every request
    if (e == hipSuccess) e = hipEventCreate(&srv->t_ref);
    if (e == hipSuccess) e = hipEventRecord(srv->t_ref, ctx->own_stream);
    if (e == hipSuccess) e = hipEventSynchronize(srv->t_ref);
    if (e != hipSuccess) {
        wmh_status st = device_fail(ctx, e, "server setup");
        wmh_server_destroy(srv);
        return st;
    }
    if (cfg.build_index && cfg.mode != WMH_MODE_BATCHED && cfg.mode != WMH_MODE_PLAIN &&
        index_fits(cfg.k)) {
        wmh_status st = ensure_index(ctx, &srv->index, cfg.seed, cfg.k, ctx->own_stream);
        if (st == WMH_OK) {
            const hipError_t se = hipStreamSynchronize(ctx->own_stream);
            if (se != hipSuccess) st = device_fail(ctx, se, "index build");
        }
        if (st != WMH_OK) {
            wmh_server_destroy(srv);
            return st;
        }
    }
    ctx->servers++;
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return WMH_OK;
}

wmh_status wmh_server_submit(wmh_server *srv, const uint64_t *row_ptr, const uint32_t *col,
                             const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint16_t *sig,
                             uint64_t arrival_ns, uint64_t *ticket)
{
    if (!srv || !ticket) return WMH_E_ARG;
    wmh_ctx *ctx = srv->ctx;
    if (!row_ptr || (n_rows && !sig) || (nnz && (!col || !val)))
        return fail(ctx, WMH_E_ARG, "null buffer");
    // row_ptr here (it sizes the copies); every entry is checked on the device
    for (uint64_t r = 0; r < n_rows; ++r)
        if (row_ptr[r] > row_ptr[r + 1] || row_ptr[r + 1] > nnz)
            return fail(ctx, WMH_E_ROW_PTR, "row %llu: row_ptr decreasing or beyond nnz",
                        (unsigned long long)r);
    const uint64_t bytes = (n_rows + 1) * 8 + nnz * 8 + n_rows * (uint64_t)srv->cfg.k * 2;
    if (bytes > srv->cfg.mem_budget)
        return fail(ctx, WMH_E_NOMEM, "request needs %llu bytes, budget %llu",
                    (unsigned long long)bytes, (unsigned long long)srv->cfg.mem_budget);
    Request *r = new (std::nothrow) Request();
    if (!r) return WMH_E_NOMEM;
    r->row_ptr = row_ptr;
    r->col = col;
    r->val = val;
    r->n_rows = n_rows;
    r->nnz = nnz;
    r->sig = sig;
    r->arrival_ns = arrival_ns ? arrival_ns : steady_ns();
    r->bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->id = srv->next_id++;
        srv->requests[r->id] = r;
        ++srv->submitted;
        if (n_rows == 0) {
            r->done = true;
            r->done_ns = steady_ns();
        } else {
            srv->queue.push_back(r);
            srv->max_queued = std::max<uint64_t>(srv->max_queued, srv->queue.size());
        }
        *ticket = r->id;
    }
    srv->cv_work.notify_one();
    return WMH_OK;
}

wmh_status wmh_server_poll(wmh_server *srv, uint64_t ticket, int *done, double *latency_ms)
{
    if (!srv || !done) return WMH_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end()) return WMH_E_ARG;
    Request *r = it->second;
    *done = r->done ? 1 : 0;
    if (!r->done) return WMH_OK;
    if (latency_ms) *latency_ms = (double)(r->done_ns - r->arrival_ns) * 1e-6;
    const wmh_status st = r->status;
    srv->requests.erase(it);
    delete r;
    return st;
}

wmh_status wmh_server_wait(wmh_server *srv, uint64_t ticket, double *latency_ms)
{
    if (!srv) return WMH_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end()) return WMH_E_ARG;
    Request *r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    if (latency_ms) *latency_ms = (double)(r->done_ns - r->arrival_ns) * 1e-6;
    const wmh_status st = r->status;
    srv->requests.erase(ticket);
    delete r;
    return st;
}

wmh_status wmh_server_drain(wmh_server *srv)
{
    if (!srv) return WMH_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->queue.empty() && srv->inflight == 0; });
    return srv->failed ? WMH_E_DEVICE : WMH_OK;
}

wmh_status wmh_server_reserve(wmh_server *srv, uint64_t max_rows, uint64_t max_nnz)
{
    if (!srv) return WMH_E_ARG;
    wmh_ctx *ctx = srv->ctx;
    const uint64_t bytes = (max_rows + 1) * 8 + max_nnz * 8 + max_rows * (uint64_t)srv->cfg.k * 2;
    if (bytes > srv->cfg.mem_budget)
        return fail(ctx, WMH_E_NOMEM, "a request of %llu rows and %llu nonzeros exceeds the budget",
                    (unsigned long long)max_rows, (unsigned long long)max_nnz);
    std::unique_lock<std::mutex> lk(srv->mu);
    // with nothing queued or admitted the worker touches no slot while the lock is held
    srv->cv_done.wait(lk, [&] { return srv->queue.empty() && srv->inflight == 0; });
    if (hipSetDevice(ctx->device) != hipSuccess) return WMH_E_DEVICE;
    for (Slot &slot : srv->slots) {
        const hipError_t e = grow_slot(slot, max_rows, max_nnz, srv->cfg.k);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? WMH_E_NOMEM : WMH_E_DEVICE;
    }
    return WMH_OK;
}

wmh_status wmh_server_stats(wmh_server *srv, wmh_serving_stats *out)
{
    if (!srv || !out) return WMH_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->rejected = srv->rejected;
    out->queued = srv->queue.size();
    out->max_queued = srv->max_queued;
    out->peak_bytes = srv->peak_bytes;
    out->hashes = srv->hashes;
    out->loads = srv->loads;
    std::vector<double> v = srv->latencies_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(q * v.size()) - 1);
            return v[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->p999_ms = pct(0.999);
        out->max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / v.size();
    }
    if (srv->last_done_ns > srv->first_admit_ns && srv->first_admit_ns) {
        out->busy_s = (double)(srv->last_done_ns - srv->first_admit_ns) * 1e-9;
        out->hashes_per_s = (double)srv->hashes / out->busy_s;
    }
    out->max_on_device = most_at_once(srv->on_device, nullptr);
    out->max_computing = most_at_once(srv->computing, &out->overlap_s);
    return WMH_OK;
}

wmh_status wmh_server_reset_stats(wmh_server *srv)
{
    if (!srv) return WMH_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted = srv->queue.size() + srv->inflight;
    srv->completed = srv->failed = srv->rejected = 0;
    srv->max_queued = srv->queue.size();
    srv->peak_bytes = srv->inflight_bytes;
    srv->hashes = srv->loads = 0;
    srv->latencies_ms.clear();
    srv->on_device.clear();
    srv->computing.clear();
    srv->first_admit_ns = srv->last_done_ns = 0;
    return WMH_OK;
}

void wmh_server_destroy(wmh_server *srv)
{
    if (!srv) return;
    if (srv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stopping = true;
        }
        srv->cv_work.notify_all();
        srv->worker.join();
        srv->ctx->servers--;
    }
    (void)hipSetDevice(srv->ctx->device);
    for (Slot &slot : srv->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.d_row_ptr) (void)hipFree(slot.d_row_ptr);
        if (slot.d_col) (void)hipFree(slot.d_col);
        if (slot.d_val) (void)hipFree(slot.d_val);
        if (slot.d_sig) (void)hipFree(slot.d_sig);
        if (slot.h_sig) (void)hipHostFree(slot.h_sig);
        if (slot.h_row_ptr) (void)hipHostFree(slot.h_row_ptr);
        if (slot.d_tile_counter) (void)hipFree(slot.d_tile_counter);
        if (slot.d_row_counter) (void)hipFree(slot.d_row_counter);
        if (slot.finished) (void)hipEventDestroy(slot.finished);
        if (slot.checked) (void)hipEventDestroy(slot.checked);
        if (slot.t_begin) (void)hipEventDestroy(slot.t_begin);
        if (slot.t_compute) (void)hipEventDestroy(slot.t_compute);
        if (slot.t_end) (void)hipEventDestroy(slot.t_end);
        if (slot.d_check) (void)hipFree(slot.d_check);
        if (slot.h_check) (void)hipHostFree(slot.h_check);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
    }
    if (srv->d_stream) (void)hipFree(srv->d_stream);
    if (srv->t_ref) (void)hipEventDestroy(srv->t_ref);
    free_index(&srv->index);
    for (auto &kv : srv->requests) delete kv.second;
    delete srv;
}

}  // extern "C"
