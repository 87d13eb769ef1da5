// Autotuner of the batched walk's tile plan: rows per block R, hash ids per tile J and
// wavefronts per workgroup W (the scheduling choices of the persistent launch; they change
// only the time, never a hash value).  Rows the planner sends to the component index get the
// index rows kernel's plan tuned instead: wavefronts per workgroup, keys per round trip and
// how wavefronts take rows.  Each candidate plan hashes the caller's rows on the
// device, timed with HIP events; the fastest is kept in the context under (D, value width, k,
// step class) and taken by later wmh_hash calls whose key matches and which leave the plan
// options at 0.  Results can be saved to and loaded from a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

namespace {

constexpr char kTuneHeader[] = "wmh-tune 6";
constexpr int32_t kIndexWalk = 4;  // a tuning line of the index rows kernel

void put_entry(wmh_ctx *ctx, const TuneEntry &e)
{
    for (TuneEntry &x : ctx->tuned)
        if (x.key == e.key) {
            x = e;
            return;
        }
    ctx->tuned.push_back(e);
}

void put_index_entry(wmh_ctx *ctx, const IndexTuneEntry &e)
{
    for (IndexTuneEntry &x : ctx->tuned_index)
        if (x.key == e.key) {
            x = e;
            return;
        }
    ctx->tuned_index.push_back(e);
}

bool valid_index_plan(uint32_t batch, uint32_t claim, uint32_t W)
{
    return (batch == 8 || batch == 16) && (claim == 1 || claim == 2) && W >= 1 &&
           W <= kIndexMaxWaves;
}

bool valid_plan(uint32_t R, uint32_t J, uint32_t W, int32_t walk, uint32_t K, uint32_t G,
                int32_t V)
{
    return (R == 1 || R == 2 || R == 4 || R == 8 || R == 16) && J >= 1 && W >= 1 && W <= 16 &&
           (walk == 1 || (walk == 2 && R == 4) || (walk == 3 && R == 1 && K == 1)) &&
           (K == R || (K == 4 && R < 4)) && G >= 1 && G <= kMaxHashGroups &&
           (G == 1 || walk == 3) && (V == 1 || (V == 2 && walk != 2 && R <= 4));
}

}  // namespace

extern "C" {

wmh_status wmh_tune(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                    const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k, uint64_t seed,
                    uint16_t *sig, void *stream, uint32_t reps, wmh_tune_result *out)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (!ctx->has_bounds) return fail(ctx, WMH_E_NO_BOUNDS, "wmh_set_bounds was not called");
    if (k == 0 || k > kMaxK) return fail(ctx, WMH_E_ARG, "k must be in [1, 2^24]");
    if (n_rows == 0 || !row_ptr || !sig || !out || (nnz && (!col || !val)))
        return fail(ctx, WMH_E_ARG, "null buffer or no rows");
    if (reps == 0) reps = 3;
    if (reps > 100) return fail(ctx, WMH_E_ARG, "reps must be in [1, 100]");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    const Rows rows{row_ptr, col, val, n_rows, nnz};
    RowStats stats;
    wmh_status st = gather_stats(ctx, rows, k, s, true, index_fits(k), &stats);
    if (st != WMH_OK) return st;

    wmh_opts base;
    wmh_opts_init(&base);
    BatchedPlan def{};
    const bool batched_ok = plan_batched(ctx, k, stats, base, &def, false);
    // the index's build is left out: the tuner builds it, and later calls reuse it
    const bool to_index = choose_path(ctx, WMH_MODE_AUTO, batched_ok, true, k, n_rows, nnz,
                                      stats) == Path::kIndexed;
    if (!batched_ok && !to_index)
        return fail(ctx, WMH_E_ARG, "no batched plan fits for D=%u", ctx->dims);

    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return fail(ctx, WMH_E_DEVICE, "hipEventCreate");
    }
    // best of `reps` timed wmh_hash calls with options o after one untimed call
    auto time_call = [&](const wmh_opts &o, float *ms) -> wmh_status {
        float best = 1e30f;
        for (uint32_t r = 0; r <= reps; ++r) {
            if (hipEventRecord(t0, s) != hipSuccess) return WMH_E_DEVICE;
            wmh_status h = wmh_hash(ctx, row_ptr, col, val, n_rows, nnz, k, seed, sig, s, &o);
            if (h != WMH_OK) return h;
            if (hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess)
                return WMH_E_DEVICE;
            float e = 0.f;
            if (hipEventElapsedTime(&e, t0, t1) != hipSuccess) return WMH_E_DEVICE;
            if (r > 0) best = std::min(best, e);
        }
        *ms = best;
        return WMH_OK;
    };

    if (to_index) {
        // the index rows kernel's plans: wavefronts per workgroup x keys per trip x claims
        wmh_opts o = base;
        o.mode = WMH_MODE_INDEXED;
        o.validate = 0;
        o.use_graph = 0;
        float default_ms = 0.f;
        st = time_call(o, &default_ms);  // the launcher's own choices (builds the index)
        IndexTuneEntry best;
        best.key = tune_key(ctx, k, stats);
        best.ms = 1e30f;
        uint32_t tried = 1;
        for (uint32_t W : {1u, 2u, 4u, 8u, 16u}) {
            if (index_rows_waves(k, W) == 0) continue;
            for (uint32_t B : {16u, 8u}) {
                for (uint32_t C : {1u, 2u}) {
                    if (st != WMH_OK) break;
                    o.waves_per_block = W;
                    o.index_batch = B;
                    o.index_claim = C;
                    float ms = 0.f;
                    st = time_call(o, &ms);
                    if (st != WMH_OK) break;
                    ++tried;
                    if (ms < best.ms) {
                        best.plan.waves = W;
                        best.plan.batch = B;
                        best.plan.claim = C;
                        best.ms = ms;
                    }
                }
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (st != WMH_OK) return st;
        put_index_entry(ctx, best);
        wmh_tune_result res{};
        res.waves_per_block = best.plan.waves;
        res.index_batch = best.plan.batch;
        res.index_claim = best.plan.claim;
        res.best_ms = best.ms;
        res.default_ms = default_ms;
        res.candidates = tried;
        res.steps_class = best.key.steps_class;
        res.walk = kIndexWalk;
        *out = res;
        return WMH_OK;
    }
    // best of `reps` timed calls after one untimed call; <0 when the plan does not fit
    auto time_plan = [&](uint32_t R, uint32_t J, uint32_t W, int32_t walk, uint32_t K,
                         uint32_t G, int32_t V, float *ms) -> wmh_status {
        wmh_opts o = base;
        o.walk = walk;
        o.hash_groups = G;
        o.values = V;
        o.steps_per_lane = K;
        o.mode = WMH_MODE_BATCHED;
        o.validate = 0;
        o.use_graph = 0;
        o.rows_per_block = R;
        o.hashes_per_tile = J;
        o.waves_per_block = W;
        o.stream_depth = def.stream_depth;
        BatchedPlan p{};
        *ms = -1.f;
        if (!plan_batched(ctx, k, stats, o, &p, false)) return WMH_OK;
        return time_call(o, ms);
    };

    wmh_tune_result res{};
    float default_ms = 0.f;
    const int32_t def_values = def.coarse ? 2 : 1;
    const int32_t def_walk = def.ballot ? 3 : def.independent_rows ? 2 : 1;
    st = time_plan(def.rows_per_block, def.hashes_per_tile, def.waves_per_block, def_walk,
                   def.steps_per_lane, 1, def_values, &default_ms);
    TuneEntry best;
    best.key = tune_key(ctx, k, stats);
    best.R = def.rows_per_block;
    best.J = def.hashes_per_tile;
    best.W = def.waves_per_block;
    best.walk = def_walk;
    best.K = def.steps_per_lane;
    best.V = def_values;
    best.ms = default_ms;
    uint32_t tried = 1;
    std::vector<uint32_t> Js{std::min(k, 1024u), std::min(k, 512u), std::min(k, 256u)};
    Js.erase(std::unique(Js.begin(), Js.end()), Js.end());
    // shared windows for every R with K = R, and K = 4 for R < 4; independent rows at R = 4;
    // the ballot walk at R = 1
    struct Shape {
        int32_t walk;
        uint32_t R, K;
    };
    const Shape shapes[] = {{1, 1, 1}, {1, 1, 4}, {1, 2, 2}, {1, 2, 4}, {1, 4, 4},
                            {1, 8, 8}, {1, 16, 16}, {2, 4, 4}, {3, 1, 1}};
    // the ballot walk also with its hash ids in 2, 4 or 8 groups (J then follows from G)
    std::vector<uint32_t> groups_of_ballot{1u};
    for (uint32_t G : {2u, 4u, 8u})
        if ((uint64_t)(G - 1) * ((k + G - 1) / G) < k) groups_of_ballot.push_back(G);
    // rows with a bound of 65536 or more: every plan with exact 32-bit rows and with coarse
    // codes (the latter without hash groups)
    std::vector<int32_t> values{1};
    if (ctx->max_bound > 0xFFFFu) values.push_back(2);
    for (const Shape &sh : shapes) {
        for (int32_t V : values) {
            if (V == 2 && (sh.walk == 2 || sh.R > 4)) continue;
            for (uint32_t G : sh.walk == 3 && V == 1 ? groups_of_ballot : std::vector<uint32_t>{1u}) {
                for (uint32_t W : {4u, 8u, 16u}) {
                    for (uint32_t J : G == 1 ? Js : std::vector<uint32_t>{(k + G - 1) / G}) {
                        if (st != WMH_OK) break;
                        if (sh.walk == def_walk && sh.R == def.rows_per_block &&
                            sh.K == def.steps_per_lane && J == def.hashes_per_tile &&
                            W == def.waves_per_block && V == def_values && G == 1)
                            continue;
                        float ms = -1.f;
                        st = time_plan(sh.R, J, W, sh.walk, sh.K, G, V, &ms);
                        if (st == WMH_OK && ms >= 0.f) {
                            ++tried;
                            if (ms < best.ms) {
                                best.R = sh.R;
                                best.J = J;
                                best.W = W;
                                best.walk = sh.walk;
                                best.K = sh.K;
                                best.G = G;
                                best.V = V;
                                best.ms = ms;
                            }
                        }
                    }
                }
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != WMH_OK) return st;
    put_entry(ctx, best);
    res.rows_per_block = best.R;
    res.hashes_per_tile = best.J;
    res.waves_per_block = best.W;
    res.stream_depth = def.stream_depth;
    res.best_ms = best.ms;
    res.default_ms = default_ms;
    res.candidates = tried;
    res.steps_class = best.key.steps_class;
    res.walk = best.walk;
    res.steps_per_lane = best.K;
    res.hash_groups = best.G;
    res.values = best.V;
    *out = res;
    return WMH_OK;
}

wmh_status wmh_tune_save(wmh_ctx *ctx, const char *path)
{
    if (!ctx || !path) return WMH_E_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(ctx, WMH_E_ARG, "cannot write %s", path);
    std::fprintf(f, "%s\n", kTuneHeader);
    for (const TuneEntry &e : ctx->tuned)
        std::fprintf(f, "%u %d %u %d %u %u %u %d %u %u %d %.6f\n", e.key.dims,
                     e.key.narrow ? 1 : 0, e.key.k, e.key.steps_class, e.R, e.J, e.W, e.walk, e.K,
                     e.G, e.V, (double)e.ms);
    // index rows plans: keys per trip and claim in the R and J columns, walk 4
    for (const IndexTuneEntry &e : ctx->tuned_index)
        std::fprintf(f, "%u %d %u %d %u %u %u %d %u %u %d %.6f\n", e.key.dims,
                     e.key.narrow ? 1 : 0, e.key.k, e.key.steps_class, e.plan.batch, e.plan.claim,
                     e.plan.waves, kIndexWalk, 0u, 1u, 0, (double)e.ms);
    const bool ok = std::fclose(f) == 0;
    return ok ? WMH_OK : fail(ctx, WMH_E_ARG, "cannot write %s", path);
}

wmh_status wmh_tune_load(wmh_ctx *ctx, const char *path)
{
    if (!ctx || !path) return WMH_E_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(ctx, WMH_E_ARG, "cannot read %s", path);
    char line[256];
    std::vector<TuneEntry> got;
    std::vector<IndexTuneEntry> got_index;
    bool ok = std::fgets(line, sizeof(line), f) &&
              std::strncmp(line, kTuneHeader, sizeof(kTuneHeader) - 1) == 0;
    while (ok && std::fgets(line, sizeof(line), f)) {
        TuneEntry e;
        int narrow = 0;
        double ms = 0;
        if (std::sscanf(line, "%u %d %u %d %u %u %u %d %u %u %d %lf", &e.key.dims, &narrow,
                        &e.key.k, &e.key.steps_class, &e.R, &e.J, &e.W, &e.walk, &e.K, &e.G,
                        &e.V, &ms) != 12 ||
            (narrow != 0 && narrow != 1) || e.key.k == 0) {
            ok = false;
            break;
        }
        e.key.narrow = narrow != 0;
        e.ms = (float)ms;
        if (e.walk == kIndexWalk) {
            if (!valid_index_plan(e.R, e.J, e.W) || index_rows_waves(e.key.k, e.W) == 0) {
                ok = false;
                break;
            }
            IndexTuneEntry x;
            x.key = e.key;
            x.plan.batch = e.R;
            x.plan.claim = e.J;
            x.plan.waves = e.W;
            x.ms = e.ms;
            got_index.push_back(x);
            continue;
        }
        if (!valid_plan(e.R, e.J, e.W, e.walk, e.K, e.G, e.V)) {
            ok = false;
            break;
        }
        got.push_back(e);
    }
    std::fclose(f);
    if (!ok) return fail(ctx, WMH_E_ARG, "%s is not a tuning file", path);
    for (const TuneEntry &e : got) put_entry(ctx, e);
    for (const IndexTuneEntry &e : got_index) put_index_entry(ctx, e);
    return WMH_OK;
}

}  // extern "C"
