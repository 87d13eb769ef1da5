// C-ABI of the (K, L) banding index (kernels in wmh_lsh.hip).
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

struct wmh_lsh {
    wmh_ctx *ctx = nullptr;
    uint64_t n = 0;
    uint32_t k = 0, K = 0, L = 0, cap_log2 = 0;
    uint16_t *bands = nullptr;
    unsigned long long *table_key = nullptr;
    uint32_t *table_head = nullptr;
    uint32_t *next = nullptr;
};

extern "C" {

void wmh_lsh_destroy(wmh_lsh *ix)
{
    if (!ix) return;
    (void)hipSetDevice(ix->ctx->device);
    if (ix->bands) (void)hipFree(ix->bands);
    if (ix->table_key) (void)hipFree(ix->table_key);
    if (ix->table_head) (void)hipFree(ix->table_head);
    if (ix->next) (void)hipFree(ix->next);
    delete ix;
}

wmh_status wmh_lsh_build(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                         uint32_t K, uint32_t L, void *stream, wmh_lsh **out)
{
    if (!ctx || !out) return WMH_E_ARG;
    *out = nullptr;
    ctx->last_error.clear();
    if (K == 0 || L == 0 || k == 0 || (uint64_t)K * L > k)
        return fail(ctx, WMH_E_ARG, "need 1 <= K, 1 <= L and K * L <= k");
    if (L > 4096) return fail(ctx, WMH_E_ARG, "L must be <= 4096");
    if (n_rows >= 0xFFFFFFFFull) return fail(ctx, WMH_E_ARG, "too many rows");
    if (n_rows && !sig) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    wmh_lsh *ix = new (std::nothrow) wmh_lsh();
    if (!ix) return WMH_E_NOMEM;
    ix->ctx = ctx;
    ix->n = n_rows;
    ix->k = k;
    ix->K = K;
    ix->L = L;
    uint32_t lg = 4;
    while ((1ull << lg) < 2 * n_rows) ++lg;  // at least twice as many slots as rows
    ix->cap_log2 = lg;
    const uint64_t cap = 1ull << lg;
    hipError_t e = hipMalloc(&ix->table_key, cap * L * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&ix->table_head, cap * L * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&ix->next, (n_rows ? n_rows : 1) * L * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&ix->bands, (n_rows ? n_rows : 1) * (uint64_t)L * K * sizeof(uint16_t));
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    if (e == hipSuccess)
        e = launch_lsh_build(sig, n_rows, k, K, L, lg, ix->bands, ix->table_key, ix->table_head,
                             ix->next, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        const wmh_status st = device_fail(ctx, e, "banding index");
        wmh_lsh_destroy(ix);
        return st;
    }
    *out = ix;
    return WMH_OK;
}

wmh_status wmh_lsh_query(wmh_lsh *ix, const uint16_t *query, uint64_t n_queries, uint32_t k,
                         uint32_t max_out, uint32_t *out, uint32_t *out_count, void *stream)
{
    if (!ix) return WMH_E_ARG;
    wmh_ctx *ctx = ix->ctx;
    ctx->last_error.clear();
    if (k != ix->k) return fail(ctx, WMH_E_ARG, "queries must have the index's k");
    if (n_queries == 0) return WMH_OK;
    if (!query || !out_count || (max_out && !out)) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    hipError_t e = launch_lsh_query(query, n_queries, k, ix->K, ix->L, ix->n, ix->cap_log2,
                                    ix->bands, ix->table_key, ix->table_head, ix->next, max_out,
                                    out, out_count, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? WMH_OK : device_fail(ctx, e, "banding query");
}

}  // extern "C"
