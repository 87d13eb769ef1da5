// C-ABI of the b-bit signature codec (kernels in wmh_codec.hip): width selection, packing,
// unpacking and collision counts on packed signatures.
#include <hip/hip_runtime.h>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

namespace {

hipStream_t pick(wmh_ctx *ctx, void *stream)
{
    return stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
}

wmh_status check_shape(wmh_ctx *ctx, uint32_t k, uint32_t bits)
{
    if (k == 0) return fail(ctx, WMH_E_ARG, "k must be >= 1");
    if (bits < 1 || bits > 16) return fail(ctx, WMH_E_ARG, "bits must be in [1, 16]");
    return WMH_OK;
}

}  // namespace

extern "C" {

uint32_t wmh_pack_words(uint32_t k, uint32_t bits) { return pack_words(k, bits); }

wmh_status wmh_sig_bits(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                        uint32_t *bits, uint32_t *max_value, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (k == 0 || !bits || (n_rows && !sig)) return fail(ctx, WMH_E_ARG, "null buffer or k = 0");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = pick(ctx, stream);
    uint32_t *m = reinterpret_cast<uint32_t *>(ctx->d_codec);
    hipError_t e = launch_fill_u32(m, 0u, 1, s);
    if (e == hipSuccess && n_rows) e = launch_sig_max(sig, n_rows * (uint64_t)k, m, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_codec, ctx->d_codec, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(ctx, e, "signature maximum");
    const uint32_t mx = *reinterpret_cast<const uint32_t *>(ctx->h_codec);
    uint32_t b = 1;
    while (b < 16 && (mx >> b) != 0) ++b;
    *bits = b;
    if (max_value) *max_value = mx;
    return WMH_OK;
}

wmh_status wmh_pack(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                    uint32_t bits, uint32_t *packed, uint64_t *n_saturated, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    wmh_status st = check_shape(ctx, k, bits);
    if (st != WMH_OK) return st;
    if (n_rows && (!sig || !packed)) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = pick(ctx, stream);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->d_codec), 0u, 2, s);
    if (e == hipSuccess && n_rows) e = launch_pack(sig, n_rows, k, bits, packed, ctx->d_codec, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_codec, ctx->d_codec, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(ctx, e, "pack");
    if (n_saturated) *n_saturated = ctx->h_codec[0];
    return WMH_OK;
}

wmh_status wmh_unpack(wmh_ctx *ctx, const uint32_t *packed, uint64_t n_rows, uint32_t k,
                      uint32_t bits, uint16_t *sig, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    wmh_status st = check_shape(ctx, k, bits);
    if (st != WMH_OK) return st;
    if (n_rows == 0) return WMH_OK;
    if (!sig || !packed) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = pick(ctx, stream);
    hipError_t e = launch_unpack(packed, n_rows, k, bits, sig, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? WMH_OK : device_fail(ctx, e, "unpack");
}

wmh_status wmh_packed_collisions(wmh_ctx *ctx, const uint32_t *A, uint64_t NA, const uint32_t *B,
                                 uint64_t NB, uint32_t k, uint32_t bits, uint32_t *counts,
                                 void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    wmh_status st = check_shape(ctx, k, bits);
    if (st != WMH_OK) return st;
    if (NA == 0 || NB == 0) return WMH_OK;
    if (!A || !B || !counts) return fail(ctx, WMH_E_ARG, "null buffer");
    if (NA > 65535ull * 64) return fail(ctx, WMH_E_ARG, "NA too large for one call (max 4194240)");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = pick(ctx, stream);
    hipError_t e = launch_packed_collisions(A, NA, B, NB, k, bits, counts, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? WMH_OK : device_fail(ctx, e, "packed collisions");
}

wmh_status wmh_packed_estimate(wmh_ctx *ctx, const uint32_t *A, const uint32_t *B,
                               uint64_t n_pairs, uint32_t k, uint32_t bits, uint32_t *count,
                               double *jhat, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    wmh_status st = check_shape(ctx, k, bits);
    if (st != WMH_OK) return st;
    if (n_pairs == 0) return WMH_OK;
    if (!A || !B || (!count && !jhat)) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = pick(ctx, stream);
    hipError_t e = launch_packed_estimate(A, B, n_pairs, k, bits, count, jhat, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? WMH_OK : device_fail(ctx, e, "packed estimate");
}

}  // extern "C"
