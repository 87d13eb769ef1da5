// C-ABI of the fixed-point scaling step (Sec. 4, Practical Issues): the scale choice (host) and
// the quantization of real values on the device (kernel in wmh_quantize.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/wmh.h"
#include "wmh_context.h"
#include "wmh_internal.h"

using namespace wmh;

namespace {

// sum_i ceil(alpha * m_i), or -1 when some ceil(alpha * m_i) exceeds limit
double scaled_total(const double *m, uint32_t D, double alpha, double limit)
{
    double total = 0;
    for (uint32_t i = 0; i < D; ++i) {
        const double c = std::ceil(alpha * m[i]);
        if (c > limit) return -1.0;
        total += c;
    }
    return total;
}

}  // namespace

extern "C" {

wmh_status wmh_choose_scale(const double *m, uint32_t D, uint32_t limit, uint32_t components,
                            uint32_t steps, double *alpha_out, double *efficiency,
                            uint32_t *m_q)
{
    if (!m || D == 0 || !alpha_out) return WMH_E_ARG;
    const double lim = limit ? (double)limit : 4294967295.0;
    double top = 0, sum = 0;
    for (uint32_t i = 0; i < D; ++i) {
        if (!(m[i] >= 0) || !std::isfinite(m[i])) return WMH_E_ARG;
        top = std::max(top, m[i]);
        sum += m[i];
    }
    if (top <= 0) return WMH_E_OVERFLOW;
    // the largest scale that keeps every bound within the limit
    double amax = lim / top;
    while (scaled_total(m, D, amax, lim) < 0) amax = std::nextafter(amax, 0.0);
    double best = amax, best_g = amax / scaled_total(m, D, amax, lim);
    // g = alpha / sum ceil(alpha m_i) peaks where alpha * m_i is an integer: try the
    // breakpoints n / m_i just below amax for the components with the largest bounds
    std::vector<uint32_t> order(D);
    for (uint32_t i = 0; i < D; ++i) order[i] = i;
    const uint32_t C = std::min(D, components ? components : 8u);
    std::partial_sort(order.begin(), order.begin() + C, order.end(),
                      [&](uint32_t a, uint32_t b) { return m[a] > m[b]; });
    const uint32_t T = steps ? steps : 8u;
    for (uint32_t c = 0; c < C; ++c) {
        const double mi = m[order[c]];
        if (mi <= 0) continue;
        const double n0 = std::floor(amax * mi);
        for (uint32_t t = 0; t < T && n0 - t >= 1; ++t) {
            // one ulp below n / m_i, so that rounding of alpha * m_i cannot push it past n
            const double a = std::nextafter((n0 - t) / mi, 0.0);
            if (a <= 0 || a > amax) continue;
            const double s = scaled_total(m, D, a, lim);
            if (s <= 0) continue;
            if (a / s > best_g) {
                best_g = a / s;
                best = a;
            }
        }
    }
    *alpha_out = best;
    if (efficiency) *efficiency = best_g * sum;  // alpha * sum(m) / sum(ceil(alpha m)) <= 1
    if (m_q)
        for (uint32_t i = 0; i < D; ++i) m_q[i] = (uint32_t)std::ceil(best * m[i]);
    return WMH_OK;
}

wmh_status wmh_quantize(wmh_ctx *ctx, const float *x, const uint32_t *col, uint64_t nnz,
                        double alpha, uint32_t *out, uint64_t *n_clipped, void *stream)
{
    if (!ctx) return WMH_E_ARG;
    ctx->last_error.clear();
    if (!ctx->has_bounds) return fail(ctx, WMH_E_NO_BOUNDS, "wmh_set_bounds was not called");
    if (!(alpha > 0) || !std::isfinite(alpha)) return fail(ctx, WMH_E_ARG, "alpha must be > 0");
    if (nnz && (!x || !col || !out)) return fail(ctx, WMH_E_ARG, "null buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, WMH_E_DEVICE, "hipSetDevice");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->own_stream;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->d_codec), 0u, 2, s);
    if (e == hipSuccess)
        e = launch_quantize(x, nnz, col, ctx->d_bound, ctx->dims, alpha, out, ctx->d_codec, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_codec, ctx->d_codec, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(ctx, e, "quantize");
    if (n_clipped) *n_clipped = ctx->h_codec[0];
    return WMH_OK;
}

}  // extern "C"
