// Fixed-point scaling of real-valued data (Sec. 4, Practical Issues).  The walk needs integer
// bounds; real data is scaled by alpha and rounded: x_q = floor(alpha * x + 1/2), bounds
// m_q = ceil(alpha * m).  The expected step count is M / sum(x) (Theorem 2), so the scale
// should maximize alpha * sum(x) / sum(ceil(alpha * m_i)); sum(x) is a common factor, so the
// best scale depends on the bounds alone: g(alpha) = alpha / sum(ceil(alpha * m_i)).  Between
// two points where some alpha * m_i crosses an integer the denominator is constant and g rises,
// so the maxima sit where alpha * m_i is an integer for some i.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "wmh_internal.h"

namespace wmh {

namespace {

// One thread per value; products and sums in IEEE double, rounded separately (no fused
// multiply-add), so the host computes the same integers.
__global__ __launch_bounds__(256) void quantize_kernel(const float *__restrict__ x, uint64_t n,
                                                       const uint32_t *__restrict__ col,
                                                       const uint32_t *__restrict__ bound_q,
                                                       uint32_t dims, double alpha,
                                                       uint32_t *__restrict__ out,
                                                       unsigned long long *clipped)
{
    uint32_t mine = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double v = __dadd_rn(__dmul_rn(alpha, (double)x[i]), 0.5);
        const double q = floor(v > 0.0 ? v : 0.0);
        const uint32_t c = col[i];
        const uint32_t cap = c < dims ? bound_q[c] : 0u;
        uint32_t r = q >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)q;
        if (r > cap) {
            r = cap;
            ++mine;
        }
        out[i] = r;
    }
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if ((threadIdx.x & (kWave - 1u)) == 0 && mine) atomicAdd(clipped, (unsigned long long)mine);
}

}  // namespace

hipError_t launch_quantize(const float *x, uint64_t n, const uint32_t *col, const uint32_t *bound_q,
                           uint32_t dims, double alpha, uint32_t *out, unsigned long long *clipped,
                           hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 65536);
    quantize_kernel<<<grid, 256, 0, stream>>>(x, n, col, bound_q, dims, alpha, out, clipped);
    return hipGetLastError();
}

}  // namespace wmh
