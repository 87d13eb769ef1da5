// All-pairs collision counts for the estimator J_hat = collisions / k (eq. Estimator).
//
// counts[a * nb + b] = #{j : A[a, j] == B[b, j]}.  Equality of uint16 hashes is not a dot
// product, so this is VALU work, not MFMA: two hashes are packed per 32-bit word, xored, and
// the zero half-words counted with a carry-free test, two comparisons per few instructions.
// A workgroup owns a 64 x 64 block of pairs, stages both 64-row slices of a 64-hash chunk in
// LDS, and each thread accumulates a 4 x 4 register tile of pairs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wmh_internal.h"

namespace wmh {

namespace {

constexpr int kTile = 64;        // rows of A (and of B) per workgroup
constexpr int kChunk = 64;       // hashes per staged chunk
constexpr int kWords = kChunk / 2;
constexpr int kPitch = kWords + 1;  // LDS row pitch in words (odd: spreads banks)

// number of equal 16-bit halves of a and b
__device__ __forceinline__ uint32_t equal_halves(uint32_t a, uint32_t b)
{
    const uint32_t d = a ^ b;
    // high bit of each half set iff that half of d is zero
    const uint32_t z = ~(((d & 0x7FFF7FFFu) + 0x7FFF7FFFu) | d) & 0x80008000u;
    return __builtin_popcount(z);
}

__global__ __launch_bounds__(256) void collide_kernel(const uint16_t *__restrict__ A, uint64_t na,
                                                      const uint16_t *__restrict__ B, uint64_t nb,
                                                      uint32_t k, uint32_t *__restrict__ counts)
{
    __shared__ uint32_t sa[kTile * kPitch];
    __shared__ uint32_t sb[kTile * kPitch];
    const uint64_t a0 = (uint64_t)blockIdx.y * kTile;
    const uint64_t b0 = (uint64_t)blockIdx.x * kTile;
    const uint32_t tx = threadIdx.x & 15u, ty = threadIdx.x >> 4;
    uint32_t acc[4][4] = {};

    for (uint32_t j0 = 0; j0 < k; j0 += kChunk) {
        // stage: word w of row r holds hashes j0+2w, j0+2w+1; beyond k (or beyond the last
        // row) A pads with 0 and B with 1 so padding never counts as a collision
        for (uint32_t i = threadIdx.x; i < kTile * kWords; i += blockDim.x) {
            const uint32_t r = i / kWords, w = i - r * kWords;
            const uint32_t j = j0 + 2u * w;
            uint32_t va = 0u, vb = 0x00010001u;
            if (a0 + r < na) {
                const uint16_t *row = A + (a0 + r) * k;
                const uint32_t lo = j < k ? row[j] : 0u;
                const uint32_t hi = j + 1 < k ? row[j + 1] : 0u;
                va = lo | (hi << 16);
            }
            if (b0 + r < nb) {
                const uint16_t *row = B + (b0 + r) * k;
                const uint32_t lo = j < k ? row[j] : 1u;
                const uint32_t hi = j + 1 < k ? row[j + 1] : 1u;
                vb = lo | (hi << 16);
            }
            sa[r * kPitch + w] = va;
            sb[r * kPitch + w] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int w = 0; w < kWords; ++w) {
            uint32_t ra[4], rb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra[i] = sa[(ty + 16 * i) * kPitch + w];
                rb[i] = sb[(tx + 16 * i) * kPitch + w];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] += equal_halves(ra[i], rb[q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t a = a0 + ty + 16 * i;
        if (a >= na) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t b = b0 + tx + 16 * q;
            if (b < nb) counts[a * nb + b] = acc[i][q];
        }
    }
}

}  // namespace

hipError_t launch_collisions(const uint16_t *A, uint64_t na, const uint16_t *B, uint64_t nb,
                             uint32_t k, uint32_t *counts, hipStream_t stream)
{
    if (na == 0 || nb == 0) return hipSuccess;
    const uint64_t gx = (nb + kTile - 1) / kTile, gy = (na + kTile - 1) / kTile;
    if (gx > 0x7FFFFFFFull || gy > 65535ull) return hipErrorInvalidValue;
    dim3 grid((uint32_t)gx, (uint32_t)gy);
    collide_kernel<<<grid, 256, 0, stream>>>(A, na, B, nb, k, counts);
    return hipGetLastError();
}

}  // namespace wmh
