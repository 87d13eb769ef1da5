// Device primitives of the hash walk: the counter-based position sequence, the bounded draw and
// the position-to-component lookup.  gfx950 only.
//
// Position of step t (t >= 1) of hash j: Philox4x32-10 (Salmon et al., SC'11) under key
// (seed lo, seed hi) at counter ((t-1)/2, j, a, 0) gives 128 bits; odd steps take the low 64,
// even steps the high 64; the 64-bit word u becomes p = floor(u * M / 2^64) when the low half
// of u * M is at least 2^64 mod M (Lemire's exactly uniform bounded draw), else the step
// redraws from attempt a + 1.  This is the paper's consistent sequence of uniform positions on
// [0, M) (Algorithm 3 and the consistency paragraph after Definition 1), in integers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wmh {

constexpr uint32_t kCap = 65535u;  // largest hash value
constexpr uint32_t kWave = 64u;    // CDNA wavefront width

// Read-only view of the bounds tables (device memory).
struct Bounds {
    const uint64_t *prefix;   // P[0..D], P[0] = 0
    const uint32_t *bucket;   // T[0..n_buckets]: T[b] = max{i < D : P[i] <= b << shift}
    const uint32_t *bound;    // m[0..D)
    uint64_t total;           // M = P[D]
    uint64_t threshold;       // 2^64 mod M
    uint32_t shift;           // bucket width = 2^shift positions
    uint32_t dims;            // D
};

__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)kMul0 * c0;
        const uint64_t b = (uint64_t)kMul1 * c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Bounded draw: returns true and sets *p when the word is accepted.
__device__ __forceinline__ bool bounded_draw(uint64_t u, uint64_t total, uint64_t threshold,
                                             uint64_t *p)
{
    const uint64_t low = u * total;
    if (low < threshold) return false;
    *p = __umul64hi(u, total);
    return true;
}

// Full position of step t of hash j (every attempt); used where a lane draws for itself.
__device__ __forceinline__ uint64_t position(uint64_t seed, uint32_t j, uint32_t t,
                                             uint64_t total, uint64_t threshold)
{
    const uint32_t pair = (t - 1u) >> 1;
    const bool high = ((t - 1u) & 1u) != 0;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t attempt = 0;; ++attempt) {
        const uint4 w = philox4x32_10(pair, j, attempt, 0u, k0, k1);
        const uint64_t u = high ? (((uint64_t)w.w << 32) | w.z) : (((uint64_t)w.y << 32) | w.x);
        uint64_t p;
        if (bounded_draw(u, total, threshold, &p)) return p;
    }
}

// Redraw path of one half of a pair once its first-attempt word was rejected.
__device__ __noinline__ uint64_t redraw(uint64_t seed, uint32_t j, uint32_t pair, bool high,
                                        uint64_t total, uint64_t threshold)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t attempt = 1;; ++attempt) {
        const uint4 w = philox4x32_10(pair, j, attempt, 0u, k0, k1);
        const uint64_t u = high ? (((uint64_t)w.w << 32) | w.z) : (((uint64_t)w.y << 32) | w.x);
        uint64_t p;
        if (bounded_draw(u, total, threshold, &p)) return p;
    }
}

// Both positions of a pair of steps (2*pair + 1, 2*pair + 2) from one Philox block.
__device__ __forceinline__ void position_pair(uint64_t seed, uint32_t j, uint32_t pair,
                                              uint64_t total, uint64_t threshold, uint64_t *p_odd,
                                              uint64_t *p_even)
{
    const uint4 w = philox4x32_10(pair, j, 0u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u0 = ((uint64_t)w.y << 32) | w.x;
    const uint64_t u1 = ((uint64_t)w.w << 32) | w.z;
    if (!bounded_draw(u0, total, threshold, p_odd))
        *p_odd = redraw(seed, j, pair, false, total, threshold);
    if (!bounded_draw(u1, total, threshold, p_even))
        *p_even = redraw(seed, j, pair, true, total, threshold);
}

// Component of position p: c = max{i : P[i] <= p}, found in [T[b], T[b+1]] for b = p >> shift
// (the uniform bucket table replaces Algorithm 4's one-entry-per-integer map, whose size would
// be M).  Returns c and sets *offset = p - P[c].
template <typename PrefixPtr, typename BucketPtr>
__device__ __forceinline__ uint32_t component_of(uint64_t p, PrefixPtr prefix, BucketPtr bucket,
                                                 uint32_t shift, uint64_t *offset)
{
    const uint64_t b = p >> shift;
    uint32_t lo = bucket[b];
    uint32_t hi = bucket[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (prefix[mid] <= p) lo = mid;
        else hi = mid - 1u;
    }
    *offset = p - prefix[lo];
    return lo;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

}  // namespace wmh
