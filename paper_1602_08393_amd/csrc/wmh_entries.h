// What the batched walks share: the layout of a block's dense rows in LDS and the entries of
// the shared position stream.  Entry j * depth + t - 1 holds step t of hash j: wide entries
// are (component c, offset) pairs of 32-bit words; packed entries are one word,
// (offset << 16) | (c * scale), where c * scale is the LDS byte offset of component c's group
// of dense-row values (scale = RowLayout::kGroup); coarse entries replace the offset by its
// 16-bit code (see below) for rows held as 16-bit value codes.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wmh_device.h"

namespace wmh {

// LDS layout of the R dense rows of a block (D components each): the value of component c of
// row r sits at byte c * kGroup + row_byte(r).  Four rows of 16-bit values form two planes of
// row pairs (rows 0 and 1, then rows 2 and 3), one 4-byte word per component: the 32 lanes of
// one half-wavefront serve one row pair, so the components they read spread over all 32 banks
// (with 8-byte groups they would fall on every other bank).  Other blocks keep one group of R
// values per component.  The host's stream scale is kGroup.
template <typename XT, int R>
struct RowLayout {
    static constexpr bool kPlanes = R == 4 && sizeof(XT) == 2;
    static constexpr uint32_t kGroup = kPlanes ? 4u : R * (uint32_t)sizeof(XT);
    __device__ static uint32_t row_byte(uint32_t r, uint32_t dims)
    {
        if constexpr (kPlanes) return (r & 1u) * 2u + (r >> 1) * dims * 4u;
        else return r * (uint32_t)sizeof(XT);
    }
    __device__ static XT *at(unsigned char *base, uint32_t c, uint32_t r, uint32_t dims)
    {
        return reinterpret_cast<XT *>(base + (size_t)c * kGroup + row_byte(r, dims));
    }
};

// Coarse 16-bit codes for pieces whose bounds do not fit 16 bits.  With B code bits (B <= 15;
// 15 by default), in a piece of size m >= 1, q(y) = floor(y * 2^B / m) is nondecreasing on
// 0 <= y <= m, so for an offset o < m and a value x <= m: q(o) < q(x) gives o < x (green) and
// q(o) > q(x) gives o > x (red).  When q(o) = q(x), o < x is possible only if x is not the
// smallest y with that code, i.e. when q(x - 1) = q(x), i.e. when the remainder
// x * 2^B - q(x) * m is at least 2^B.  A stream entry carries the odd code v = 2 q(o) + 1 and
// the dense row the value code
//   z = 0 (x = 0), 0xFFFF (x >= m), else 2 q(x) + [x * 2^B - q(x) * m >= 2^B],
// so that v < z means green, v > z red, and v = z a tie, settled from the row's exact value and
// the step's exact offset (the walks test a window with a tie again with in-lane draws).  For
// m <= 2^B the map q is one-to-one and no tie occurs; above, a tested step in the row's support
// ties with probability below 2^-B (fewer bits make ties frequent, which tests use).
constexpr uint32_t kCoarseBits = 15u;

// floor(y * 2^B / m) and its remainder, for y <= m, 1 <= m, B <= 15: a float estimate (within
// one of the quotient) made exact by the remainder.
__device__ __forceinline__ uint32_t coarse_q(uint32_t y, uint32_t m, uint32_t bits, uint32_t *rem)
{
    const float est = (float)y * ((float)(1u << bits) * __builtin_amdgcn_rcpf((float)m));
    uint32_t q = (uint32_t)est;
    int64_t r = (int64_t)((uint64_t)y << bits) - (int64_t)q * (int64_t)m;
    while (r < 0) {
        --q;
        r += m;
    }
    while (r >= (int64_t)m) {
        ++q;
        r -= m;
    }
    *rem = (uint32_t)r;
    return q;
}

// The code of an offset o < m of a step (odd, at most 2^(B+1) - 1).
__device__ __forceinline__ uint32_t coarse_offset_code(uint32_t o, uint32_t m, uint32_t bits)
{
    uint32_t rem;
    return 2u * coarse_q(o, m, bits, &rem) + 1u;
}

// The code of a row's value x in a piece of size m.
__device__ __forceinline__ uint32_t coarse_value_code(uint32_t x, uint32_t m, uint32_t bits)
{
    if (x == 0) return 0u;
    if (x >= m) return 0xFFFFu;
    uint32_t rem;
    const uint32_t q = coarse_q(x, m, bits, &rem);
    return 2u * q + (rem >= (1u << bits) ? 1u : 0u);
}

// The exact value of component c in CSR row `row` (columns strictly increasing), 0 if absent.
__device__ __forceinline__ uint32_t csr_value(const uint64_t *row_ptr, const uint32_t *col,
                                              const uint32_t *val, uint64_t row, uint32_t c)
{
    uint64_t lo = row_ptr[row];
    const uint64_t end = row_ptr[row + 1];
    uint64_t hi = end;
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && col[lo] == c ? val[lo] : 0u;
}

// The next tile of a workgroup (called by one thread, `claimed` starting false): from the
// counter of a persistent launch, or, with no counter, the workgroup's own tile (blockIdx.x) the
// first time and none after it (one workgroup per tile; ~0 is past every tile).
__device__ __forceinline__ uint64_t next_tile(unsigned long long *counter, bool &claimed)
{
    if (counter) return atomicAdd(counter, 1ull);
    const uint64_t t = claimed ? ~0ull : (uint64_t)blockIdx.x;
    claimed = true;
    return t;
}

// K consecutive shared-stream entries of one lane (4-byte packed or 8-byte wide), read with the
// widest aligned loads: the first entry index is a multiple of K.
template <int K, bool kPacked>
struct EntryRun {
    static constexpr int kWordsPerEntry = kPacked ? 1 : 2;
    static constexpr int kWords = K * kWordsPerEntry;
    uint32_t w[kWords];

    // the run starting `lane_word` words after a (wave-uniform) window start
    __device__ __forceinline__ void load_at(const uint32_t *window, uint32_t lane_word)
    {
        load(window + lane_word, 0);
    }

    __device__ __forceinline__ void load(const void *entries, uint64_t index)
    {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(entries) + index * (kPacked ? 1 : 2);
        if constexpr (kWords == 1) {
            w[0] = p[0];
        } else if constexpr (kWords == 2) {
            const uint2 q = *reinterpret_cast<const uint2 *>(p);
            w[0] = q.x;
            w[1] = q.y;
        } else {
#pragma unroll
            for (int i = 0; i < kWords / 4; ++i) {
                const uint4 q = reinterpret_cast<const uint4 *>(p)[i];
                w[4 * i] = q.x;
                w[4 * i + 1] = q.y;
                w[4 * i + 2] = q.z;
                w[4 * i + 3] = q.w;
            }
        }
    }
    // LDS byte offset of the step's component group (c * scale) and the offset in the piece
    __device__ __forceinline__ void get(int k, uint32_t scale, uint32_t *lds, uint32_t *off) const
    {
        if (kPacked) {
            *lds = w[k] & 0xFFFFu;
            *off = w[k] >> 16;
        } else {
            *lds = w[2 * k] * scale;
            *off = w[2 * k + 1];
        }
    }
};

}  // namespace wmh
