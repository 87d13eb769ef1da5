// The component index: the capped position sequence filed by component, an exact second
// evaluation order of the hash for sparse green regions.
//
// Hash j of x is the first step t <= 65534 whose position is green for x, else 65535
// (Algorithm 3, Definition 1, with the walk capped).  A position is green exactly when it falls
// in a piece c with x_c > 0 and its offset inside the piece is below x_c (Sec. 3.1).  Filing
// every draw (j, t <= 65534) under its component c as the key (offset << 32) | (t << 16) | j,
// hash j of x is the smallest t over the keys of x's nonzero components whose offset is below
// x_c, and 65535 when there is none.  The keys of a component are sorted in chunks of
// kChunk, so a row reads only the green keys of its pieces plus one key per chunk: the work
// per row is about nnz + k * 65534 * s (s = sum(x) / M) instead of the walk's
// k * min(1/s, 65535), which wins by orders of magnitude when s is small (Theorem 2 gives the
// walk's 1/s; Sec. 4 discusses the small-s regime).  Both orders compute the same values.
//
// Build, once per (bounds, seed, k): count draws per component, round each count up to whole
// 128-byte lines of keys, exclusive scan, fill the buffer with ~0 keys (red in both orders),
// draw again and scatter the keys, sort each chunk (a wavefront per list of at most 64 keys, a
// workgroup in LDS for longer chunks; the ~0 pads sort last).  A row reads each of its lists
// from the list's start, so aligned starts save the partly used first line of every read.  The order in which draws land in a list varies between builds, so
// which keys share a chunk of a list longer than kChunk may vary too: that changes the cost of
// reading the list, never a hash value.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "wmh_internal.h"

namespace wmh {

namespace {

constexpr uint32_t kIndexPairs = (kCap - 1u) / 2u;  // pairs of steps (1,2) ... (65533,65534)
constexpr uint32_t kChunk = 4096;                   // keys sorted together (32 KB of LDS)
constexpr uint32_t kBatch = 16;      // most keys a lane loads per round trip (long lists)
constexpr uint32_t kShortBatch = 8;  // keys per round trip where lists are short
constexpr uint32_t kScanBlock = 1024;

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1u); }

__device__ __forceinline__ uint32_t wave_index()
{
    return (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Every lane's LDS operations before this point are visible to the wave's later ones (LDS
// executes one wavefront's instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass 1 and pass 2 of the build: one thread per (j, pair of steps).  Pass 1 counts the draws
// of each component; pass 2 claims a slot in the component's list and writes the key.
template <bool kScatter>
__global__ __launch_bounds__(256) void index_draw_kernel(Bounds b, uint64_t seed, uint32_t k,
                                                         uint32_t *__restrict__ counter,
                                                         uint64_t *__restrict__ entries)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)kIndexPairs * k) return;
    const uint32_t j = (uint32_t)(idx / kIndexPairs);
    const uint32_t pair = (uint32_t)(idx - (uint64_t)j * kIndexPairs);
    uint64_t p[2];
    position_pair(seed, j, pair, b.total, b.threshold, &p[0], &p[1]);
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
        uint64_t off;
        const uint32_t c = component_of(p[h], b.prefix, b.bucket, b.shift, &off);
        const uint32_t at = atomicAdd(&counter[c], 1u);
        if (kScatter) {
            const uint32_t t = 2u * pair + h + 1u;
            entries[at] = (off << 32) | ((uint64_t)t << 16) | j;
        }
    }
}

// Exclusive scan of n counts: per-block scans, then the block sums, then the carry added.
__global__ __launch_bounds__(kScanBlock) void scan_blocks_kernel(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out,
                                                                 uint32_t *__restrict__ block_sums,
                                                                 uint64_t n)
{
    __shared__ uint32_t s[kScanBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const uint32_t v = i < n ? in[i] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < kScanBlock; d <<= 1) {
        const uint32_t add = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

// One workgroup: exclusive scan of the block sums in place, chunk by chunk.
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(uint32_t *__restrict__ sums,
                                                               uint32_t n_blocks)
{
    __shared__ uint32_t s[kScanBlock];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n_blocks; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < n_blocks ? sums[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t d = 1; d < kScanBlock; d <<= 1) {
            const uint32_t add = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n_blocks) sums[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry += s[threadIdx.x];
        __syncthreads();
    }
}

// counts[i] rounded up to a multiple of align (a power of two), for i < n.
__global__ __launch_bounds__(256) void round_counts_kernel(uint32_t *__restrict__ counts,
                                                           uint64_t n, uint32_t align)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counts[i] = (counts[i] + align - 1u) & ~(align - 1u);
}

// offsets[i] += block carry; cursor[i] = offsets[i] (the scatter pass's claim counters).
__global__ __launch_bounds__(256) void scan_add_kernel(uint32_t *__restrict__ offsets,
                                                       uint32_t *__restrict__ cursor,
                                                       const uint32_t *__restrict__ block_sums,
                                                       uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = offsets[i] + block_sums[i / kScanBlock];
    offsets[i] = v;
    cursor[i] = v;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// Lists of 2..64 keys: one wavefront per list, bitonic sort across lanes (pads are ~0).
__global__ __launch_bounds__(256) void sort_small_kernel(const uint32_t *__restrict__ offsets,
                                                         uint32_t dims,
                                                         uint64_t *__restrict__ entries)
{
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t ln = lane();
    for (uint32_t c = blockIdx.x * waves + wave_index(); c < dims; c += gridDim.x * waves) {
        const uint32_t a = offsets[c];
        const uint32_t n = offsets[c + 1] - a;
        if (n < 2 || n > kWave) continue;  // uniform across the wavefront
        uint64_t v = ln < n ? entries[a + ln] : ~0ull;
#pragma unroll
        for (uint32_t size = 2; size <= kWave; size <<= 1) {
#pragma unroll
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                const uint64_t o = __shfl_xor(v, (int)stride);
                const bool ascending = (ln & size) == 0;
                const bool lower = (ln & stride) == 0;
                v = lower == ascending ? umin64(v, o) : umax64(v, o);
            }
        }
        if (ln < n) entries[a + ln] = v;
    }
}

// Lists of more than 64 keys: one workgroup per list, each chunk of kChunk keys sorted in LDS.
__global__ __launch_bounds__(256) void sort_chunks_kernel(const uint32_t *__restrict__ offsets,
                                                          uint32_t dims,
                                                          uint64_t *__restrict__ entries)
{
    __shared__ uint64_t s[kChunk];
    for (uint32_t c = blockIdx.x; c < dims; c += gridDim.x) {
        const uint32_t a = offsets[c], z = offsets[c + 1];
        if (z - a <= kWave) continue;  // uniform across the workgroup
        for (uint32_t base = a; base < z; base += kChunk) {
            const uint32_t n = std::min(z - base, kChunk);
            uint32_t size = 2;
            while (size < n) size <<= 1;
            for (uint32_t i = threadIdx.x; i < size; i += blockDim.x)
                s[i] = i < n ? entries[base + i] : ~0ull;
            __syncthreads();
            for (uint32_t span = 2; span <= size; span <<= 1) {
                for (uint32_t stride = span >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) {
                        const uint32_t partner = i ^ stride;
                        if (partner > i) {
                            const bool ascending = (i & span) == 0;
                            const uint64_t x = s[i], y = s[partner];
                            if ((x > y) == ascending) {
                                s[i] = y;
                                s[partner] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) entries[base + i] = s[i];
            __syncthreads();
        }
    }
}

// The same draws keyed by step: (t << 48) | (j << 32) | offset, list by list in place of the
// offset-ordered copy (sorted afterwards with the same chunks).
__global__ __launch_bounds__(256) void step_keys_kernel(const uint64_t *__restrict__ by_offset,
                                                        uint64_t n, uint64_t *__restrict__ by_step)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = by_offset[i];
    const uint64_t t = (key >> 16) & 0xFFFFu, j = key & 0xFFFFu, off = key >> 32;
    by_step[i] = (t << 48) | (j << 32) | off;
}

// Hashes of rows from the index: one wavefront per row, the running minimum of each hash id in
// LDS.  A lane takes one nonzero (c, x_c) at a time.  Offset order: the lane reads c's keys
// chunk by chunk up to the first offset >= x_c (every green key).  Step order, for rows whose
// hashes are small: the lane reads c's keys up to the first step > T1, where every hash of the
// row is at most T1 with probability 1 - 1/16 (Theorem 2: Pr(h > T) = (1 - s)^T); a row left
// with a hash id above T1 is read again up to T2 (probability 1 - 1e-4), then in offset order,
// so the values are exact either way.  The row takes step order when T2 * sum(m_c) < 65534 *
// sum(x_c) over its nonzeros (keys read in one pass to T2: k * T2 * sum(m_c) / M, against
// k * 65534 * sum(x_c) / M in offset order).  The rule leaves rows at the margin in offset order
// on purpose: a row with few nonzeros waits for its longest list, and step-order lists are as
// long as their bounds m_c, offset-order ones only as x_c.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Keys i .. i + kBatch - 1 of a list buffer, two keys per 16-byte load (global loads need only
// 4-byte alignment; a key address is 8-byte aligned).
typedef uint32_t KeyPair __attribute__((ext_vector_type(4), aligned(8)));
static_assert(kBatch % 2 == 0 && kShortBatch % 2 == 0 && kShortBatch <= kBatch &&
                  kIndexPadKeys + 1 >= kBatch,
              "a batch that starts at a list's last key stays inside the padded buffer");

template <uint32_t B>
__device__ __forceinline__ void load_batch(const uint64_t *__restrict__ keys, uint32_t i,
                                           uint64_t (&key)[B])
{
    const KeyPair *p = reinterpret_cast<const KeyPair *>(keys + i);
#pragma unroll
    for (uint32_t v = 0; v < B / 2; ++v) {
        const KeyPair q = p[v];
        key[2 * v] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        key[2 * v + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
    }
}

template <uint32_t B>
__device__ __forceinline__ void offset_scan(const uint64_t *__restrict__ entries, uint32_t a,
                                            uint32_t z, uint32_t x, uint32_t *hmin)
{
    for (uint32_t base = a; base < z; base += kChunk) {
        const uint32_t end = std::min(z, base + kChunk);
        // B consecutive keys per round trip (keys past the chunk's end, in the next list
        // or in the buffer's padding, count as red); the chunk is sorted, so the first red key
        // ends it
        for (uint32_t i = base; i < end; i += B) {
            uint64_t key[B];
            load_batch(entries, i, key);
            bool all_green = true;
#pragma unroll
            for (uint32_t u = 0; u < B; ++u) {
                const bool green = i + u < end && (uint32_t)(key[u] >> 32) < x;
                if (green) atomicMin(&hmin[(uint32_t)key[u] & 0xFFFFu], ((uint32_t)key[u]) >> 16);
                all_green = all_green && green;
            }
            if (!all_green) break;
        }
    }
}

template <uint32_t B>
__device__ __forceinline__ void step_scan(const uint64_t *__restrict__ by_step, uint32_t a,
                                          uint32_t z, uint32_t x, uint32_t T, uint32_t *hmin)
{
    for (uint32_t base = a; base < z; base += kChunk) {
        const uint32_t end = std::min(z, base + kChunk);
        // keys in step order inside the chunk: read up to the first step > T
        for (uint32_t i = base; i < end; i += B) {
            uint64_t key[B];
            load_batch(by_step, i, key);
            bool all_in = true;
#pragma unroll
            for (uint32_t u = 0; u < B; ++u) {
                const uint32_t t = (uint32_t)(key[u] >> 48);
                const bool in = i + u < end && t <= T;
                if (in && (uint32_t)key[u] < x)
                    atomicMin(&hmin[(uint32_t)(key[u] >> 32) & 0xFFFFu], t);
                all_in = all_in && in;
            }
            if (!all_in) break;
        }
    }
}

template <bool kFiltered, uint32_t B>
__global__ __launch_bounds__(1024) void index_rows_kernel(Rows rows,
                                                         const uint32_t *__restrict__ offsets,
                                                         const uint64_t *__restrict__ entries,
                                                         const uint64_t *__restrict__ by_step,
                                                         const uint32_t *__restrict__ bound,
                                                         uint64_t total, uint32_t dims, uint32_t k,
                                                         double log_first, double log_final,
                                                         unsigned long long *row_counter,
                                                         bool claim_rows,
                                                         uint16_t *__restrict__ sig)
{
    extern __shared__ uint32_t lds[];
    const uint32_t wave = wave_index();
    const uint32_t ln = lane();
    uint32_t *hmin = lds + (size_t)wave * k;
    // In a large batch rows are claimed from a counter that starts at zero, so a wavefront that
    // drew cheap rows takes more of them (row costs differ by orders of magnitude): one row per
    // claim, or, under a row filter, 64 rows per claim, of which the wavefront picks the rows it keeps
    // with one ballot (claims on one counter are serialized, and most rows of a filtered batch
    // belong to the other path).  The next claim is sent before the current rows are read, so
    // its latency hides behind them.  (The counter's address is offset by a lane count that is
    // zero in lane 0: the compiler then sees a per-lane address and issues the one lane's
    // atomic as written, where for a uniform address it would combine the wavefront's requests
    // and wait for the result at once.)
    unsigned long long *const claim_at = row_counter + __builtin_amdgcn_mbcnt_lo(0u, 0u);
    constexpr unsigned long long group = kFiltered ? kWave : 1u;
    auto claim = [&]() {
        unsigned long long r = 0;
        if (ln == 0) r = atomicAdd(claim_at, group);
        return r;  // lane 0's value, read through a broadcast
    };
    auto hash_row = [&](uint64_t row) {
        for (uint32_t j = ln; j < k; j += kWave) hmin[j] = kCap;
        wave_lds_fence();
        const uint64_t lo = rows.row_ptr[row], hi = rows.row_ptr[row + 1];
        // the row's sum(x) and sum(m) over its nonzero columns
        uint64_t sx = 0, sm = 0;
        for (uint64_t e = lo + ln; e < hi; e += kWave) {
            const uint32_t c = rows.col[e];
            const uint32_t x = rows.val[e];
            if (x == 0 || c >= dims) continue;
            sx += x;
            sm += bound[c];
        }
        sx = wave_sum64(sx);
        sm = wave_sum64(sm);
        const bool live = sx != 0;
        // step bounds T1 <= T2 of the row and the cheaper key order (uniform over the wavefront).
        // Where lists are short a pass reads about one batch per nonzero whatever its bound, so
        // a first pass to T1 saves little and the second costs a whole pass: one pass to T2.
        constexpr bool kTwoPass = B == kBatch;
        uint32_t T1 = kCap, T2 = kCap;
        bool by_steps = false;
        if (live && by_step) {
            const double s = (double)sx / (double)total;
            const double t2 = index_step_bound(s, log_final);
            const double t1 = kTwoPass ? index_step_bound(s, log_first) : t2;
            T1 = t1 < (double)kCap ? (uint32_t)t1 : kCap;
            T2 = t2 < (double)kCap ? (uint32_t)t2 : kCap;
            by_steps = T2 < kCap - 1u && t2 * (double)sm < 65534.0 * (double)sx;
        }
        for (uint64_t e = lo + ln; e < hi; e += kWave) {
            const uint32_t c = rows.col[e];
            const uint32_t x = rows.val[e];
            if (x == 0 || c >= dims) continue;
            if (by_steps) step_scan<B>(by_step, offsets[c], offsets[c + 1], x, T1, hmin);
            else offset_scan<B>(entries, offsets[c], offsets[c + 1], x, hmin);
        }
        wave_lds_fence();
        // A hash id with no green step up to T1 after the first pass: read the row's lists again
        // up to T2, then, if one is still open, in offset order.  A minimum found by a pass that
        // read every key up to its bound is final, and each pass only lowers minima to green
        // steps, so the values are exact whichever passes run.
        auto any_open = [&](uint32_t T) {
            bool open = false;
            for (uint32_t j = ln; j < k; j += kWave) open = open || hmin[j] > T;
            return __ballot(open) != 0;
        };
        if (by_steps && any_open(T1)) {
            if (kTwoPass && T2 > T1) {
                for (uint64_t e = lo + ln; e < hi; e += kWave) {
                    const uint32_t c = rows.col[e];
                    const uint32_t x = rows.val[e];
                    if (x == 0 || c >= dims) continue;
                    step_scan<B>(by_step, offsets[c], offsets[c + 1], x, T2, hmin);
                }
                wave_lds_fence();
            }
            if (any_open(T2)) {
                for (uint64_t e = lo + ln; e < hi; e += kWave) {
                    const uint32_t c = rows.col[e];
                    const uint32_t x = rows.val[e];
                    if (x == 0 || c >= dims) continue;
                    offset_scan<B>(entries, offsets[c], offsets[c + 1], x, hmin);
                }
                wave_lds_fence();
            }
        }
        uint16_t *out = sig + row * (uint64_t)k;
        for (uint32_t j = ln; j < k; j += kWave)
            out[j] = live ? (uint16_t)hmin[j] : (uint16_t)0;
        wave_lds_fence();
    };
    if (!kFiltered && !claim_rows) {  // a small batch: every G-th row, G the grid's wavefronts
        const uint32_t waves = blockDim.x / kWave;
        for (uint64_t row = (uint64_t)blockIdx.x * waves + wave; row < rows.n_rows;
             row += (uint64_t)gridDim.x * waves)
            hash_row(row);
        return;
    }
    unsigned long long pending = claim();
    if constexpr (!kFiltered) {
        for (;;) {
            const uint64_t row = __shfl(pending, 0);
            if (row >= rows.n_rows) break;
            pending = claim();
            hash_row(row);
        }
    } else {
        for (;;) {
            const uint64_t first = __shfl(pending, 0);
            if (first >= rows.n_rows) break;
            pending = claim();
            // the claimed rows this path computes, one bit each (uniform over the wavefront)
            const uint64_t r = first + ln;
            uint64_t todo = __ballot(r < rows.n_rows && !rows.skips(r));
            while (todo != 0) {
                hash_row(first + (uint64_t)__builtin_ctzll(todo));
                todo &= todo - 1;
            }
        }
    }
}

}  // namespace

hipError_t launch_index_build(const Bounds &b, uint64_t seed, uint32_t k, const IndexBuffers &ix,
                              hipStream_t stream)
{
    const uint64_t D = b.dims;
    const uint64_t n_scan = D + 1;  // offsets[D] is the total
    const uint32_t n_blocks = (uint32_t)((n_scan + kScanBlock - 1) / kScanBlock);
    hipError_t e = launch_fill_u32(ix.cursor, 0u, n_scan, stream);
    if (e != hipSuccess) return e;
    const uint32_t align = ix.align;
    if (align != 1 && align != kIndexListAlign) return hipErrorInvalidValue;
    const uint64_t threads = (uint64_t)kIndexPairs * k;
    const uint32_t grid = (uint32_t)((threads + 255) / 256);
    index_draw_kernel<false><<<grid, 256, 0, stream>>>(b, seed, k, ix.cursor, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the buffer's keys: the lists (padded) and kIndexPadKeys past them, all ~0 until scattered
    const uint64_t capacity = index_padded_count(k, (uint32_t)D, align) + kIndexPadKeys;
    if (align > 1) {
        round_counts_kernel<<<(uint32_t)((D + 255) / 256), 256, 0, stream>>>(ix.cursor, D, align);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(ix.entries), 0xFFFFFFFFu, 2 * capacity,
                            stream);
        if (e != hipSuccess) return e;
    }
    scan_blocks_kernel<<<n_blocks, kScanBlock, 0, stream>>>(ix.cursor, ix.offsets, ix.block_sums,
                                                          n_scan);
    scan_sums_kernel<<<1, kScanBlock, 0, stream>>>(ix.block_sums, n_blocks);
    scan_add_kernel<<<(uint32_t)((n_scan + 255) / 256), 256, 0, stream>>>(ix.offsets, ix.cursor,
                                                                         ix.block_sums, n_scan);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    index_draw_kernel<true><<<grid, 256, 0, stream>>>(b, seed, k, ix.cursor, ix.entries);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint32_t sort_grid = (uint32_t)std::min<uint64_t>((D + 3) / 4, 16384);
    sort_small_kernel<<<sort_grid, 256, 0, stream>>>(ix.offsets, (uint32_t)D, ix.entries);
    sort_chunks_kernel<<<(uint32_t)std::min<uint64_t>(D, 4096), 256, 0, stream>>>(
        ix.offsets, (uint32_t)D, ix.entries);
    if ((e = hipGetLastError()) != hipSuccess || !ix.by_step) return e;
    // the step-ordered copy: the same lists and chunks, keys re-packed (a ~0 pad stays ~0),
    // then sorted
    const uint64_t n = align > 1 ? capacity : (uint64_t)kIndexPairs * 2u * k;
    step_keys_kernel<<<(uint32_t)((n + 255) / 256), 256, 0, stream>>>(ix.entries, n, ix.by_step);
    sort_small_kernel<<<sort_grid, 256, 0, stream>>>(ix.offsets, (uint32_t)D, ix.by_step);
    sort_chunks_kernel<<<(uint32_t)std::min<uint64_t>(D, 4096), 256, 0, stream>>>(
        ix.offsets, (uint32_t)D, ix.by_step);
    return hipGetLastError();
}

constexpr size_t kIndexRowsLdsMax = 64 * 1024;  // running minima of one workgroup

uint32_t index_rows_waves(uint32_t k, uint32_t waves)
{
    if (waves == 0) waves = k <= 2048 ? 4u : 1u;
    if (waves > kIndexMaxWaves || (size_t)waves * k * sizeof(uint32_t) > kIndexRowsLdsMax)
        return 0;
    return waves;
}

int index_rows_blocks_per_cu(uint32_t k, uint32_t waves_in)
{
    const uint32_t waves = index_rows_waves(k, waves_in);
    if (waves == 0) return 1;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, index_rows_kernel<false, kBatch>,
                                                     waves * kWave,
                                                     (size_t)waves * k * sizeof(uint32_t)) !=
        hipSuccess)
        return 1;
    return std::max(1, n);
}

hipError_t launch_index_rows(const Rows &rows, const IndexBuffers &ix, const Bounds &b, uint32_t k,
                             uint16_t *sig, unsigned long long *row_counter, uint32_t grid,
                             hipStream_t stream, const IndexPlan &plan)
{
    if (rows.n_rows == 0) return hipSuccess;
    const uint32_t waves = index_rows_waves(k, plan.waves);
    if (waves == 0 || (plan.batch != 0 && plan.batch != kBatch && plan.batch != kShortBatch) ||
        plan.claim > 2)
        return hipErrorInvalidValue;
    const uint64_t need = (rows.n_rows + waves - 1) / waves;
    const uint32_t g = (uint32_t)std::min<uint64_t>(need, grid);
    // every hash of a step-order row is <= T1 with probability >= 1 - 1/16, <= T2 with >= 1 - 1e-4
    const double log_first = std::log(kIndexFirstMiss / (double)k);
    const double log_final = std::log(kIndexFinalMiss / (double)k);
    // Long lists (text-like: ~1000 keys each) read 16 keys per trip, short ones (~16 keys, as
    // for D = 2^20 and k = 256) 8; large batches hand out rows from a counter, small ones (a
    // serving request) by a fixed stride, which measured faster there.
    const bool long_lists = plan.batch ? plan.batch == kBatch
                                       : (double)k * kIndexSteps / (double)b.dims >= 64.0;
    const bool claim_rows = plan.claim ? plan.claim == 1 : rows.n_rows >= 16ull * g * waves;
    if (claim_rows || rows.row_class) {
        const hipError_t e =
            launch_fill_u32(reinterpret_cast<uint32_t *>(row_counter), 0u, 2, stream);
        if (e != hipSuccess) return e;
    }
    // a filtered launch claims rows 64 at a time: one wavefront takes at most every 64th row
    const uint64_t need_filtered = (rows.n_rows + kWave * waves - 1) / (kWave * waves);
    const uint32_t gf = (uint32_t)std::min<uint64_t>(need_filtered, g);
    const size_t lds = (size_t)waves * k * sizeof(uint32_t);
    const uint32_t threads = waves * kWave;
#define WMH_INDEX_ROWS(F, B, G)                                                                    \
    index_rows_kernel<F, B><<<G, threads, lds, stream>>>(rows, ix.offsets, ix.entries, ix.by_step, \
                                                         b.bound, b.total, b.dims, k, log_first,  \
                                                         log_final, row_counter, claim_rows, sig)
    if (rows.row_class) {
        if (long_lists) WMH_INDEX_ROWS(true, kBatch, gf);
        else WMH_INDEX_ROWS(true, kShortBatch, gf);
    } else {
        if (long_lists) WMH_INDEX_ROWS(false, kBatch, g);
        else WMH_INDEX_ROWS(false, kShortBatch, g);
    }
#undef WMH_INDEX_ROWS
    return hipGetLastError();
}

}  // namespace wmh
