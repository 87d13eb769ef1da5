// (K, L) banding over signatures: the LSH index that consumes weighted minwise hashes (the
// paper's introduction names sublinear search through LSH as the main use of the k hashes).
// Band b of a signature is its values at hash ids [b*K, (b+1)*K); a database row is a
// candidate for a query when at least one band is equal value for value.  A pair whose hashes
// collide independently with probability J becomes a candidate with probability
// 1 - (1 - J^K)^L.
//
// Build: every band's K values are copied out (so the index owns them) and mixed into a 64-bit
// key; each band has an open-addressing table of keys (linear probing, atomicCAS) whose slots
// head a chain of the rows with that key (atomicExch on the head, one next pointer per row).
// Query: one wavefront per query; lane b < L takes band b, probes its table and walks the
// chain, keeping rows whose band equals the query's exactly (a key match alone is not enough);
// the wavefront then sorts its candidates in LDS and writes the distinct rows in increasing
// order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "wmh_internal.h"

namespace wmh {

namespace {

constexpr unsigned long long kEmpty = ~0ull;
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1u); }

// 64-bit mix of K values (FNV-1a over the 16-bit values, then a SplitMix64 finalizer); the
// value kEmpty is moved to kEmpty - 1 so that it can mark free slots.
__device__ __forceinline__ unsigned long long band_key(const uint16_t *v, uint32_t K)
{
    unsigned long long h = 0xCBF29CE484222325ull;
    for (uint32_t i = 0; i < K; ++i) {
        h ^= v[i];
        h *= 0x100000001B3ull;
    }
    h ^= h >> 30;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 27;
    h *= 0x94D049BB133111EBull;
    h ^= h >> 31;
    return h == kEmpty ? kEmpty - 1 : h;
}

// Thread per (band, row): copy the band's values, then insert the row.
__global__ __launch_bounds__(256) void lsh_insert_kernel(const uint16_t *__restrict__ sig,
                                                         uint64_t n, uint32_t k, uint32_t K,
                                                         uint32_t L, uint32_t cap_log2,
                                                         uint16_t *__restrict__ bands,
                                                         unsigned long long *table_key,
                                                         uint32_t *table_head,
                                                         uint32_t *__restrict__ next)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * L) return;
    const uint32_t b = (uint32_t)(idx / n);
    const uint64_t row = idx - (uint64_t)b * n;
    const uint16_t *src = sig + row * k + (uint64_t)b * K;
    uint16_t *dst = bands + ((uint64_t)b * n + row) * K;
    for (uint32_t i = 0; i < K; ++i) dst[i] = src[i];
    const unsigned long long key = band_key(src, K);
    const uint64_t cap = 1ull << cap_log2;
    unsigned long long *keys = table_key + (uint64_t)b * cap;
    uint64_t slot = key & (cap - 1);
    while (true) {
        const unsigned long long prev = atomicCAS(&keys[slot], kEmpty, key);
        if (prev == kEmpty || prev == key) break;
        slot = (slot + 1) & (cap - 1);
    }
    next[(uint64_t)b * n + row] = atomicExch(&table_head[(uint64_t)b * cap + slot], (uint32_t)row);
}

// One wavefront per query.  out_count[q] = number of distinct candidate rows, or kNoRow when
// the query's raw matches (counted once per band) exceed the wavefront's buffer.
__global__ __launch_bounds__(256) void lsh_query_kernel(const uint16_t *__restrict__ query,
                                                        uint64_t nq, uint32_t k, uint32_t K,
                                                        uint32_t L, uint64_t n,
                                                        uint32_t cap_log2,
                                                        const uint16_t *__restrict__ bands,
                                                        const unsigned long long *__restrict__ table_key,
                                                        const uint32_t *__restrict__ table_head,
                                                        const uint32_t *__restrict__ next,
                                                        uint32_t max_out, uint32_t *__restrict__ out,
                                                        uint32_t *__restrict__ out_count)
{
    constexpr uint32_t kBuf = kLshQueryBuffer;
    extern __shared__ uint32_t smem_lsh[];
    __shared__ uint32_t fill[256 / kWave];
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t *buf = smem_lsh + wave * kBuf;
    const uint64_t cap = 1ull << cap_log2;
    for (uint64_t q = (uint64_t)blockIdx.x * waves + wave; q < nq; q += (uint64_t)gridDim.x * waves) {
        if (lane() == 0) fill[wave] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint16_t *qv = query + q * k;
        for (uint32_t b = lane(); b < L; b += kWave) {
            const uint16_t *qb = qv + (uint64_t)b * K;
            const unsigned long long key = band_key(qb, K);
            const unsigned long long *keys = table_key + (uint64_t)b * cap;
            uint64_t slot = key & (cap - 1);
            uint32_t row = kNoRow;
            while (true) {
                const unsigned long long have = keys[slot];
                if (have == key) {
                    row = table_head[(uint64_t)b * cap + slot];
                    break;
                }
                if (have == kEmpty) break;
                slot = (slot + 1) & (cap - 1);
            }
            for (; row != kNoRow; row = next[(uint64_t)b * n + row]) {
                const uint16_t *rb = bands + ((uint64_t)b * n + row) * K;
                bool same = true;
                for (uint32_t i = 0; i < K && same; ++i) same = rb[i] == qb[i];
                if (!same) continue;
                const uint32_t at = atomicAdd(&fill[wave], 1u);
                if (at < kBuf) buf[at] = row;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t m = __builtin_amdgcn_readfirstlane(fill[wave]);
        if (m > kBuf) {
            if (lane() == 0) out_count[q] = kNoRow;
            continue;
        }
        // bitonic sort of the m candidates (padded with kNoRow to a power of two)
        uint32_t size = 1;
        while (size < m) size <<= 1;
        for (uint32_t i = m + lane(); i < size; i += kWave) buf[i] = kNoRow;
        for (uint32_t span = 2; span <= size; span <<= 1) {
            for (uint32_t stride = span >> 1; stride > 0; stride >>= 1) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (uint32_t i = lane(); i < size; i += kWave) {
                    const uint32_t partner = i ^ stride;
                    if (partner > i) {
                        const bool ascending = (i & span) == 0;
                        const uint32_t x = buf[i], y = buf[partner];
                        if ((x > y) == ascending) {
                            buf[i] = y;
                            buf[partner] = x;
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // distinct rows in order: position of each first occurrence = number of firsts before it
        uint32_t written = 0;
        for (uint32_t i0 = 0; i0 < m; i0 += kWave) {
            const uint32_t i = i0 + lane();
            const bool first = i < m && (i == 0 || buf[i] != buf[i - 1]);
            const uint64_t firsts = __ballot(first);
            const uint32_t rank = written + __builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(firsts >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)firsts, 0u));
            if (first && rank < max_out) out[q * max_out + rank] = buf[i];
            written += (uint32_t)__builtin_popcountll(firsts);
        }
        if (lane() == 0) out_count[q] = written;
    }
}

}  // namespace

hipError_t launch_lsh_build(const uint16_t *sig, uint64_t n, uint32_t k, uint32_t K, uint32_t L,
                            uint32_t cap_log2, uint16_t *bands, unsigned long long *table_key,
                            uint32_t *table_head, uint32_t *next, hipStream_t stream)
{
    const uint64_t cap = 1ull << cap_log2;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(table_key), 0xFFFFFFFFu,
                                   2 * cap * L, stream);
    if (e == hipSuccess) e = launch_fill_u32(table_head, kNoRow, cap * L, stream);
    if (e != hipSuccess || n == 0) return e;
    const uint64_t threads = n * L;
    lsh_insert_kernel<<<(uint32_t)((threads + 255) / 256), 256, 0, stream>>>(
        sig, n, k, K, L, cap_log2, bands, table_key, table_head, next);
    return hipGetLastError();
}

hipError_t launch_lsh_query(const uint16_t *query, uint64_t nq, uint32_t k, uint32_t K, uint32_t L,
                            uint64_t n, uint32_t cap_log2, const uint16_t *bands,
                            const unsigned long long *table_key, const uint32_t *table_head,
                            const uint32_t *next, uint32_t max_out, uint32_t *out,
                            uint32_t *out_count, hipStream_t stream)
{
    if (nq == 0) return hipSuccess;
    const uint32_t waves = 4;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((nq + waves - 1) / waves, 65536);
    lsh_query_kernel<<<grid, waves * kWave, (size_t)waves * kLshQueryBuffer * sizeof(uint32_t), stream>>>(
        query, nq, k, K, L, n, cap_log2, bands, table_key, table_head, next, max_out, out, out_count);
    return hipGetLastError();
}

}  // namespace wmh
