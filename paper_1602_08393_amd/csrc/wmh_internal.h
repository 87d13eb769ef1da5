// Internal interface between the C-ABI host code (wmh_host.cpp) and the kernel launchers
// (wmh_kernels.hip, wmh_collide.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wmh_device.h"

namespace wmh {

// Validation verdict codes, ordered by entry: the code of a row is that of its first bad entry.
enum : uint32_t {
    kCheckRowPtr = 1,   // row_ptr[r] > row_ptr[r+1] or row_ptr[r+1] > nnz
    kCheckColumn = 2,   // col >= D
    kCheckUnsorted = 3, // col[e-1] >= col[e] inside a row
    kCheckBound = 4,    // val > m[col]
};

// Device words written by the validation kernel (one allocation, reset before each launch).
struct CheckWords {
    // minima, starting at ~0 (the first kCheckMinima words)
    unsigned long long first_error;      // (row << 4) | code, minimum over rows; ~0 when valid
    unsigned long long min_green;        // smallest sum(x) over non-empty rows; ~0 if none
    unsigned long long walk_min_green;   // row split: smallest sum(x) of the walk's rows
    // counters, starting at 0
    unsigned long long n_empty;          // rows with sum(x) == 0
    unsigned long long walk_steps;       // sum over non-empty rows of min(M / sum(x), 65535)
    unsigned long long index_keys;       // sum over non-empty rows of the index keys per hash
    unsigned long long walk_rows;        // row split: rows classed for the walk (empty ones too)
    unsigned long long walk_class_steps; // row split: their expected walk steps
    unsigned long long index_rows;       // row split: rows classed for the index
    unsigned long long index_nnz;        // row split: their nonzeros
    unsigned long long index_class_keys; // row split: their index keys per hash
};
constexpr uint32_t kCheckMinima = 3;

// Row split: the validation pass writes row_class[r] = 1 for rows whose estimated cost on the
// component index (k * keys * key_cost + nnz * nnz_cost) is below their walk's (k * steps, in
// units of one walk test), else 0.
struct RowSplit {
    uint8_t *row_class = nullptr;
    uint32_t k = 0;
    float key_cost = 0.f;
    float nnz_cost = 0.f;
};

struct Rows {
    const uint64_t *row_ptr;
    const uint32_t *col;
    const uint32_t *val;
    uint64_t n_rows;
    uint64_t nnz;
    // optional row filter: with row_class set, kernels that honour it (the shared-window and
    // ballot walks, the index rows) process only rows r with row_class[r] == keep and leave
    // the other rows' signatures untouched
    const uint8_t *row_class = nullptr;
    uint32_t keep = 0;
    __host__ __device__ bool skips(uint64_t r) const { return row_class && row_class[r] != keep; }
};

// One shared-stream entry: the component c and the offset inside it of one step's position.
// Wide entries are (c, offset) as two uint32; packed entries are (offset << 16) | (c * scale)
// with scale = R * sizeof(dense value), the LDS byte offset of component c's group of R dense
// values; used when every bound is below 65536 and D * scale <= 65536.  Coarse entries hold the
// offset's 16-bit coarse code in place of the offset (rows held as coarse value codes).
struct StreamEntry {
    uint32_t comp;
    uint32_t offset;
};

struct BatchedPlan {
    uint32_t rows_per_block;   // R
    uint32_t steps_per_lane;   // K: steps a lane tests per window (R, or 4 when R < 4)
    uint32_t hashes_per_tile;  // J
    uint32_t stream_depth;     // T0: 0 (every draw in-lane) or whole cycles of three windows
                               // (a window is 64 / R * K steps), below the cap
    uint32_t waves_per_block;
    bool narrow;               // dense rows stored as uint16: the values (every bound < 65536)
                               // or, with coarse, their coarse codes
    bool packed;               // 4-byte stream entries
    bool coarse = false;       // rows hold coarse value codes, the stream coarse offset codes,
                               // and ties are settled exactly (shared-window and ballot walks)
    uint32_t coarse_bits = 15; // resolution of the coarse codes (1..15)
    bool independent_rows;     // each row of a block walks its own hash ids (R = 4 only)
    bool ballot;               // one row per block, first green step from the window's ballot
                               // (R = 1, K = 1 only)
    uint32_t hash_groups = 1;  // ballot walk: hash ids in this many blocks of J ids, one tile
                               // counter each (1: a single counter over (row, block) tiles)
    // LDS bytes per component of the block's dense rows (RowLayout::kGroup): four rows of
    // 16-bit values sit in two planes of row pairs, 4 bytes per component
    uint32_t scale() const
    {
        return rows_per_block == 4 && narrow ? 4u : rows_per_block * (narrow ? 2u : 4u);
    }
    uint32_t window() const { return 64u / rows_per_block * steps_per_lane; }
    // the shared walk prefetches three windows ahead of the one it tests
    uint32_t cycle() const { return 3u * window(); }
    // stream of k hash ids, plus the three windows that the last id's prefetches read past it
    size_t stream_bytes(uint32_t k) const
    {
        return stream_depth ? ((size_t)stream_depth * k + cycle()) * (packed ? 4u : 8u) : 0u;
    }
};

// Checks the rows and gathers the statistics of CheckWords (M = total, for the cost estimates);
// index_keys only with want_keys (it is left at 0 otherwise).
// With split (want_keys must be set) it also classes every row and fills the per-class words.
// bound_blocks: the per-block minima and means of the bounds (bound_block_table), or nullptr.
hipError_t launch_validate(const Rows &rows, const uint32_t *bound, uint32_t dims, uint64_t total,
                           uint32_t k, bool want_keys, CheckWords *words, hipStream_t stream,
                           const RowSplit *split = nullptr,
                           const uint32_t *bound_blocks = nullptr);

// Components per block of the validation pass's block table, and whether a table is kept for
// D components: when m does not fit in the pass's LDS but the table (two words per block) does.
constexpr uint32_t kBoundBlock = 32;
constexpr size_t kValidateLdsMax = 76 * 1024;
inline bool bound_blocks_wanted(uint32_t dims)
{
    const uint64_t blocks = ((uint64_t)dims + kBoundBlock - 1) / kBoundBlock;
    return (uint64_t)dims * 4 > kValidateLdsMax && blocks * 8 <= kValidateLdsMax;
}

hipError_t launch_plain(const Bounds &b, const Rows &rows, uint64_t row_begin,
                        uint64_t row_end, uint32_t k, uint64_t seed, uint16_t *sig, bool narrow,
                        bool dense, hipStream_t stream);

hipError_t launch_draws(const Bounds &b, uint64_t seed, uint32_t j0, uint32_t n_hashes,
                        uint32_t depth, uint64_t *pos, uint32_t *comp, uint64_t *off,
                        hipStream_t stream);

// coarse_bits > 0: entries carry the offset's coarse code of that many bits (needs packed)
hipError_t launch_stream_build(const Bounds &b, uint64_t seed, uint32_t k, uint32_t depth,
                               bool packed, uint32_t scale, uint32_t coarse_bits, void *entries,
                               hipStream_t stream);

// Dynamic LDS a walk's workgroup may take: the CU's 160 KiB less room for the kernels' static
// LDS (tile slots and the wavefronts' claim words, under 512 bytes).
constexpr size_t kMaxDynamicLds = 160 * 1024 - 512;

// Tile counters a batched launch may use (one per hash group), u64 each, cleared before it.
constexpr uint32_t kMaxHashGroups = 8;

// Returns hipErrorInvalidValue when the plan does not fit (LDS).
hipError_t launch_batched(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                          uint16_t *sig, const BatchedPlan &plan, const void *entries,
                          unsigned long long *tile_counter, uint32_t grid, hipStream_t stream);

// Dynamic LDS bytes a batched plan needs.
size_t batched_lds_bytes(uint32_t dims, const BatchedPlan &plan);

// The shared-window walk (no checks: launch_batched validates the plan) and its occupancy.
hipError_t launch_shared_walk(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                              uint16_t *sig, const BatchedPlan &plan, const void *entries,
                              unsigned long long *tile_counter, uint32_t grid, hipStream_t stream);
int shared_walk_blocks_per_cu(const BatchedPlan &plan, size_t lds);

// The ballot walk (R = 1, K = 1; no checks) and its occupancy.
hipError_t launch_ballot_walk(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                              uint16_t *sig, const BatchedPlan &plan, const void *entries,
                              unsigned long long *tile_counter, uint32_t grid, hipStream_t stream);
int ballot_walk_blocks_per_cu(const BatchedPlan &plan, size_t lds);

// Resident workgroups per CU for a batched plan (0 when it does not fit).
int batched_blocks_per_cu(uint32_t dims, const BatchedPlan &plan);

hipError_t launch_estimate(const uint16_t *A, const uint16_t *B, uint64_t n_pairs, uint32_t k,
                           uint32_t *count, double *jhat, hipStream_t stream);

hipError_t launch_collisions(const uint16_t *A, uint64_t na, const uint16_t *B, uint64_t nb,
                             uint32_t k, uint32_t *counts, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t stream);
// Starting values of the validation pass's words (minima ~0, counters 0).
hipError_t launch_check_init(CheckWords *words, hipStream_t stream);

// Component index of the capped sequence (wmh_index.hip).  entries: the k * 65534 keys
// (offset << 32) | (t << 16) | j grouped by component (by_step: the same lists in step order),
// each list padded to a multiple of `align` keys with ~0 keys (red in both orders: offset
// 2^32 - 1, step 65535), so that with align = 16 every list starts on a 128-byte line;
// offsets: D + 1 list starts; cursor: D + 1 counters; block_sums: ceil((D + 1) / 1024) scan
// carries.
struct IndexBuffers {
    uint64_t *entries = nullptr;
    uint64_t *by_step = nullptr;  // the same lists keyed (t << 48) | (j << 32) | offset; optional
    uint32_t *offsets = nullptr;
    uint32_t *cursor = nullptr;
    uint32_t *block_sums = nullptr;
    uint32_t align = 1;  // keys per list are a multiple of this (1 or kIndexListAlign)
};

constexpr uint32_t kIndexSteps = 65534u;  // steps 1 .. cap - 1 decide every capped hash value
constexpr uint32_t kIndexMaxK = 8192u;    // j fits the key's 16 bits; LDS of the row kernel

// Step-order passes of the component index over a row with green fraction s (Theorem 2: one
// hash exceeds T with probability (1 - s)^T): a first pass reads every list up to T1, where all
// k hashes are <= T1 with probability >= 1 - kIndexFirstMiss; a row it leaves open is read again
// up to T2 (probability >= 1 - kIndexFinalMiss), and a row still open after that in offset order.
constexpr double kIndexFirstMiss = 1.0 / 16.0;
constexpr double kIndexFinalMiss = 1e-4;
// T with (1 - s)^T <= p / k, for log_p_k = log(p / k)
__host__ __device__ inline double index_step_bound(double s, double log_p_k)
{
    return s >= 1.0 ? 1.0 : ceil(log_p_k / log1p(-s));
}
constexpr uint32_t kIndexPadKeys = 16u;  // allocated past the last list: row scans load
                                         // whole batches of keys and mask those past a list
inline uint64_t index_entry_count(uint32_t k) { return (uint64_t)k * kIndexSteps; }
constexpr uint32_t kIndexListAlign = 16u;  // keys per 128-byte line
// Keys a buffer holds for k hashes over `dims` lists padded to multiples of `align` (an upper
// bound: each list adds at most align - 1 pads), without the kIndexPadKeys past the end.
inline uint64_t index_padded_count(uint32_t k, uint32_t dims, uint32_t align)
{
    return index_entry_count(k) + (uint64_t)(align - 1) * dims;
}
inline uint64_t index_scan_blocks(uint32_t dims) { return ((uint64_t)dims + 1 + 1023) / 1024; }

// ix.align sets the lists' padding; the buffers hold index_padded_count(k, D, ix.align) +
// kIndexPadKeys keys.
hipError_t launch_index_build(const Bounds &b, uint64_t seed, uint32_t k, const IndexBuffers &ix,
                              hipStream_t stream);

// Scheduling of the index rows kernel (it never changes a value); 0 leaves a choice to the
// launcher.
struct IndexPlan {
    uint32_t waves = 0;  // wavefronts per workgroup, 1..16 with waves * k * 4 bytes of LDS
                         // (0: 4 for k <= 2048, else 1)
    uint32_t batch = 0;  // keys a lane loads per round trip, 8 or 16 (0: 16 where lists are
                         // long, 8 where short)
    uint32_t claim = 0;  // 1: wavefronts claim rows from a counter, 2: a fixed stride over the
                         // batch (0: the counter for batches of >= 16 rows per wavefront)
};
constexpr uint32_t kIndexMaxWaves = 16u;
// The plan's wavefronts per workgroup for k hashes, or 0 when they do not fit.
uint32_t index_rows_waves(uint32_t k, uint32_t waves);

// row_counter: one device word, cleared by launches that claim rows from it.
hipError_t launch_index_rows(const Rows &rows, const IndexBuffers &ix, const Bounds &b, uint32_t k,
                             uint16_t *sig, unsigned long long *row_counter, uint32_t grid,
                             hipStream_t stream, const IndexPlan &plan = IndexPlan{});

// Resident workgroups per CU of the index row kernel with `waves` wavefronts (0: default).
int index_rows_blocks_per_cu(uint32_t k, uint32_t waves = 0);

// b-bit signatures (wmh_codec.hip): f = 32 / bits fields per word, W = ceil(k / f) words a row.
uint32_t pack_words(uint32_t k, uint32_t bits);  // 0 when bits is not in [1, 16] or k = 0
hipError_t launch_pack(const uint16_t *sig, uint64_t n_rows, uint32_t k, uint32_t bits,
                       uint32_t *packed, unsigned long long *saturated, hipStream_t stream);
hipError_t launch_unpack(const uint32_t *packed, uint64_t n_rows, uint32_t k, uint32_t bits,
                         uint16_t *sig, hipStream_t stream);
hipError_t launch_sig_max(const uint16_t *sig, uint64_t n, uint32_t *max_value, hipStream_t stream);
hipError_t launch_packed_collisions(const uint32_t *A, uint64_t na, const uint32_t *B, uint64_t nb,
                                    uint32_t k, uint32_t bits, uint32_t *counts, hipStream_t stream);
// (K, L) banding index over signatures (wmh_lsh.hip).
constexpr uint32_t kLshQueryBuffer = 2048;  // candidate matches a query may collect (a power of 2)
hipError_t launch_lsh_build(const uint16_t *sig, uint64_t n, uint32_t k, uint32_t K, uint32_t L,
                            uint32_t cap_log2, uint16_t *bands, unsigned long long *table_key,
                            uint32_t *table_head, uint32_t *next, hipStream_t stream);
hipError_t launch_lsh_query(const uint16_t *query, uint64_t nq, uint32_t k, uint32_t K, uint32_t L,
                            uint64_t n, uint32_t cap_log2, const uint16_t *bands,
                            const unsigned long long *table_key, const uint32_t *table_head,
                            const uint32_t *next, uint32_t max_out, uint32_t *out,
                            uint32_t *out_count, hipStream_t stream);

hipError_t launch_quantize(const float *x, uint64_t n, const uint32_t *col, const uint32_t *bound_q,
                           uint32_t dims, double alpha, uint32_t *out, unsigned long long *clipped,
                           hipStream_t stream);
hipError_t launch_packed_estimate(const uint32_t *A, const uint32_t *B, uint64_t n_pairs,
                                  uint32_t k, uint32_t bits, uint32_t *count, double *jhat,
                                  hipStream_t stream);

}  // namespace wmh
