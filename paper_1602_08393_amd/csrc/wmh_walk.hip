// The shared-window walk (batched path) for gfx950: persistent workgroups over (row block,
// hash block) tiles, one shared position stream for every row, windows of consecutive steps
// tested by all lanes at once.
//
// This file is compiled with uniform regions left unstructured
// (-structurizecfg-skip-uniform-regions): every branch of the window loop is scalar, and
// without structurization its early exits leave the loop directly, so the wait for each
// prefetched window is exact instead of a wait for every load in flight.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wmh_entries.h"
#include "wmh_internal.h"

namespace wmh {

namespace {

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1u); }

// Claims on a counter shared by a workgroup's wavefronts.  Every lane of the claiming
// wavefront adds 1 (so no lane-divergent region sits on the loop's path), each to its own
// word of a 64-word LDS array (one word per bank): the 64 atomics do not queue on one word.
// Lane 0's word counts the wavefronts' claims; its value before the add, broadcast, is the
// claim.  Called with every lane active; reset() by threads 0..63 between uses.
struct WaveClaims {
    uint32_t word[kWave];
    __device__ __forceinline__ void reset()
    {
        if (threadIdx.x < kWave) word[threadIdx.x] = 0u;
    }
    __device__ __forceinline__ uint32_t claim()
    {
        const uint32_t before = atomicAdd(&word[threadIdx.x & (kWave - 1u)], 1u);
        return (uint32_t)__builtin_amdgcn_readfirstlane(before);
    }
};

// ---------------------------------------------------------------------------------------------
// Batched persistent walk.
//
// A tile is (row block of R rows) x (block of J hash ids).  Workgroups take tiles from an
// atomic counter; the R rows of a tile's row block sit in LDS component-major (RowLayout), so
// one stream entry locates component c for every row.  A wavefront walks one hash id for the whole
// row block, a window of L * K consecutive steps at a time (L = 64 / R lanes per row, K steps
// per lane): lane l serves row l / L and K consecutive steps of the window, keeps the first
// green one, and a ballot tells which rows have a green step so far; the walk ends when every
// row of the block has one.  Every row of the block sees the same draw, so one draw serves R
// rows (the sequence depends only on (seed, j, t), never on the row), and the window replaces
// the per-lane geometric tail of the plain walk by at most one partly used window per (block,
// hash).  Draws come from the shared stream for t <= depth and are made in-lane beyond it.
// ---------------------------------------------------------------------------------------------
// min(v, v of the lane the DPP control selects); lanes outside the written rows, or whose
// source lies outside their row, keep v.
template <int kCtrl, int kRows>
__device__ __forceinline__ uint32_t dpp_min(uint32_t v)
{
    const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)v, kCtrl,
                                                             kRows, 0xF, false);
    return min(v, t);
}

// Minimum of v over each group of L consecutive lanes (L a power of two <= 64), left in the
// group's last lane: prefix minima by row shifts inside 16-lane DPP rows, then row broadcasts
// (lane 15 into the next row, lane 31 into rows 2 and 3) for groups of 32 and 64 lanes.
template <uint32_t L>
__device__ __forceinline__ uint32_t group_min_at_last_lane(uint32_t v)
{
    if constexpr (L >= 2) v = dpp_min<0x111, 0xF>(v);   // row_shr:1
    if constexpr (L >= 4) v = dpp_min<0x112, 0xF>(v);   // row_shr:2
    if constexpr (L >= 8) v = dpp_min<0x114, 0xF>(v);   // row_shr:4
    if constexpr (L >= 16) v = dpp_min<0x118, 0xF>(v);  // row_shr:8
    if constexpr (L >= 32) v = dpp_min<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    if constexpr (L >= 64) v = dpp_min<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// The top bit of every L-lane segment of a 64-bit lane mask.
template <uint32_t L>
__host__ __device__ constexpr uint64_t segment_tops()
{
    uint64_t m = 0;
    for (uint32_t r = 0; r < kWave / L; ++r) m |= 1ull << (r * L + L - 1);
    return m;
}

// What coarse codes are made from: the bounds m and the code bits.
struct Codes {
    const uint32_t *bound;
    uint32_t bits;
};

// The LDS value of a row's nonzero x at component c: x itself, or its coarse code.
template <typename XT, bool kCoarse>
__device__ __forceinline__ XT lds_value(uint32_t x, uint32_t c, const Codes &codes)
{
    if constexpr (kCoarse) return (XT)coarse_value_code(x, codes.bound[c], codes.bits);
    else return (XT)x;
}

// Green test of a step drawn in-lane (exact offset o at component c) against the LDS value
// lv of CSR row `row`: o < x, with x itself in LDS, or from the coarse codes (a tie reads the
// row's exact value).
template <bool kCoarse>
__device__ __forceinline__ bool lane_green(uint64_t o, uint32_t lv, uint32_t c, const Codes &codes,
                                           const Rows &rows, uint64_t row)
{
    if constexpr (kCoarse) {
        if (lv == 0) return false;
        const uint32_t v = coarse_offset_code((uint32_t)o, codes.bound[c], codes.bits);
        if (v != lv) return v < lv;
        return o < (uint64_t)csr_value(rows.row_ptr, rows.col, rows.val, row, c);
    } else {
        return o < (uint64_t)lv;
    }
}

// The next tile of a workgroup and what staging its rows needs, read ahead by thread 0 while
// the current tile is walked: the tile (n_tiles or more: none), the CSR entries of its n rows
// (from lo; row r ends at lo + end[r], so a block's entries number below 2^32, as rows of
// distinct columns below D do) and the rows the row filter leaves to another path (bit r).  A
// workgroup keeps two, the current tile's and the next one's.
template <int R>
struct TileAhead {
    uint64_t tile;
    uint64_t lo;
    uint32_t end[R];
    uint32_t skip;
};

// The walks' static LDS (two TileAheads, the claim words, a flag) fits the room the dynamic
// limit leaves.
static_assert(2 * sizeof(TileAhead<16>) + sizeof(WaveClaims) + 16 <= 160 * 1024 - kMaxDynamicLds,
              "static LDS of the walks exceeds the room below the dynamic limit");

// Fills `a` for `tile` of a walk over row blocks of R rows (thread 0 only).  Every load is
// issued before the first store.
template <int R>
__device__ __forceinline__ void read_ahead(TileAhead<R> &a, const Rows &rows, uint64_t tile,
                                           uint64_t n_tiles, uint32_t n_hash_tiles)
{
    a.tile = tile;
    if (tile >= n_tiles) return;
    const uint64_t row0 = tile / n_hash_tiles * R;
    const uint32_t n = (uint32_t)min((uint64_t)R, rows.n_rows - row0);
    uint64_t rp[R + 1];
    uint32_t skip = 0;
#pragma unroll
    for (int q = 0; q <= R; ++q) rp[q] = (uint32_t)q <= n ? rows.row_ptr[row0 + q] : 0ull;
    if (rows.row_class)
        for (uint32_t r = 0; r < n; ++r) skip |= rows.skips(row0 + r) ? 1u << r : 0u;
    a.lo = rp[0];
#pragma unroll
    for (int q = 0; q < R; ++q) a.end[q] = (uint32_t)(rp[q + 1] - rp[0]);
    a.skip = skip;
}

// Zeroes the first `bytes` bytes of LDS (rounded up to 16) with 16-byte stores.  Called by the
// whole workgroup.
__device__ __forceinline__ void zero_lds(unsigned char *smem, size_t bytes)
{
    uint4 *z = reinterpret_cast<uint4 *>(smem);
    const uint32_t n = (uint32_t)((bytes + 15) / 16);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) z[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Scatters the CSR entries [lo, lo + count) of consecutive rows into the dense rows in LDS
// (RowLayout; coarse codes with kCoarse): an entry's row is the number of the interior
// boundaries bnd[0 .. R-2] (row_ptr of rows 1 .. R-1 of the block, minus lo; count for rows
// past the block's end) at or below its index; rows with bit r of `skip` are left alone.  A
// block's entries number at most R * D < 2^32.  Each thread reads four entries at a time (two
// for coarse codes of several rows), all loads in flight before the first store.  Returns bit
// r for every row r with a nonzero value among the thread's entries.
template <typename XT, int R, bool kCoarse>
__device__ __forceinline__ uint32_t scatter_entries(unsigned char *smem, const Rows &rows,
                                                    uint64_t lo, uint32_t count,
                                                    const uint32_t *bnd, uint32_t D,
                                                    const Codes &codes, uint32_t skip)
{
    using Layout = RowLayout<XT, R>;
    constexpr int kBatch = kCoarse && R > 1 ? 2 : 4;  // coarse codes hold a bound per entry
    const uint32_t *col = rows.col + lo;
    const uint32_t *val = rows.val + lo;
    uint32_t mine = 0;
    for (uint32_t i0 = threadIdx.x; i0 < count; i0 += kBatch * blockDim.x) {
        uint32_t c[kBatch], v[kBatch], m[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const uint32_t i = i0 + q * blockDim.x;
            c[q] = i < count ? col[i] : 0u;
            v[q] = i < count ? val[i] : 0u;
        }
        if constexpr (kCoarse) {
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const uint32_t i = i0 + q * blockDim.x;
                m[q] = i < count && c[q] < D ? codes.bound[c[q]] : 1u;
            }
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const uint32_t i = i0 + q * blockDim.x;
            if (i >= count) continue;
            uint32_t r = 0;
#pragma unroll
            for (int b = 0; b + 1 < R; ++b) r += i >= bnd[b] ? 1u : 0u;
            if ((skip >> r) & 1u) continue;
            if (c[q] < D) {
                if constexpr (kCoarse)
                    *Layout::at(smem, c[q], r, D) = (XT)coarse_value_code(v[q], m[q], codes.bits);
                else
                    *Layout::at(smem, c[q], r, D) = (XT)v[q];
            }
            if (v[q]) mine |= 1u << r;
        }
    }
    return mine;
}

// Stages the n_here rows of a block whose CSR entries start at lo (row r ending at
// lo + end[r]): zeroes the block's LDS rows, scatters the rows' entries in one pass over the
// block's contiguous CSR range and sets bit r of *nonempty for every row r with a nonzero value;
// rows with bit r of `skip` stay zero.  Called by the whole workgroup.
template <typename XT, int R, bool kCoarse>
__device__ __forceinline__ void stage_block(unsigned char *smem, const Rows &rows, uint64_t lo,
                                            const uint32_t *end, uint32_t n_here, uint32_t D,
                                            const Codes &codes, uint32_t *nonempty,
                                            uint32_t skip = 0)
{
    zero_lds(smem, (size_t)D * R * sizeof(XT));
    if (threadIdx.x == 0) *nonempty = 0;
    __syncthreads();
    const uint32_t count = end[n_here - 1];
    uint32_t bnd[R > 1 ? R - 1 : 1];
#pragma unroll
    for (int q = 0; q + 1 < R; ++q) bnd[q] = (uint32_t)(q + 1) < n_here ? end[q] : count;
    const uint32_t mine = scatter_entries<XT, R, kCoarse>(smem, rows, lo, count, bnd, D, codes, skip);
    if (mine) atomicOr(nonempty, mine);
    __syncthreads();
}

// Writes a tile's hash values (staged in LDS, row r at hbuf[r * hashes_per_tile]) row by row,
// coalesced along j, except rows with bit r of `skip`, and resets the claim counter for the
// next tile.  Called by the whole workgroup; ends with a barrier.
__device__ __forceinline__ void write_tile(uint16_t *__restrict__ sig, const uint16_t *hbuf,
                                           uint64_t row0, uint32_t n_here, uint32_t k,
                                           uint32_t j0, uint32_t j1, uint32_t hashes_per_tile,
                                           WaveClaims &units, uint32_t skip = 0)
{
    __syncthreads();
    const uint32_t width = j1 - j0;
    for (uint32_t r = 0; r < n_here; ++r) {
        if ((skip >> r) & 1u) continue;
        uint16_t *out = sig + (row0 + r) * (uint64_t)k + j0;
        for (uint32_t q = threadIdx.x; q < width; q += blockDim.x) out[q] = hbuf[r * hashes_per_tile + q];
    }
    units.reset();
    __syncthreads();
}

// Up to four rows per block the walk fits eight wavefronts per SIMD (at most 64 VGPRs and a
// few scalar registers spilled to vector lanes); wider blocks keep their registers.
template <int R>
constexpr int walk_waves_per_eu() { return R <= 4 ? 8 : 1; }

template <typename XT, int R, int K, bool kPacked, bool kCoarse>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(walk_waves_per_eu<R>()))) void batched_kernel(Bounds b, Rows rows, uint32_t k,
                                                       uint64_t seed, uint16_t *__restrict__ sig,
                                                       uint32_t hashes_per_tile, uint32_t depth,
                                                       const void *entries,
                                                       unsigned long long *tile_counter,
                                                       uint32_t coarse_bits)
{
    const Codes codes{b.bound, coarse_bits};
    // Lane layout of one window: lane l serves row r = l / L (L = 64 / R lanes per row) and
    // the K consecutive steps base + g*K + 1 .. base + g*K + K, g = l mod L; the 64 lanes
    // cover steps base + 1 .. base + kWin of all R rows, kWin = L * K.
    constexpr uint32_t L = kWave / R;
    constexpr uint32_t kWin = L * K;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ TileAhead<R> ahead[2];  // the current tile's and the next one's
    __shared__ WaveClaims units;
    __shared__ uint32_t nonempty;
    const uint32_t D = b.dims;
    uint16_t *hbuf = reinterpret_cast<uint16_t *>(smem + (((size_t)D * R * sizeof(XT) + 15) & ~(size_t)15));
    const uint32_t my_row = lane() / L;
    const uint32_t my_grp = lane() % L;
    using Layout = RowLayout<XT, R>;
    constexpr uint32_t kScale = Layout::kGroup;  // LDS bytes per component group
    const uint32_t row_byte = Layout::row_byte(my_row, D);
    // 1 + position in a window of each of the lane's K steps; offset of its run in words
    uint32_t step_in_window[K];
#pragma unroll
    for (int q = 0; q < (int)K; ++q) step_in_window[q] = my_grp * K + q + 1u;
    const uint32_t lane_words = my_grp * K * EntryRun<K, kPacked>::kWordsPerEntry;

    const uint64_t n_blocks = (rows.n_rows + R - 1) / R;
    const uint32_t n_hash_tiles = (k + hashes_per_tile - 1) / hashes_per_tile;
    const uint64_t n_tiles = n_blocks * n_hash_tiles;
    uint64_t staged = ~0ull;
    bool claimed = false;

    // Tiles are claimed one ahead: while a tile is walked, thread 0 claims the next one and
    // reads its rows' CSR boundaries and filter bits into the other TileAhead, so the claim and
    // those reads are off the staging path.  The barriers that end a tile publish it.
    uint32_t cur = 0;
    if (threadIdx.x == 0)
        read_ahead<R>(ahead[0], rows, next_tile(tile_counter, claimed), n_tiles, n_hash_tiles);
    units.reset();
    __syncthreads();
    while (true) {
        const uint64_t tile = ahead[cur].tile;
        if (tile >= n_tiles) break;
        const uint64_t blk = tile / n_hash_tiles;
        const uint32_t ht = (uint32_t)(tile - blk * n_hash_tiles);
        const uint64_t row0 = blk * R;
        const uint32_t n_here = (uint32_t)min((uint64_t)R, rows.n_rows - row0);
        // rows another path computes (row filter): not staged, not walked, not written
        const uint32_t skip = __builtin_amdgcn_readfirstlane(ahead[cur].skip);
        if (skip == (1u << n_here) - 1u) {
            if (threadIdx.x == 0)
                read_ahead<R>(ahead[cur ^ 1u], rows, next_tile(tile_counter, claimed), n_tiles,
                              n_hash_tiles);
            __syncthreads();
            cur ^= 1u;
            continue;
        }

        if (blk != staged) {
            stage_block<XT, R, kCoarse>(smem, rows, ahead[cur].lo, ahead[cur].end, n_here, D,
                                        codes, &nonempty, skip);
            staged = blk;
        }
        if (threadIdx.x == 0)
            read_ahead<R>(ahead[cur ^ 1u], rows, next_tile(tile_counter, claimed), n_tiles,
                          n_hash_tiles);
        // Wave-uniform values are read into scalar registers so every branch on them is a
        // scalar branch: no lane-divergent region sits on the unit loop's path.
        const uint32_t live = __builtin_amdgcn_readfirstlane(nonempty);
        const bool my_row_live = ((live >> my_row) & 1u) != 0;
        const uint32_t j0 = ht * hashes_per_tile;
        const uint32_t j1 = min(k, j0 + hashes_per_tile);

        while (true) {
            // claim the next hash id of the tile
            const uint32_t j = j0 + units.claim();
            if (j >= j1) break;

            // Each lane keeps the first green step among its own steps (kNoStep: none yet); a
            // row's hash is the smallest of its lanes' values, since together they cover every
            // step, and a row whose smallest value is above the cap saturates at 65535.  Lanes
            // of rows with no green unit start at 0, so the stop test sees them as done.
            constexpr uint32_t kNoStep = 0xFFFFFFFFu;
            constexpr uint32_t kNotGreen = 0x10000u;  // base + kNotGreen is past the cap
            uint32_t lane_h = my_row_live ? kNoStep : 0u;
            // The walk goes on while some row's L-lane segment of the "has a green step" ballot
            // is zero: the lowest zero segment takes no borrow from below, so it shows its top
            // bit in (seen - bottoms) & ~seen, and a nonzero segment v shows it only when v - 1
            // has the top bit, which v then has as well.
            constexpr uint64_t kTops = segment_tops<L>();
            constexpr uint64_t kBottoms = kTops >> (L - 1);
            auto goes_on = [&]() {
                const uint64_t seen = __builtin_amdgcn_ballot_w64(lane_h <= kCap);
                return ((seen - kBottoms) & ~seen & kTops) != 0;
            };
            // window [base + 1, base + kWin] from the lane's K stream entries; with coarse
            // codes, true when some step of the wavefront's window tied (the caller then tests
            // the window again with in-lane draws, which are exact; ties count as red here)
            auto stream_window = [&](const EntryRun<K, kPacked> &run, uint32_t base) -> bool {
                uint32_t xv[K], off[K];  // all K reads in flight before the first compare
#pragma unroll
                for (int q = 0; q < (int)K; ++q) {
                    uint32_t lds;
                    run.get(q, kScale, &lds, &off[q]);
                    xv[q] = *reinterpret_cast<const XT *>(smem + lds + row_byte);
                }
                uint32_t c = kNotGreen;  // 1 + position in the window of the lane's first green step
#pragma unroll
                for (int q = K - 1; q >= 0; --q) c = off[q] < xv[q] ? step_in_window[q] : c;
                lane_h = min(lane_h, base + c);
                if constexpr (kCoarse) {
                    bool tie = false;
#pragma unroll
                    for (int q = 0; q < (int)K; ++q) tie = tie || off[q] == xv[q];
                    return __builtin_amdgcn_ballot_w64(tie) != 0;
                } else {
                    return false;
                }
            };
            // the same window with the draws made in-lane, one step at a time; step 65536 of
            // the last window may show up here: it is above the cap like "no green step"
            auto lane_window = [&](uint32_t base) {
                uint32_t c = kNotGreen;
#pragma unroll 1
                for (int q = K - 1; q >= 0; --q) {
                    const uint32_t t = base + my_grp * K + q + 1u;
                    const uint64_t p = position(seed, j, t, b.total, b.threshold);
                    uint64_t o64;
                    const uint32_t comp = component_of(p, b.prefix, b.bucket, b.shift, &o64);
                    const uint32_t lv = *reinterpret_cast<const XT *>(smem + (size_t)comp * kScale + row_byte);
                    c = lane_green<kCoarse>(o64, lv, comp, codes, rows, row0 + my_row) ? my_grp * K + q + 1u : c;
                }
                lane_h = min(lane_h, base + c);
            };

            // Stream windows.  The depth is a whole number of cycles of three windows below
            // the cap, so these windows test nothing but the stop condition.  Entries are
            // prefetched three windows ahead into a ring of three register sets, each reloaded
            // right after its window is tested; the buffer holds one spare cycle past the last
            // id's entries for the prefetches of the last cycle (read, never used).  The
            // window's address is scalar; each lane adds its own 32-bit offset.
            bool walking = live != 0;
            uint32_t base = 0;
            if (walking && depth != 0) {
                const uint32_t *id_entries =
                    reinterpret_cast<const uint32_t *>(entries) +
                    (uint64_t)j * depth * EntryRun<K, kPacked>::kWordsPerEntry;
                // Each prefetch stays where it is issued: the empty asm after it is a compiler
                // barrier for memory (entries is not a restrict pointer, so the loads are not
                // known to read memory that nothing writes; such loads are otherwise sunk to the
                // window that uses them, which then waits for them).
                auto fetch = [&](uint32_t at) {
                    EntryRun<K, kPacked> run;
                    run.load_at(id_entries + (size_t)at * EntryRun<K, kPacked>::kWordsPerEntry,
                                lane_words);
                    asm volatile("" ::: "memory");
                    return run;
                };
                EntryRun<K, kPacked> e0 = fetch(0), e1 = fetch(kWin), e2 = fetch(2 * kWin);
                for (; base < depth; base += 3 * kWin) {
                    if (stream_window(e0, base)) lane_window(base);
                    if (!goes_on()) break;
                    e0 = fetch(base + 3 * kWin);
                    if (stream_window(e1, base + kWin)) lane_window(base + kWin);
                    if (!goes_on()) break;
                    e1 = fetch(base + 4 * kWin);
                    if (stream_window(e2, base + 2 * kWin)) lane_window(base + 2 * kWin);
                    if (!goes_on()) break;
                    e2 = fetch(base + 5 * kWin);
                }
                walking = base >= depth;
            }
            // past the stream (rare): draws made in-lane, up to the window that holds the cap
            for (; walking && base < kCap; base += kWin) {
                lane_window(base);
                walking = goes_on();
            }
            // smallest lane value of each row, in the row's last lane; above the cap: no green
            // step, the hash saturates
            const uint32_t best = group_min_at_last_lane<L>(lane_h);
            // empty rows hash to 0
            const uint32_t h = !my_row_live ? 0u : min(best, kCap);
            // every lane stores; only each row's last lane writes a tile value
            const uint32_t slot = my_grp == L - 1 ? my_row * hashes_per_tile + (j - j0)
                                                  : R * hashes_per_tile + lane();
            hbuf[slot] = (uint16_t)h;
        }
        write_tile(sig, hbuf, row0, n_here, k, j0, j1, hashes_per_tile, units, skip);
        cur ^= 1u;
    }
}


// ---------------------------------------------------------------------------------------------
// Ballot walk: one row per block (R = 1), one hash id at a time per wavefront, lane l testing
// step base + l + 1 of each 64-step window.  Lanes follow the steps in order, so the row's first
// green step is the lowest set bit of the window's ballot: the stop test is the ballot itself
// and the hash is base + ctz(ballot) + 1, both on the scalar unit, with no per-lane state and no
// cross-lane reduction.  Stream windows come three at a time from a ring prefetched three windows
// ahead (as in the shared-window walk); steps past the stream are drawn in-lane.  Hash ids are
// claimed in pairs whose first windows are requested together (see below).
//
// Hash groups (groups = G > 1): the hash ids are cut into G blocks of hashes_per_tile ids, and
// group g's tiles are (row, block g) for every row, claimed from counter g.  A workgroup starts
// on group blockIdx.x mod G and moves on to the next group once its own is exhausted.
// Workgroups are dispatched to the chip's XCDs in turn, so with G = 8 (or a divisor of 8) the
// workgroups of one XCD mostly walk one block of hash ids, and that XCD's L2 holds only that
// block's part of the position stream; each row is then staged once per group.
// ---------------------------------------------------------------------------------------------
template <typename XT, bool kPacked, bool kCoarse>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void ballot_kernel(
    Bounds b, Rows rows, uint32_t k, uint64_t seed, uint16_t *__restrict__ sig,
    uint32_t hashes_per_tile, uint32_t depth, const void *entries, unsigned long long *tile_counter,
    uint32_t groups, uint32_t coarse_bits)
{
    const Codes codes{b.bound, coarse_bits};
    constexpr uint32_t kWords = EntryRun<1, kPacked>::kWordsPerEntry;
    extern __shared__ __align__(16) unsigned char smem[];
    // A tile (row, hash block ht) and its row's CSR range and filter bit, read ahead.
    struct RowAhead {
        uint64_t row;  // ~0: no tile left
        uint64_t lo, hi;
        uint32_t ht, skip;
    };
    __shared__ RowAhead ahead[2];  // the current tile's and the next one's
    __shared__ WaveClaims units;
    __shared__ uint32_t nonempty;
    const uint32_t D = b.dims;
    uint16_t *hbuf = reinterpret_cast<uint16_t *>(smem + (((size_t)D * sizeof(XT) + 15) & ~(size_t)15));
    const uint32_t lane_words = lane() * kWords;
    const uint32_t n_hash_tiles = (k + hashes_per_tile - 1) / hashes_per_tile;
    const uint64_t n_tiles = rows.n_rows * n_hash_tiles;
    uint64_t staged = ~0ull;
    bool claimed = false;
    uint32_t group_step = 0;  // thread 0: groups left behind, counted from the workgroup's own

    // Tiles are claimed one ahead (as in the shared-window walk): thread 0 claims the next tile
    // and reads its row's CSR range while the current one is walked.
    auto claim_ahead = [&](RowAhead &a) {
        uint64_t r = ~0ull;
        uint32_t h = 0;
        if (groups <= 1) {
            const uint64_t t = next_tile(tile_counter, claimed);
            if (t < n_tiles) {
                r = t / n_hash_tiles;
                h = (uint32_t)(t - r * n_hash_tiles);
            }
        } else {
            // every group's counter passes n_rows at most once per workgroup: the loop ends
            for (; group_step < groups; ++group_step) {
                const uint32_t g = (blockIdx.x + group_step) % groups;
                const uint64_t u = atomicAdd(&tile_counter[g], 1ull);
                if (u < rows.n_rows) {
                    r = u;
                    h = g;
                    break;
                }
            }
        }
        uint64_t lo = 0, hi = 0;
        uint32_t skip = 0;
        if (r != ~0ull) {
            lo = rows.row_ptr[r];
            hi = rows.row_ptr[r + 1];
            skip = rows.skips(r) ? 1u : 0u;
        }
        a.row = r;
        a.ht = h;
        a.lo = lo;
        a.hi = hi;
        a.skip = skip;
    };
    uint32_t cur = 0;
    if (threadIdx.x == 0) claim_ahead(ahead[0]);
    units.reset();
    __syncthreads();
    while (true) {
        const uint64_t row = ahead[cur].row;
        if (row == ~0ull) break;
        const uint32_t ht = ahead[cur].ht;
        if (ahead[cur].skip) {  // a row another path computes (row filter)
            if (threadIdx.x == 0) claim_ahead(ahead[cur ^ 1u]);
            __syncthreads();
            cur ^= 1u;
            continue;
        }
        if (row != staged) {
            zero_lds(smem, (size_t)D * sizeof(XT));
            if (threadIdx.x == 0) nonempty = 0;
            __syncthreads();
            const uint32_t none = 0;
            const uint64_t lo = ahead[cur].lo;
            const uint32_t mine = scatter_entries<XT, 1, kCoarse>(
                smem, rows, lo, (uint32_t)(ahead[cur].hi - lo), &none, D, codes, 0u);
            if (mine) atomicOr(&nonempty, mine);
            __syncthreads();
            staged = row;
        }
        const bool live = __builtin_amdgcn_readfirstlane(nonempty) != 0;
        const uint32_t j0 = ht * hashes_per_tile;
        if (threadIdx.x == 0) claim_ahead(ahead[cur ^ 1u]);
        if (j0 >= k) {  // an empty hash block (the host's plans leave none)
            __syncthreads();
            cur ^= 1u;
            continue;
        }
        const uint32_t j1 = min(k, j0 + hashes_per_tile);

        // ballot of the lanes whose step is green in the window the run holds; with coarse
        // codes *tie is the ballot of the lanes whose codes tie (0 otherwise)
        auto stream_ballot = [&](const EntryRun<1, kPacked> &run, uint64_t *tie) {
            uint32_t lds, off;
            run.get(0, (uint32_t)sizeof(XT), &lds, &off);
            const uint32_t xv = *reinterpret_cast<const XT *>(smem + lds);
            if constexpr (kCoarse) *tie = __builtin_amdgcn_ballot_w64(off == xv);
            else *tie = 0;
            return __builtin_amdgcn_ballot_w64(off < xv);
        };
        // whether a tie lies below the lowest green lane (the window is then walked on with
        // in-lane draws, which are exact); tested only when the window has a green or tied lane
        auto tie_first = [](uint64_t green, uint64_t tie) {
            const uint64_t below = green ? (green & (0ull - green)) - 1ull : ~0ull;
            return (tie & below) != 0;
        };
        // each prefetch stays where it is issued (see the shared-window walk)
        auto fetch = [&](uint32_t j, uint32_t at) {
            EntryRun<1, kPacked> run;
            run.load_at(reinterpret_cast<const uint32_t *>(entries) +
                            ((uint64_t)j * depth + at) * kWords,
                        lane_words);
            asm volatile("" ::: "memory");
            return run;
        };
        // every lane stores; only lane 0 writes the tile value
        auto store = [&](uint32_t j, uint32_t h) {
            hbuf[lane() == 0 ? j - j0 : hashes_per_tile + lane()] = (uint16_t)h;
        };
        // draws made in-lane from step base + 1 up to the window that holds the cap: the first
        // green step, or the cap (a green step 65536 in the last window is past it as well)
        auto lane_walk = [&](uint32_t j, uint32_t base) -> uint32_t {
            for (; base < kCap; base += kWave) {
                const uint32_t t = base + lane() + 1u;
                const uint64_t p = position(seed, j, t, b.total, b.threshold);
                uint64_t o64;
                const uint32_t comp = component_of(p, b.prefix, b.bucket, b.shift, &o64);
                const uint32_t lv = *reinterpret_cast<const XT *>(smem + (size_t)comp * sizeof(XT));
                const uint64_t green =
                    __builtin_amdgcn_ballot_w64(lane_green<kCoarse>(o64, lv, comp, codes, rows, row));
                if (green) return min(base + (uint32_t)__builtin_ctzll(green) + 1u, kCap);
            }
            return kCap;
        };
        // hash id j from its three requested windows, then the stream, then in-lane draws
        auto walk_id = [&](uint32_t j, EntryRun<1, kPacked> &e0, EntryRun<1, kPacked> &e1,
                           EntryRun<1, kPacked> &e2) {
            uint64_t tie = 0;
            for (uint32_t base = 0; base < depth; base += 3 * kWave) {
                uint64_t green = stream_ballot(e0, &tie);
                if (green | tie) {
                    if (tie && tie_first(green, tie)) return store(j, lane_walk(j, base));
                    if (green) return store(j, base + (uint32_t)__builtin_ctzll(green) + 1u);
                }
                e0 = fetch(j, base + 3 * kWave);
                green = stream_ballot(e1, &tie);
                if (green | tie) {
                    if (tie && tie_first(green, tie)) return store(j, lane_walk(j, base + kWave));
                    if (green) return store(j, base + kWave + (uint32_t)__builtin_ctzll(green) + 1u);
                }
                e1 = fetch(j, base + 4 * kWave);
                green = stream_ballot(e2, &tie);
                if (green | tie) {
                    if (tie && tie_first(green, tie))
                        return store(j, lane_walk(j, base + 2 * kWave));
                    if (green)
                        return store(j, base + 2 * kWave + (uint32_t)__builtin_ctzll(green) + 1u);
                }
                e2 = fetch(j, base + 5 * kWave);
            }
            store(j, lane_walk(j, depth));  // past the stream (rare)
        };
        // claim u: hash ids 2u and 2u + 1
        auto claim_pair = [&]() { return j0 + 2u * units.claim(); };
        if (!live || depth == 0) {
            // empty rows hash to 0; without a stream every draw is made in-lane
            for (uint32_t ja = claim_pair(); ja < j1; ja = claim_pair())
                for (uint32_t j = ja; j < min(ja + 2u, j1); ++j) store(j, live ? lane_walk(j, 0) : 0u);
        } else {
            // Both ids' first windows are requested at once, each into its own registers, so the
            // second id starts on entries that arrived while the first was walked.  A pair cut
            // by the tile's end requests its first id's windows twice (unused the second time).
            for (uint32_t ja = claim_pair(); ja < j1; ja = claim_pair()) {
                const uint32_t jb = min(ja + 1u, j1 - 1u);
                EntryRun<1, kPacked> a0 = fetch(ja, 0), a1 = fetch(ja, kWave), a2 = fetch(ja, 2 * kWave);
                EntryRun<1, kPacked> b0 = fetch(jb, 0), b1 = fetch(jb, kWave), b2 = fetch(jb, 2 * kWave);
                walk_id(ja, a0, a1, a2);
                if (jb != ja) walk_id(jb, b0, b1, b2);
            }
        }
        write_tile(sig, hbuf, row, 1u, k, j0, j1, hashes_per_tile, units);
        cur ^= 1u;
    }
}

// Raises the kernel's dynamic LDS limit once per process; the launches return its status, so
// a limit the runtime refuses fails at the launch that needs it.
template <typename XT, int R, int K, bool kPacked, bool kCoarse>
hipError_t configure_batched()
{
    static const hipError_t status =
        hipFuncSetAttribute((const void *)batched_kernel<XT, R, K, kPacked, kCoarse>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    return status;
}

template <typename XT, int R, int K, bool kPacked, bool kCoarse>
int batched_occupancy_t(const BatchedPlan &plan, size_t lds)
{
    configure_batched<XT, R, K, kPacked, kCoarse>();
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel<XT, R, K, kPacked, kCoarse>,
                                                     plan.waves_per_block * kWave, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <typename XT, int R, int K, bool kPacked, bool kCoarse>
hipError_t launch_batched_t(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                                   uint16_t *sig, const BatchedPlan &plan, const void *entries,
                                   unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    const size_t lds = batched_lds_bytes(b.dims, plan);
    const hipError_t e = configure_batched<XT, R, K, kPacked, kCoarse>();
    if (e != hipSuccess) return e;
    batched_kernel<XT, R, K, kPacked, kCoarse><<<grid, plan.waves_per_block * kWave, lds, stream>>>(
        b, rows, k, seed, sig, plan.hashes_per_tile, plan.stream_depth, entries, tile_counter,
        plan.coarse_bits);
    return hipGetLastError();
}

template <typename XT, bool kPacked, bool kCoarse>
hipError_t configure_ballot()
{
    static const hipError_t status =
        hipFuncSetAttribute((const void *)ballot_kernel<XT, kPacked, kCoarse>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    return status;
}

template <typename XT, bool kPacked, bool kCoarse>
int ballot_occupancy_t(const BatchedPlan &plan, size_t lds)
{
    configure_ballot<XT, kPacked, kCoarse>();
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, ballot_kernel<XT, kPacked, kCoarse>,
                                                     plan.waves_per_block * kWave, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <typename XT, bool kPacked, bool kCoarse>
hipError_t launch_ballot_t(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                           uint16_t *sig, const BatchedPlan &plan, const void *entries,
                           unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    const size_t lds = batched_lds_bytes(b.dims, plan);
    const hipError_t e = configure_ballot<XT, kPacked, kCoarse>();
    if (e != hipSuccess) return e;
    ballot_kernel<XT, kPacked, kCoarse><<<grid, plan.waves_per_block * kWave, lds, stream>>>(
        b, rows, k, seed, sig, plan.hashes_per_tile, plan.stream_depth, entries, tile_counter,
        plan.hash_groups, plan.coarse_bits);
    return hipGetLastError();
}

// Calls F<XT, R, K, packed, coarse>() for the plan's template parameters: K = R, or K = 4 for
// R < 4; coarse codes for R <= 4 only.
template <template <typename, int, int, bool, bool> class F, typename... Args>
auto dispatch_batched(const BatchedPlan &plan, Args &&...args)
    -> decltype(F<uint16_t, 1, 1, true, false>::run(args...))
{
#define WMH_RK_CASE(RR, KK, COARSE)                                                              \
    if (plan.rows_per_block == RR && plan.steps_per_lane == KK) {                                \
        if (plan.coarse) {                                                                       \
            if (COARSE && plan.narrow && plan.packed)                                            \
                return F<uint16_t, RR, KK, true, COARSE>::run(args...);                          \
            return F<uint16_t, 1, 1, true, false>::fail();                                       \
        }                                                                                        \
        if (plan.narrow)                                                                         \
            return plan.packed ? F<uint16_t, RR, KK, true, false>::run(args...)                  \
                               : F<uint16_t, RR, KK, false, false>::run(args...);                \
        return plan.packed ? F<uint32_t, RR, KK, true, false>::run(args...)                      \
                           : F<uint32_t, RR, KK, false, false>::run(args...);                    \
    }
    WMH_RK_CASE(1, 1, true)
    WMH_RK_CASE(1, 4, true)
    WMH_RK_CASE(2, 2, true)
    WMH_RK_CASE(2, 4, true)
    WMH_RK_CASE(4, 4, true)
    WMH_RK_CASE(8, 8, false)
    WMH_RK_CASE(16, 16, false)
#undef WMH_RK_CASE
    return F<uint16_t, 1, 1, true, false>::fail();
}

template <typename XT, int R, int K, bool kPacked, bool kCoarse>
struct LaunchBatched {
    static hipError_t run(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                          uint16_t *sig, const BatchedPlan &plan, const void *entries,
                          unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
    {
        return launch_batched_t<XT, R, K, kPacked, kCoarse>(b, rows, k, seed, sig, plan, entries,
                                                            tile_counter, grid, stream);
    }
    static hipError_t fail() { return hipErrorInvalidValue; }
};

template <typename XT, int R, int K, bool kPacked, bool kCoarse>
struct OccupancyBatched {
    static int run(const BatchedPlan &plan, size_t lds)
    {
        return batched_occupancy_t<XT, R, K, kPacked, kCoarse>(plan, lds);
    }
    static int fail() { return 0; }
};

}  // namespace

hipError_t launch_shared_walk(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                              uint16_t *sig, const BatchedPlan &plan, const void *entries,
                              unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    return dispatch_batched<LaunchBatched>(plan, b, rows, k, seed, sig, plan, entries,
                                           tile_counter, grid, stream);
}

int shared_walk_blocks_per_cu(const BatchedPlan &plan, size_t lds)
{
    return dispatch_batched<OccupancyBatched>(plan, plan, lds);
}

hipError_t launch_ballot_walk(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                              uint16_t *sig, const BatchedPlan &plan, const void *entries,
                              unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    if (plan.coarse) {
        if (!plan.narrow || !plan.packed) return hipErrorInvalidValue;
        return launch_ballot_t<uint16_t, true, true>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
    }
    if (plan.narrow)
        return plan.packed
                   ? launch_ballot_t<uint16_t, true, false>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream)
                   : launch_ballot_t<uint16_t, false, false>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
    return launch_ballot_t<uint32_t, false, false>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
}

int ballot_walk_blocks_per_cu(const BatchedPlan &plan, size_t lds)
{
    if (plan.coarse) return plan.narrow && plan.packed ? ballot_occupancy_t<uint16_t, true, true>(plan, lds) : 0;
    if (plan.narrow)
        return plan.packed ? ballot_occupancy_t<uint16_t, true, false>(plan, lds)
                           : ballot_occupancy_t<uint16_t, false, false>(plan, lds);
    return ballot_occupancy_t<uint32_t, false, false>(plan, lds);
}

}  // namespace wmh
