// HIP kernels of the hash walk for gfx950: input validation, the plain per-lane walk, the
// shared position stream and the independent-rows walk (the shared-window walk has a file of
// its own).
//
// Work per (row, hash j): draw positions p_1, p_2, ... of hash j, map each to its component c
// and offset (Algorithm 5 with a uniform bucket table in place of Algorithm 4's per-integer
// map), and stop at the first t with offset < x_c (Algorithm 3, Definition 1).  Expected
// steps are 1/s with s = sum(x)/M (Theorem 2), so the step counts are geometric and the
// kernels are organised so that lanes do not idle on the long tails.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "wmh_entries.h"
#include "wmh_internal.h"

namespace wmh {

namespace {

__device__ __forceinline__ uint32_t lane() { return threadIdx.x & (kWave - 1u); }

// Index of this wavefront in its workgroup, in a scalar register.
__device__ __forceinline__ uint32_t wave_index()
{
    return (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t count_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// v of the lane the DPP control selects, or 0 where that lane lies outside the written rows
template <int kCtrl, int kRows>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRows, 0xF, false);
}

template <int kCtrl, int kRows>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t v)
{
    const uint64_t t = ((uint64_t)dpp_or_zero<kCtrl, kRows>((uint32_t)(v >> 32)) << 32) |
                       dpp_or_zero<kCtrl, kRows>((uint32_t)v);
    return v + t;
}

// Sum over the wavefront, in a scalar register: prefix sums inside 16-lane DPP rows (row
// shifts), then the row totals carried forward by row broadcasts; lane 63 ends with the sum.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
    v = dpp_add64<0x111, 0xF>(v);  // row_shr:1
    v = dpp_add64<0x112, 0xF>(v);  // row_shr:2
    v = dpp_add64<0x114, 0xF>(v);  // row_shr:4
    v = dpp_add64<0x118, 0xF>(v);  // row_shr:8
    v = dpp_add64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// ---------------------------------------------------------------------------------------------
// Validation: one wavefront per row, grid-stride over rows.  kKeys: also estimate the index
// keys (needed only when the component index is a candidate path).  Where the bounds m come
// from (kBounds): kBoundsGlobal gathers them from memory, kBoundsLds copies m to LDS first,
// kBoundsBlocks copies the per-block table (the smallest and the mean bound of each block of
// kBoundBlock components) to LDS: a value at or below its block's smallest bound passes without
// its own bound, only larger values gather theirs, and the index-key estimate takes the block
// means in place of the row's bounds (an estimate that only steers the path choice).
// ---------------------------------------------------------------------------------------------
constexpr int kBoundsGlobal = 0, kBoundsLds = 1, kBoundsBlocks = 2;

template <bool kKeys, int kBounds>
__global__ __launch_bounds__(1024) void validate_kernel(Rows rows, const uint32_t *__restrict__ bound_in,
                                                        const uint32_t *__restrict__ blocks_in,
                                                        uint32_t dims, uint64_t total,
                                                        double log_final, CheckWords *words,
                                                        RowSplit split)
{
    // per-workgroup partials, so each word gets at most one global atomic per workgroup
    __shared__ unsigned long long part_err[1024 / kWave], part_green[1024 / kWave],
        part_empty[1024 / kWave], part_walk[1024 / kWave], part_keys[1024 / kWave];
    // the per-class words of a row split: walk min green, walk rows, walk steps, index rows,
    // index nonzeros, index keys
    __shared__ unsigned long long part_split[6][1024 / kWave];
    // kBoundsLds: the workgroup first copies the bounds to LDS, so the check val <= m[col]
    // gathers from LDS instead of memory; kBoundsBlocks: the same for the block table
    extern __shared__ uint32_t lds_bound[];
    const uint32_t *bound = bound_in;
    const uint32_t n_blocks = (dims + kBoundBlock - 1) / kBoundBlock;
    if constexpr (kBounds == kBoundsLds) {
        for (uint32_t i = threadIdx.x; i < dims; i += blockDim.x) lds_bound[i] = bound_in[i];
        __syncthreads();
        bound = lds_bound;
    } else if constexpr (kBounds == kBoundsBlocks) {
        for (uint32_t i = threadIdx.x; i < 2 * n_blocks; i += blockDim.x) lds_bound[i] = blocks_in[i];
        __syncthreads();
    }
    const uint32_t *block_min = lds_bound, *block_mean = lds_bound + n_blocks;
    const uint32_t waves = blockDim.x / kWave;
    const uint64_t first = (uint64_t)blockIdx.x * waves + wave_index();
    const uint64_t stride = (uint64_t)gridDim.x * waves;
    uint64_t w_err = ~0ull, w_green = ~0ull, w_empty = 0;  // this wave's partials (uniform)
    uint64_t w_walk = 0, w_keys = 0;  // cost statistics: expected walk steps, green index keys
    uint64_t w_split[6] = {~0ull, 0, 0, 0, 0, 0};  // per-class statistics (row split)
    const bool classify = kKeys && split.row_class != nullptr;
    // M / sum(x) in double is exact after flooring while M < 2^53 (the rounding error of the
    // quotient stays below the distance 1 / sum(x) to the next integer)
    const bool exact_double = total < (1ull << 53);
    for (uint64_t r = first; r < rows.n_rows; r += stride) {
        const uint64_t lo = rows.row_ptr[r];
        const uint64_t hi = rows.row_ptr[r + 1];
        if (lo > hi || hi > rows.nnz) {
            w_err = min(w_err, (unsigned long long)((r << 4) | kCheckRowPtr));
            // a row split without the check still runs: the bad row gets a valid class byte
            if (classify && lane() == 0) split.row_class[r] = 0;
            continue;
        }
        uint64_t sum = 0, sum_m = 0;  // sum(x) and sum(m_c) over the row's nonzeros
        uint64_t bad = ~0ull;  // (entry << 4) | code of this lane's first bad entry
        // each lane checks a group of 4 consecutive entries per pass, groups aligned to
        // multiples of 4 entries so col and val load as 16-byte vectors (entries of the group
        // outside the row are skipped; at the arrays' end the loads go one by one)
        constexpr uint32_t kPer = 4;
        for (uint64_t g = (lo & ~(uint64_t)(kPer - 1)) + (uint64_t)lane() * kPer; g < hi;
             g += (uint64_t)kWave * kPer) {
            uint32_t c[kPer], v[kPer], m[kPer];
            if (g + kPer <= rows.nnz) {
                const uint4 cc = *reinterpret_cast<const uint4 *>(rows.col + g);
                const uint4 vv = *reinterpret_cast<const uint4 *>(rows.val + g);
                c[0] = cc.x; c[1] = cc.y; c[2] = cc.z; c[3] = cc.w;
                v[0] = vv.x; v[1] = vv.y; v[2] = vv.z; v[3] = vv.w;
            } else {
#pragma unroll
                for (uint32_t i = 0; i < kPer; ++i) {
                    const bool in = g + i < rows.nnz;
                    c[i] = in ? rows.col[g + i] : 0u;
                    v[i] = in ? rows.val[g + i] : 0u;
                }
            }
            const uint32_t prev = g > lo ? rows.col[g - 1] : 0u;
            uint32_t mk[kPer];  // the bound the index-key estimate takes
            if constexpr (kBounds == kBoundsBlocks) {
                // a value above its block's smallest bound gathers its own bound
#pragma unroll
                for (uint32_t i = 0; i < kPer; ++i) {
                    const uint32_t b = c[i] < dims ? block_min[c[i] / kBoundBlock] : 0u;
                    m[i] = c[i] < dims && v[i] > b ? bound_in[c[i]] : b;
                    mk[i] = c[i] < dims ? block_mean[c[i] / kBoundBlock] : 0u;
                }
            } else {
#pragma unroll
                for (uint32_t i = 0; i < kPer; ++i) mk[i] = m[i] = c[i] < dims ? bound[c[i]] : 0u;
            }
#pragma unroll
            for (uint32_t i = 0; i < kPer; ++i) {
                const uint64_t e = g + i;
                if (e < lo || e >= hi) continue;
                const uint32_t before = i ? c[i - 1] : prev;
                uint32_t code = 0;
                if (c[i] >= dims) code = kCheckColumn;
                else if (e > lo && before >= c[i]) code = kCheckUnsorted;
                else if (v[i] > m[i]) code = kCheckBound;
                if (code && bad == ~0ull) bad = ((e - lo) << 4) | code;
                sum += v[i];
                if (kKeys) sum_m += v[i] ? mk[i] : 0u;
            }
        }
        if (__builtin_amdgcn_ballot_w64(bad != ~0ull) != 0) {  // some entry of the row is bad
            w_err = min(w_err, (unsigned long long)((r << 4) | (wave_min(bad) & 15u)));
            if (classify && lane() == 0) split.row_class[r] = 0;
            continue;
        }
        sum = wave_sum(sum);
        if (sum == 0) {
            ++w_empty;
            if (classify) {
                ++w_split[1];  // empty rows go with the walk (signature 0)
                if (lane() == 0) split.row_class[r] = 0;
            }
            continue;
        }
        w_green = min(w_green, (unsigned long long)sum);
        // mean capped step count ~ min(1/s, cap) (Theorem 2)
        const uint64_t q = exact_double ? (uint64_t)floor((double)total / (double)sum) : total / sum;
        w_walk += min(q, (uint64_t)kCap);
        if (kKeys) {
            // index keys per hash: the cheaper of offset order (65534 * s) and step order up
            // to the row's final bound T2 (T2 * sum(m) / M), as the index row kernel chooses
            // (its first pass to T1 usually settles a step-order row with fewer keys; the
            // planner's costs were measured with this count)
            sum_m = wave_sum(sum_m);
            const double s = (double)sum / (double)total;
            const double T2 = index_step_bound(s, log_final);
            const double by_offset = 65534.0 * s;
            const double by_step = T2 < 65534.0 ? T2 * ((double)sum_m / (double)total) : by_offset;
            const uint64_t keys = (uint64_t)ceil(min(by_offset, by_step));
            w_keys += keys;
            if (classify) {
                // in units of one walk test: the walk's k * steps against the index's keys and
                // the nonzeros' list lookups
                const uint64_t steps = min(q, (uint64_t)kCap);
                const double walk_cost = (double)split.k * (double)steps;
                const double index_cost = (double)split.k * (double)keys * split.key_cost +
                                          (double)(hi - lo) * split.nnz_cost;
                const bool to_index = index_cost < walk_cost;
                if (lane() == 0) split.row_class[r] = to_index ? 1 : 0;
                if (to_index) {
                    ++w_split[3];
                    w_split[4] += hi - lo;
                    w_split[5] += keys;
                } else {
                    w_split[0] = min(w_split[0], sum);
                    ++w_split[1];
                    w_split[2] += steps;
                }
            }
        }
    }
    const uint32_t wave = wave_index();
    if (lane() == 0) {
        part_err[wave] = w_err;
        part_green[wave] = w_green;
        part_empty[wave] = w_empty;
        part_walk[wave] = w_walk;
        part_keys[wave] = w_keys;
        for (int i = 0; i < 6; ++i) part_split[i][wave] = w_split[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = ~0ull, g = ~0ull, n = 0, wk = 0, ky = 0;
        for (uint32_t w = 0; w < waves; ++w) {
            e = min(e, part_err[w]);
            g = min(g, part_green[w]);
            n += part_empty[w];
            wk += part_walk[w];
            ky += part_keys[w];
        }
        if (e != ~0ull) atomicMin(&words->first_error, e);
        if (g != ~0ull) atomicMin(&words->min_green, g);
        if (n) atomicAdd(&words->n_empty, n);
        if (wk) atomicAdd(&words->walk_steps, wk);
        if (ky) atomicAdd(&words->index_keys, ky);
        if (classify) {
            unsigned long long t[6] = {~0ull, 0, 0, 0, 0, 0};
            for (uint32_t w = 0; w < waves; ++w) {
                t[0] = min(t[0], part_split[0][w]);
                for (int i = 1; i < 6; ++i) t[i] += part_split[i][w];
            }
            if (t[0] != ~0ull) atomicMin(&words->walk_min_green, t[0]);
            if (t[1]) atomicAdd(&words->walk_rows, t[1]);
            if (t[2]) atomicAdd(&words->walk_class_steps, t[2]);
            if (t[3]) atomicAdd(&words->index_rows, t[3]);
            if (t[4]) atomicAdd(&words->index_nnz, t[4]);
            if (t[5]) atomicAdd(&words->index_class_keys, t[5]);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Plain walk: one wavefront per row, `waves` rows per workgroup.  Each lane walks one
// (row, hash) pair with its own draws; a lane that stops takes the next hash id of its row
// (ballot refill), so lanes stay busy until the row's last k ids are in flight.
// ---------------------------------------------------------------------------------------------
template <typename XT, bool kDense>
__global__ __launch_bounds__(256) void plain_kernel(Bounds b, Rows rows, uint64_t row_begin,
                                                    uint64_t row_end, uint32_t k, uint64_t seed,
                                                    uint16_t *__restrict__ sig)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = wave_index();
    const uint64_t row = row_begin + (uint64_t)blockIdx.x * waves + wave;
    const bool live = row < row_end;
    const uint32_t D = b.dims;
    XT *x = reinterpret_cast<XT *>(smem) + (kDense ? (size_t)wave * D : 0);

    uint64_t lo = 0, hi = 0;
    if (live) {
        lo = rows.row_ptr[row];
        hi = rows.row_ptr[row + 1];
    }
    if (kDense) {
        for (uint32_t i = lane(); i < D; i += kWave) x[i] = 0;
        __syncthreads();
        for (uint64_t e = lo + lane(); e < hi; e += kWave) {
            const uint32_t c = rows.col[e];
            if (c < D) x[c] = (XT)rows.val[e];
        }
        __syncthreads();
    }
    if (!live) return;
    uint64_t green = 0;
    for (uint64_t e = lo + lane(); e < hi; e += kWave) green += rows.val[e];
    green = wave_sum(green);

    uint16_t *out = sig + row * (uint64_t)k;
    if (green == 0) {
        for (uint32_t j = lane(); j < k; j += kWave) out[j] = 0;
        return;
    }

    uint32_t j = lane();
    uint32_t t = 0;
    uint64_t next_even = 0;  // position of the even step of the current pair
    uint32_t next_id = kWave;
    bool active = j < k;
    while (true) {
        bool done = false;
        if (active) {
            ++t;
            uint64_t p;
            if (t & 1u) position_pair(seed, j, (t - 1u) >> 1, b.total, b.threshold, &p, &next_even);
            else p = next_even;
            uint64_t off;
            const uint32_t c = component_of(p, b.prefix, b.bucket, b.shift, &off);
            uint32_t xc;
            if (kDense) {
                xc = x[c];
            } else {
                // binary search of c among the row's sorted columns (global memory)
                uint64_t a = lo, z = hi;
                while (a < z) {
                    const uint64_t mid = (a + z) >> 1;
                    if (rows.col[mid] < c) a = mid + 1;
                    else z = mid;
                }
                xc = (a < hi && rows.col[a] == c) ? rows.val[a] : 0u;
            }
            done = off < (uint64_t)xc || t == kCap;
        }
        const uint64_t finished = __ballot(done);
        if (done) {
            out[j] = (uint16_t)t;
            j = next_id + count_below(finished);
            t = 0;
            active = j < k;
        }
        next_id += (uint32_t)__popcll(finished);
        if (!__any(active)) break;
    }
}

// ---------------------------------------------------------------------------------------------
// Shared position stream: entry j * depth + t - 1 holds step t of hash j, for t <= depth:
// wide entries (component c, offset); packed entries (offset << 16) | (c * scale), where
// c * scale is the LDS byte offset of component c's group of dense-row values; coarse entries
// (code << 16) | (c * scale) with the offset's coarse code (odd, see coarse_q).  One thread per
// Philox block (two steps).
// ---------------------------------------------------------------------------------------------
template <bool kPacked, bool kCoarse>
__global__ __launch_bounds__(256) void stream_kernel(Bounds b, uint64_t seed, uint32_t k,
                                                     uint32_t depth, uint32_t scale,
                                                     void *__restrict__ entries,
                                                     uint32_t coarse_bits)
{
    static_assert(kPacked || !kCoarse, "coarse codes come in packed entries");
    const uint64_t pairs = depth >> 1;
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= pairs * k) return;
    const uint32_t j = (uint32_t)(idx / pairs);
    const uint32_t pair = (uint32_t)(idx - (uint64_t)j * pairs);
    uint64_t p0, p1, off0, off1;
    position_pair(seed, j, pair, b.total, b.threshold, &p0, &p1);
    const uint32_t c0 = component_of(p0, b.prefix, b.bucket, b.shift, &off0);
    const uint32_t c1 = component_of(p1, b.prefix, b.bucket, b.shift, &off1);
    const uint64_t at = (uint64_t)j * depth + 2ull * pair;
    if (kPacked) {
        uint32_t v0 = (uint32_t)off0, v1 = (uint32_t)off1;
        if (kCoarse) {
            v0 = coarse_offset_code(v0, b.bound[c0], coarse_bits);
            v1 = coarse_offset_code(v1, b.bound[c1], coarse_bits);
        }
        uint32_t *e = reinterpret_cast<uint32_t *>(entries) + at;
        *reinterpret_cast<uint2 *>(e) = make_uint2((v0 << 16) | (c0 * scale),
                                                   (v1 << 16) | (c1 * scale));
    } else {
        StreamEntry *e = reinterpret_cast<StreamEntry *>(entries) + at;
        e[0] = StreamEntry{c0, (uint32_t)off0};
        e[1] = StreamEntry{c1, (uint32_t)off1};
    }
}

// The sequence with its lookup, written out: same device functions as stream_kernel.
__global__ __launch_bounds__(256) void draws_kernel(Bounds b, uint64_t seed, uint32_t j0,
                                                    uint32_t n_hashes, uint32_t depth,
                                                    uint64_t *pos, uint32_t *comp, uint64_t *off)
{
    const uint64_t pairs = (depth + 1u) >> 1;
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= pairs * n_hashes) return;
    const uint32_t jj = (uint32_t)(idx / pairs);
    const uint32_t pair = (uint32_t)(idx - (uint64_t)jj * pairs);
    uint64_t p[2], o[2];
    uint32_t c[2];
    position_pair(seed, j0 + jj, pair, b.total, b.threshold, &p[0], &p[1]);
    c[0] = component_of(p[0], b.prefix, b.bucket, b.shift, &o[0]);
    c[1] = component_of(p[1], b.prefix, b.bucket, b.shift, &o[1]);
    for (int h = 0; h < 2; ++h) {
        const uint32_t t = 2u * pair + (uint32_t)h + 1u;
        if (t > depth) break;
        const uint64_t i = (uint64_t)jj * depth + t - 1u;
        if (pos) pos[i] = p[h];
        if (comp) comp[i] = c[h];
        if (off) off[i] = o[h];
    }
}

// ---------------------------------------------------------------------------------------------
// Independent rows (R = 4): the tiles, LDS rows and shared stream of batched_kernel, but each
// row of a block walks its own hash ids.  batched_kernel tests every window for all R rows until
// the block's last row is green, so it tests about E[max of R step counts] per row instead of
// E[one] (x2.5 at R = 4); here a row group of 16 lanes (one DPP row) stops at its own first
// green window and moves on to its next hash id.  Lane l serves row r = l / 16 and steps
// base_r + (l mod 16) * 4 + 1 .. + 4 of the row's current hash id j_r; wave w of the workgroup
// takes the hash ids j0 + w, j0 + w + W, ... of every row of the tile.
// ---------------------------------------------------------------------------------------------

// Minimum of c over lanes i-15 .. i of the lane's 16-lane row (a prefix scan); lanes whose
// source lies outside the row keep their value.  Lane 15 of each row ends with the row minimum.
template <int S>
__device__ __forceinline__ uint32_t row16_scan_min(uint32_t c)
{
    const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)c, 0x110 + S,
                                                             0xF, 0xF, false);
    return min(c, t);
}

// Every 16-bit segment of g that is nonzero, as a full segment of ones.
__device__ __forceinline__ uint64_t nonzero_segments16(uint64_t g)
{
    constexpr uint64_t kHigh = 0x8000800080008000ull, kLow = ~kHigh;
    const uint64_t h = (((g & kLow) + kLow) | g) & kHigh;  // no carry leaves a segment
    return h | (h - (h >> 15));
}

__device__ __forceinline__ bool lane_bit(uint64_t mask) { return ((mask >> lane()) & 1ull) != 0; }

template <typename XT, bool kPacked>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void rows_kernel(
    Bounds b, Rows rows, uint32_t k, uint64_t seed, uint16_t *__restrict__ sig,
    uint32_t hashes_per_tile, uint32_t depth, const void *__restrict__ entries,
    unsigned long long *tile_counter)
{
    constexpr uint32_t R = 4, L = 16, K = 4;
    constexpr uint32_t kLastBase = kCap + 1u - kWave;  // window of steps 65473 .. 65536
    constexpr uint32_t kNone = 0xFFFFu;                // no green step in the lane's steps
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long tile_slot;
    __shared__ uint32_t nonempty;
    const uint32_t D = b.dims;
    XT *x = reinterpret_cast<XT *>(smem);
    uint16_t *hbuf = reinterpret_cast<uint16_t *>(smem + (((size_t)D * R * sizeof(XT) + 15) & ~(size_t)15));
    const uint32_t my_row = lane() / L;
    const uint32_t gk = (lane() % L) * K;  // first of the lane's K steps inside a window
    using Layout = RowLayout<XT, R>;
    constexpr uint32_t kScale = Layout::kGroup;
    const uint32_t row_byte = Layout::row_byte(my_row, D);
    const uint32_t waves = blockDim.x / kWave;
    const uint32_t wave = wave_index();
    const uint32_t last_base = depth - kWave;

    const uint64_t n_blocks = (rows.n_rows + R - 1) / R;
    const uint32_t n_hash_tiles = (k + hashes_per_tile - 1) / hashes_per_tile;
    const uint64_t n_tiles = n_blocks * n_hash_tiles;
    uint64_t staged = ~0ull;
    bool claimed = false;

    while (true) {
        if (threadIdx.x == 0) tile_slot = next_tile(tile_counter, claimed);
        __syncthreads();
        const uint64_t tile = tile_slot;
        if (tile >= n_tiles) break;
        const uint64_t blk = tile / n_hash_tiles;
        const uint32_t ht = (uint32_t)(tile - blk * n_hash_tiles);
        const uint64_t row0 = blk * R;
        const uint32_t n_here = (uint32_t)min((uint64_t)R, rows.n_rows - row0);

        if (blk != staged) {
            uint32_t *xz = reinterpret_cast<uint32_t *>(x);
            const uint32_t words = (uint32_t)(((size_t)D * R * sizeof(XT) + 3) / 4);
            for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) xz[i] = 0u;
            if (threadIdx.x == 0) nonempty = 0;
            __syncthreads();
            uint32_t mine = 0;
            for (uint32_t r = 0; r < n_here; ++r) {
                const uint64_t lo = rows.row_ptr[row0 + r], hi = rows.row_ptr[row0 + r + 1];
                for (uint64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
                    const uint32_t v = rows.val[e];
                    const uint32_t c = rows.col[e];
                    if (c < D) *Layout::at(smem, c, r, D) = (XT)v;
                    if (v) mine |= 1u << r;
                }
            }
            if (mine) atomicOr(&nonempty, mine);
            __syncthreads();
            staged = blk;
        }
        const uint32_t live = __builtin_amdgcn_readfirstlane(nonempty);
        const uint32_t j0 = ht * hashes_per_tile;
        const uint32_t j1 = min(k, j0 + hashes_per_tile);

        // the row's current hash id (rows without a green unit start past the end) and window
        uint32_t jr = ((live >> my_row) & 1u) ? j0 + wave : j1;
        uint32_t base = 0;
        // entry index of window 0 of id jr (jr * depth, kept by addition: the whole stream has
        // fewer than 2^32 entries); loads clamp it to the last id, so finished rows read
        // in-bounds entries and ignore them
        const uint32_t id_step = waves * depth;
        const uint32_t last_id = (k - 1u) * depth;
        uint32_t jbase = min(jr, k - 1u) * depth;
        auto fetch = [&](uint32_t first, uint32_t at) {
            EntryRun<K, kPacked> run;
            run.load(entries, (uint64_t)(min(first, last_id) + min(at, last_base) + gk));
            return run;
        };
        // cur: the window to test; nxt: the next window of the same id; nid: the first window
        // of the row's next id (jr + waves)
        EntryRun<K, kPacked> cur = fetch(jbase, 0), nxt = fetch(jbase, kWave),
                             nid = fetch(jbase + id_step, 0);
        uint64_t active = __ballot(jr < j1);
        while (active != 0) {
            uint32_t c = kNone;  // position in the window of this lane's first green step
            {
                uint32_t xv[K], off[K];
#pragma unroll
                for (int q = 0; q < (int)K; ++q) {
                    uint32_t lds;
                    cur.get(q, kScale, &lds, &off[q]);
                    xv[q] = *reinterpret_cast<const XT *>(smem + lds + row_byte);
                }
#pragma unroll
                for (int q = K - 1; q >= 0; --q) c = off[q] < xv[q] ? gk + (uint32_t)q : c;
            }
            if (base >= depth) {
                // beyond the stream (rare): draw in-lane, one step at a time
                c = kNone;
#pragma unroll 1
                for (int q = K - 1; q >= 0; --q) {
                    const uint32_t t = base + gk + (uint32_t)q + 1u;
                    const uint64_t p = position(seed, jr, t, b.total, b.threshold);
                    uint64_t o64;
                    const uint32_t comp = component_of(p, b.prefix, b.bucket, b.shift, &o64);
                    c = o64 < (uint64_t)*reinterpret_cast<const XT *>(smem + (size_t)comp * kScale + row_byte) ? gk + (uint32_t)q : c;
                }
            }
            const uint64_t at_last = __ballot(base == kLastBase);
            if (at_last) {
                // step 65536 (the last step of the row's last lane) does not count
                if (base == kLastBase && c == kWave - 1u) c = kNone;
            }
            const uint64_t green = __ballot(c != kNone);
            const uint64_t done = (nonzero_segments16(green) | at_last) & active;
            uint32_t m = c;
            m = row16_scan_min<1>(m);
            m = row16_scan_min<2>(m);
            m = row16_scan_min<4>(m);
            m = row16_scan_min<8>(m);
            const bool is_done = lane_bit(done);
            if (is_done && gk == kWave - K) {
                // lane 15 of a finished row holds the row's first green position
                hbuf[my_row * hashes_per_tile + (jr - j0)] =
                    (uint16_t)(m == kNone ? kCap : base + m + 1u);
            }
#pragma unroll
            for (int i = 0; i < EntryRun<K, kPacked>::kWords; ++i)
                cur.w[i] = is_done ? nid.w[i] : nxt.w[i];
            jr = is_done ? jr + waves : jr;
            jbase = is_done ? jbase + id_step : jbase;
            base = is_done ? 0u : base + kWave;
            // the loads below reuse the registers the select has just read: keep them after it,
            // so they stay in flight for a whole iteration and nothing copies them
            __builtin_amdgcn_sched_barrier(0);
            nxt = fetch(jbase, base + kWave);
            nid = fetch(jbase + id_step, 0);
            active = __ballot(jr < j1);
        }
        __syncthreads();
        const uint32_t width = j1 - j0;
        for (uint32_t r = 0; r < n_here; ++r) {
            uint16_t *out = sig + (row0 + r) * (uint64_t)k + j0;
            const bool row_live = ((live >> r) & 1u) != 0;
            for (uint32_t q = threadIdx.x; q < width; q += blockDim.x)
                out[q] = row_live ? hbuf[r * hashes_per_tile + q] : (uint16_t)0;
        }
        __syncthreads();
    }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// ---------------------------------------------------------------------------------------------
// Row-aligned pair estimates (eq. Estimator): one wavefront per pair.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void estimate_kernel(const uint16_t *__restrict__ A,
                                                       const uint16_t *__restrict__ B,
                                                       uint64_t n_pairs, uint32_t k,
                                                       uint32_t *count, double *jhat)
{
    const uint32_t waves = blockDim.x / kWave;
    const uint64_t first = (uint64_t)blockIdx.x * waves + wave_index();
    const uint64_t stride = (uint64_t)gridDim.x * waves;
    for (uint64_t i = first; i < n_pairs; i += stride) {
        const uint16_t *a = A + i * k;
        const uint16_t *bb = B + i * k;
        uint64_t n = 0;
        for (uint32_t j = lane(); j < k; j += kWave) n += (a[j] == bb[j]);
        n = wave_sum(n);
        if (lane() == 0) {
            if (count) count[i] = (uint32_t)n;
            if (jhat) jhat[i] = (double)n / (double)k;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------

hipError_t launch_validate(const Rows &rows, const uint32_t *bound, uint32_t dims, uint64_t total,
                           uint32_t k, bool want_keys, CheckWords *words, hipStream_t stream,
                           const RowSplit *split, const uint32_t *bound_blocks)
{
    const RowSplit sp = split ? *split : RowSplit{};
    if (sp.row_class && !want_keys) return hipErrorInvalidValue;
    if (rows.n_rows == 0) return hipSuccess;
    // the index's final step bound per row
    const double log_final = std::log(kIndexFinalMiss / (double)k);
    // bounds (or the block table) in LDS up to 76 KB: two workgroups of 16 wavefronts per CU
    // keep it fully occupied (measured on the histogram workload: 268 -> 174 us)
    const uint32_t n_blocks = (dims + kBoundBlock - 1) / kBoundBlock;
    const int mode = (size_t)dims * 4 <= kValidateLdsMax ? kBoundsLds
                     : bound_blocks && (size_t)n_blocks * 8 <= kValidateLdsMax ? kBoundsBlocks
                                                                               : kBoundsGlobal;
    static bool configured = false;
    if (mode != kBoundsGlobal && !configured) {
        for (const void *f : {(const void *)validate_kernel<true, kBoundsLds>,
                              (const void *)validate_kernel<false, kBoundsLds>,
                              (const void *)validate_kernel<true, kBoundsBlocks>,
                              (const void *)validate_kernel<false, kBoundsBlocks>}) {
            const hipError_t e = hipFuncSetAttribute(
                f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kValidateLdsMax);
            if (e != hipSuccess) return e;
        }
        configured = true;
    }
    const uint32_t threads = mode != kBoundsGlobal ? 1024 : 256;
    const uint64_t waves_needed = rows.n_rows;
    const uint32_t per_block = threads / kWave;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((waves_needed + per_block - 1) / per_block,
                                                       8192 / per_block);
    const size_t shm = mode == kBoundsLds      ? (size_t)dims * 4
                       : mode == kBoundsBlocks ? (size_t)n_blocks * 8
                                               : 0;
#define WMH_VALIDATE(KEYS, MODE)                                                                  \
    validate_kernel<KEYS, MODE><<<grid, threads, shm, stream>>>(rows, bound, bound_blocks, dims,  \
                                                                total, log_final, words, sp)
    if (want_keys) {
        if (mode == kBoundsLds) WMH_VALIDATE(true, kBoundsLds);
        else if (mode == kBoundsBlocks) WMH_VALIDATE(true, kBoundsBlocks);
        else WMH_VALIDATE(true, kBoundsGlobal);
    } else {
        if (mode == kBoundsLds) WMH_VALIDATE(false, kBoundsLds);
        else if (mode == kBoundsBlocks) WMH_VALIDATE(false, kBoundsBlocks);
        else WMH_VALIDATE(false, kBoundsGlobal);
    }
#undef WMH_VALIDATE
    return hipGetLastError();
}

hipError_t launch_plain(const Bounds &b, const Rows &rows, uint64_t row_begin, uint64_t row_end,
                        uint32_t k, uint64_t seed, uint16_t *sig, bool narrow, bool dense,
                        hipStream_t stream)
{
    if (row_end <= row_begin) return hipSuccess;
    const uint32_t waves = 4;
    const uint64_t n = row_end - row_begin;
    const uint32_t grid = (uint32_t)((n + waves - 1) / waves);
    if (dense) {
        const size_t lds = (size_t)waves * b.dims * (narrow ? 2 : 4);
        if (narrow)
            plain_kernel<uint16_t, true><<<grid, waves * kWave, lds, stream>>>(b, rows, row_begin, row_end, k, seed, sig);
        else
            plain_kernel<uint32_t, true><<<grid, waves * kWave, lds, stream>>>(b, rows, row_begin, row_end, k, seed, sig);
    } else {
        plain_kernel<uint32_t, false><<<grid, waves * kWave, 0, stream>>>(b, rows, row_begin, row_end, k, seed, sig);
    }
    return hipGetLastError();
}

hipError_t launch_draws(const Bounds &b, uint64_t seed, uint32_t j0, uint32_t n_hashes,
                        uint32_t depth, uint64_t *pos, uint32_t *comp, uint64_t *off,
                        hipStream_t stream)
{
    const uint64_t threads = (uint64_t)n_hashes * ((depth + 1u) / 2u);
    if (threads == 0) return hipSuccess;
    draws_kernel<<<(uint32_t)((threads + 255) / 256), 256, 0, stream>>>(b, seed, j0, n_hashes,
                                                                      depth, pos, comp, off);
    return hipGetLastError();
}

hipError_t launch_stream_build(const Bounds &b, uint64_t seed, uint32_t k, uint32_t depth,
                               bool packed, uint32_t scale, uint32_t coarse_bits, void *entries,
                               hipStream_t stream)
{
    if (depth == 0 || k == 0) return hipSuccess;
    if (coarse_bits > kCoarseBits || (coarse_bits && !packed)) return hipErrorInvalidValue;
    const uint64_t threads = (uint64_t)k * (depth / 2);
    const uint32_t grid = (uint32_t)((threads + 255) / 256);
    if (coarse_bits)
        stream_kernel<true, true><<<grid, 256, 0, stream>>>(b, seed, k, depth, scale, entries, coarse_bits);
    else if (packed)
        stream_kernel<true, false><<<grid, 256, 0, stream>>>(b, seed, k, depth, scale, entries, 0u);
    else
        stream_kernel<false, false><<<grid, 256, 0, stream>>>(b, seed, k, depth, scale, entries, 0u);
    return hipGetLastError();
}

size_t batched_lds_bytes(uint32_t dims, const BatchedPlan &plan)
{
    const size_t xbytes = (size_t)dims * plan.rows_per_block * (plan.narrow ? 2 : 4);
    const size_t aligned = (xbytes + 15) & ~(size_t)15;
    // per-row hash values of a tile, then one spare slot per lane
    return aligned + ((size_t)plan.rows_per_block * plan.hashes_per_tile + kWave) * 2;
}

// Raises the kernel's dynamic LDS limit once per process; its launches return the status.
template <typename XT, bool kPacked>
static hipError_t configure_rows()
{
    static const hipError_t status =
        hipFuncSetAttribute((const void *)rows_kernel<XT, kPacked>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    return status;
}

template <typename XT, bool kPacked>
static int rows_occupancy_t(const BatchedPlan &plan, size_t lds)
{
    configure_rows<XT, kPacked>();
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, rows_kernel<XT, kPacked>,
                                                     plan.waves_per_block * kWave, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <typename XT, bool kPacked>
static hipError_t launch_rows_t(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                                uint16_t *sig, const BatchedPlan &plan, const void *entries,
                                unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    const size_t lds = batched_lds_bytes(b.dims, plan);
    const hipError_t e = configure_rows<XT, kPacked>();
    if (e != hipSuccess) return e;
    rows_kernel<XT, kPacked><<<grid, plan.waves_per_block * kWave, lds, stream>>>(
        b, rows, k, seed, sig, plan.hashes_per_tile, plan.stream_depth, entries, tile_counter);
    return hipGetLastError();
}

hipError_t launch_batched(const Bounds &b, const Rows &rows, uint32_t k, uint64_t seed,
                          uint16_t *sig, const BatchedPlan &plan, const void *entries,
                          unsigned long long *tile_counter, uint32_t grid, hipStream_t stream)
{
    if (batched_lds_bytes(b.dims, plan) > kMaxDynamicLds) return hipErrorInvalidValue;
    if (plan.packed && !plan.narrow) return hipErrorInvalidValue;
    // coarse codes: 16-bit rows, packed entries, the shared-window or ballot walk
    if (plan.coarse && (!plan.narrow || !plan.packed || plan.independent_rows ||
                        plan.coarse_bits == 0 || plan.coarse_bits > kCoarseBits))
        return hipErrorInvalidValue;
    // the shared walk reads whole three-window cycles of the stream (plus one spare cycle)
    if (plan.stream_depth % plan.cycle() != 0 || plan.stream_depth >= kCap) return hipErrorInvalidValue;
    if (plan.hash_groups > 1 && (!plan.ballot || plan.hash_groups > kMaxHashGroups ||
                                 !tile_counter ||
                                 (uint64_t)(plan.hash_groups - 1) * plan.hashes_per_tile >= k))
        return hipErrorInvalidValue;
    if (plan.ballot) {
        if (plan.rows_per_block != 1 || plan.steps_per_lane != 1 || plan.independent_rows)
            return hipErrorInvalidValue;
        return launch_ballot_walk(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
    }
    if (plan.independent_rows) {
        if (plan.rows_per_block != 4 || plan.stream_depth < kWave) return hipErrorInvalidValue;
        if (plan.narrow)
            return plan.packed ? launch_rows_t<uint16_t, true>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream)
                               : launch_rows_t<uint16_t, false>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
        return launch_rows_t<uint32_t, false>(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
    }
    return launch_shared_walk(b, rows, k, seed, sig, plan, entries, tile_counter, grid, stream);
}

int batched_blocks_per_cu(uint32_t dims, const BatchedPlan &plan)
{
    const size_t lds = batched_lds_bytes(dims, plan);
    if (lds > kMaxDynamicLds) return 0;
    if (plan.ballot) {
        if (plan.rows_per_block != 1 || plan.steps_per_lane != 1) return 0;
        return ballot_walk_blocks_per_cu(plan, lds);
    }
    if (plan.independent_rows) {
        if (plan.rows_per_block != 4 || plan.coarse) return 0;
        if (plan.narrow) return plan.packed ? rows_occupancy_t<uint16_t, true>(plan, lds)
                                            : rows_occupancy_t<uint16_t, false>(plan, lds);
        return rows_occupancy_t<uint32_t, false>(plan, lds);
    }
    return shared_walk_blocks_per_cu(plan, lds);
}

hipError_t launch_estimate(const uint16_t *A, const uint16_t *B, uint64_t n_pairs, uint32_t k,
                           uint32_t *count, double *jhat, hipStream_t stream)
{
    if (n_pairs == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n_pairs + 3) / 4, 8192);
    estimate_kernel<<<grid, 256, 0, stream>>>(A, B, n_pairs, k, count, jhat);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    fill_u32_kernel<<<(uint32_t)((n + 255) / 256), 256, 0, stream>>>(p, value, n);
    return hipGetLastError();
}

hipError_t launch_check_init(CheckWords *words, hipStream_t stream)
{
    uint32_t *w = reinterpret_cast<uint32_t *>(words);
    constexpr uint32_t kMinWords = 2 * kCheckMinima;
    hipError_t e = launch_fill_u32(w, 0xFFFFFFFFu, kMinWords, stream);
    if (e == hipSuccess) e = launch_fill_u32(w + kMinWords, 0u, sizeof(CheckWords) / 4 - kMinWords, stream);
    return e;
}

}  // namespace wmh
