/*
 * wmh.h -- C-ABI of libwmh: red-green weighted minwise hashing on AMD Instinct MI355X (gfx950).
 *
 * Method: A. Shrivastava, "Exact Weighted Minwise Hashing in Constant Time" (arXiv 1602.08393).
 * For a non-negative vector x with per-dimension integer bounds m_i, the interval [0, M),
 * M = sum m_i, is cut into D pieces of size m_i; piece i is green on its first x_i units and red
 * on the rest (Sec. 3.1, eq. redGreen).  Hash j of x is the 1-based index of the first position,
 * in a random sequence shared by every vector, that lands in x's green region (Algorithm 3,
 * Definition 1).  Two vectors collide on a hash with probability equal to their generalized
 * Jaccard similarity (eq. 1, Theorem 1); the collision count over k hashes estimates it
 * (eq. Estimator).
 *
 * Exact definition computed by this library (bit-exact, no floating point):
 *   P[0] = 0, P[i+1] = P[i] + m[i] (uint64), M = P[D] >= 1.
 *   Position of step t >= 1 of hash j: for attempt a = 0, 1, ...:
 *     W = Philox4x32-10(key = (seed & 0xffffffff, seed >> 32), counter = ((t-1)/2, j, a, 0));
 *     u = (W1 << 32 | W0) for odd t, (W3 << 32 | W2) for even t;
 *     prod = u * M (128-bit); accept iff (prod mod 2^64) >= (2^64 mod M); p = prod >> 64.
 *   c(p) = max{i : P[i] <= p}; p is green for x iff p - P[c(p)] < x[c(p)].
 *   h_j(x) = first green t, capped at 65535 (the walk stops there); 0 for every j if sum x = 0.
 *
 * Conventions for every call:
 *   - Every function returns a wmh_status and never throws or aborts across the ABI.
 *   - "device" pointers are HIP device allocations on the context's device (e.g. the
 *     data_ptr() of a torch tensor on that device); "host" pointers are ordinary host memory.
 *   - The caller owns every buffer it passes; the library keeps no reference after the call
 *     returns, except the bounds, which wmh_set_bounds copies into the context.
 *   - `stream` is a hipStream_t of the context's device, or NULL for the context's own stream.
 *   - A context is not thread-safe: use one context per host thread, or serialize calls.
 *     Its device scratch (tile and row counters, shared position stream, row classes of a
 *     split, captured graph) serves every call: asynchronous calls (opts->sync = 0) on different
 *     streams must be ordered by the caller; a call that reuses a stream built by an earlier
 *     call waits for that build.
 *   - On any error the output buffers are left untouched (validation precedes every write),
 *     and wmh_last_error() describes the failure (first offending row / column where known).
 */
#ifndef WMH_H
#define WMH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMH_CAP 65535u /* largest hash value; the walk stops at this step */

typedef struct wmh_ctx wmh_ctx;

typedef enum {
    WMH_OK = 0,
    WMH_E_ARG = -1,        /* invalid argument (null pointer, k = 0, sizes out of range) */
    WMH_E_NO_BOUNDS = -2,  /* wmh_hash before wmh_set_bounds */
    WMH_E_COL_RANGE = -3,  /* a column index >= D */
    WMH_E_UNSORTED = -4,   /* columns of a row not strictly increasing */
    WMH_E_BOUND = -5,      /* a value x_i above its bound m_i (never clamped) */
    WMH_E_OVERFLOW = -6,   /* bounds sum to 0, or sizes overflow */
    WMH_E_NOMEM = -7,      /* device or host allocation failed */
    WMH_E_DEVICE = -8,     /* a HIP runtime error */
    WMH_E_ROW_PTR = -9     /* row_ptr decreasing, or row_ptr[N] > nnz */
} wmh_status;

/* Scheduling of wmh_hash.  Every mode returns identical signatures. */
typedef enum {
    WMH_MODE_AUTO = 0,     /* the cheapest of the four below by a cost estimate from the
                              rows' statistics: expected walk steps min(M / sum x, 65535) per
                              hash (Theorem 2) against the index's nnz + 65534 * k * sum x / M
                              reads (the statistics come from the validation pass, which AUTO
                              runs, and waits for, even when validate = 0) */
    WMH_MODE_PLAIN = 1,    /* one launch per batch of `batch_rows` rows, a workgroup per row
                              group, each lane walking its own (row, hash) with its own draws */
    WMH_MODE_BATCHED = 2,  /* one persistent launch over (row block, hash block) tiles; each
                              draw is shared by the rows of a block (see wmh_hash) */
    WMH_MODE_INDEXED = 3   /* the capped sequence filed by component: every draw (j, t) with
                              t <= 65534 is listed under its component with its offset, once
                              per (bounds, seed, k) and kept in the context; a row's hash j is
                              the smallest t among the keys of its nonzero components whose
                              offset is below x_c, else 65535.  The same values as the walk, in
                              O(nnz + k * 65534 * sum x / M) per row: the choice for small
                              green fractions.  The lists are kept twice, by offset and by
                              step: a row whose hashes are small (large sum x / M) reads its
                              lists in step order up to a bound T1 with Pr(any hash > T1) <=
                              1/16 (Theorem 2), a row left with a hash id above T1 again up to
                              T2 with Pr(any hash > T2) <= 1e-4, and settles any hash id above
                              T2 in offset order, so the values stay exact.  Needs k <= 8192
                              and (k * 65534 + 16) * 16 bytes of device memory */,
    WMH_MODE_SPLIT = 4     /* each row on the cheaper of the two: the validation pass classes
                              every row by its own estimated costs (k * min(M / sum x, 65535)
                              walk tests against its index keys and list lookups), the batched
                              walk takes the walk rows (its stream sized for them alone) and
                              the component index the others.  For batches whose green
                              fractions spread over orders of magnitude.  Needs what BATCHED
                              and INDEXED need; the context keeps one byte per row */,
    WMH_MODE_PLAIN_SHARED = 5 /* BATCHED's kernels, plan and shared stream scheduled plainly:
                              one launch per batch of `batch_rows` rows, one workgroup per
                              (row block, hash block) tile, no tile counter, no graph.  It
                              isolates what persistence, the tile queue and the graph add to
                              the same per-step code.  Never chosen by AUTO */
} wmh_mode;

typedef struct {
    int32_t mode;          /* wmh_mode; default WMH_MODE_AUTO */
    uint32_t batch_rows;   /* plain modes: rows per launch; 0 = 8192 */
    int32_t validate;      /* 1 (default): validate the CSR input before hashing */
    int32_t use_graph;     /* batched mode: 1 (default) replay a captured hipGraph */
    int32_t sync;          /* 1 (default): wait for completion before returning */
    /* batched-mode tile plan overrides; 0 = planner / autotuner choice */
    uint32_t rows_per_block;   /* R: rows whose dense rows share one walk (1, 2, 4, 8, 16) */
    uint32_t hashes_per_tile;  /* J: hash ids per tile */
    uint32_t stream_depth;     /* T0: steps of the shared position stream (the draws and
                                  their components for steps t <= T0 of every hash id, built
                                  once per (seed, k, T0, bounds) and kept in the context);
                                  rounded up to whole cycles of three walk windows and kept
                                  below 65535; steps beyond it are drawn in-lane.  The
                                  planner's depth (0) keeps the stream within 1 GiB, and is 0
                                  when one cycle of k hash ids would exceed it (except for the
                                  independent-rows walk, which keeps one cycle).  UINT32_MAX:
                                  no stream (every step drawn in-lane; the independent-rows
                                  walk keeps one cycle) */
    uint32_t waves_per_block;  /* wavefronts per workgroup (1..16) */
    int32_t profile;           /* 1: time the walk kernels with HIP events on the launch stream
                                  (read back with wmh_last_kernel_ms) */
    int32_t walk;              /* batched mode: 0 = planner / autotuner choice (the planner takes
                                  the ballot walk when its blocks hold one row); 1 = shared windows
                                  (every window is tested for all R rows of a block until the
                                  block's last row is green); 2 = independent rows (each row of a
                                  block walks its own hash ids; needs R = 4); 3 = ballot walk
                                  (one row per block, a wavefront per hash id, lane l testing
                                  step l + 1 of each 64-step window; the first green step is the
                                  lowest set bit of the window's ballot; needs R = 1, K = 1) */
    uint32_t steps_per_lane;   /* batched mode, K: consecutive steps a lane tests per window;
                                  0 = R; R, or 4 when R < 4.  A window covers 64 / R * K steps
                                  of each of the block's R rows */
    /* component index rows kernel (indexed mode; waves_per_block above sets its wavefronts
       per workgroup, 1..16 with waves * k * 4 bytes <= 64 KiB); 0 = autotuned plan or the
       launcher's choice.  use_graph replays the kernel (and its counter reset) as a graph */
    uint32_t index_batch;      /* keys a lane loads per round trip: 8 or 16 */
    uint32_t index_claim;      /* 1: wavefronts claim rows from a counter; 2: a fixed stride */
    uint32_t hash_groups;      /* ballot walk: 0 = planner / autotuner choice; G in 1..8 cuts
                                  the hash ids into G blocks of ceil(k / G) (fewer when a block
                                  would be empty), each with its own tile counter; a workgroup
                                  starts on block blockIdx mod G, so the workgroups of one XCD
                                  (dispatched in turn) mostly read one block's part of the
                                  shared stream from their L2.  Each row is staged once per
                                  block.  1 = one counter over all tiles */
    int32_t values;            /* shared-window and ballot walks, the dense rows in LDS:
                                  0 = planner / autotuner choice (coarse codes when some bound
                                  is 65536 or more and a plan with them fits, else the values);
                                  1 = the values (uint16 when every bound is below 65536, else
                                  uint32); 2 = 16-bit coarse codes.  A code of a value and of a
                                  step's offset, both relative to the piece's bound m and
                                  ordered like the numbers (floor(y * 2^15 / m), with one bit
                                  telling the value's code whether the value is the first of
                                  its code), decides the step unless the two codes tie; a tie
                                  (probability below 2^-15 per tested step in the row's
                                  support; none when m <= 2^15) is settled from the row's
                                  exact value and the step's exact offset, so the hashes are
                                  identical.  Half the LDS of 32-bit rows and 4-byte stream
                                  entries; needs D * scale <= 65536 (D <= 32768 at R = 1,
                                  D <= 16384 at R = 2 or 4) and not the independent-rows walk */
    uint32_t coarse_bits;      /* resolution B of the coarse codes, 1..15; 0 = 15.  Codes are
                                  floor(y * 2^B / m); a tested step in the row's support ties
                                  with probability below 2^-B, so fewer bits only make ties (and
                                  their exact settling) frequent: the hashes stay identical */
} wmh_opts;

/* Fills *opts with the defaults listed above. */
void wmh_opts_init(wmh_opts *opts);

/* Creates a context on HIP device `device` (which becomes current for the calling thread). */
wmh_status wmh_create(int device, wmh_ctx **out);

/* Releases the context and every device buffer it owns.  NULL is ignored.  Destroy the
 * context's serving loops first. */
void wmh_destroy(wmh_ctx *ctx);

/*
 * wmh_set_bounds -- one-time preprocessing of the dataset bounds (Sec. 3.1; Algorithm 4).
 *   m : host, D entries, the integer upper bound m_i of dimension i (0 allowed: an empty piece).
 *   D : number of dimensions, 1 <= D <= 2^26.
 * Builds on the device the prefix sums P[0..D] (uint64), the total M = P[D] (must be >= 1),
 * the uniform bucket table T over [0, M) used for the O(1) position-to-component lookup
 * (Algorithm 5), and the bounded-draw threshold 2^64 mod M; for 19456 < D <= 311296 also the
 * smallest and the mean bound of each block of 32 dimensions, which the validation pass keeps
 * in LDS when m itself does not fit there.  Replaces earlier bounds; bounds
 * identical to the current ones change nothing (cached graphs and indexes stay valid).
 * Synchronous.  Errors: WMH_E_ARG (null, D out of range, a serving loop of this context is
 * alive), WMH_E_OVERFLOW (M = 0), WMH_E_NOMEM, WMH_E_DEVICE.
 */
wmh_status wmh_set_bounds(wmh_ctx *ctx, const uint32_t *m, uint32_t D);

/*
 * wmh_hash -- k weighted minwise hashes of each of N CSR rows (Algorithm 3, Definition 1).
 *   row_ptr : device, N+1 entries (uint64); row r is entries [row_ptr[r], row_ptr[r+1]).
 *   col     : device, nnz entries (uint32), strictly increasing within a row, < D.
 *   val     : device, nnz entries (uint32 fixed point), val <= m[col]; 0 allowed (red).
 *   n_rows  : N (0 allowed: nothing to do).   nnz : length of col and val.
 *   k       : hashes per row, 1 <= k <= 2^24.   seed : the 64-bit key of the random sequence.
 *   sig     : device, N*k uint16, row-major: sig[r*k + j] = h_j(row r); 0 for empty rows.
 *   stream  : hipStream_t or NULL.   opts : NULL for defaults.
 * The hash sequence depends only on (seed, j, t) and the bounds, never on the row, so rows can
 * be hashed in any grouping and order with identical results, and the signature for k1 < k2
 * is a prefix of the one for k2.
 * With opts->validate (default) the rows are checked on the device first and the call waits
 * for the verdict; on failure sig is untouched.  Errors: WMH_E_NO_BOUNDS, WMH_E_ARG,
 * WMH_E_ROW_PTR, WMH_E_COL_RANGE, WMH_E_UNSORTED, WMH_E_BOUND, WMH_E_NOMEM, WMH_E_DEVICE.
 * Without validation, invalid input gives unspecified signatures but never an out-of-bounds
 * access as long as row_ptr is non-decreasing with row_ptr[N] <= nnz.
 */
wmh_status wmh_hash(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                    const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k,
                    uint64_t seed, uint16_t *sig, void *stream, const wmh_opts *opts);

/*
 * wmh_hash_noalloc -- wmh_hash's batched walk for callers that cannot allocate device memory
 * during a call: code under hipGraph capture, tight serving loops, harnesses that forbid
 * allocation.  It allocates nothing (no hipMalloc, no hipFree, no allocating library call):
 * the tile counter, the validation words and the shared position stream live in one static
 * device array of WMH_NOALLOC_SCRATCH_BYTES per device, held from the first wmh_create on that
 * device until the process ends.  Arguments, layouts and results are those of wmh_hash, with
 * these differences:
 *   - opts->mode must be WMH_MODE_AUTO or WMH_MODE_BATCHED; both run the batched walk (no
 *     plain walk, no component index, no row split), launched directly (no graph).  The tile
 *     plan options and the autotuned plans apply as in wmh_hash.
 *   - The shared stream is rebuilt on every call inside the static array.  The planner's depth
 *     shrinks to what fits (steps past it are drawn in-lane, with identical values); a
 *     stream_depth given in opts, or the independent-rows walk's stream, whose bytes
 *     ((depth * k + 3 windows) * 4 or 8) exceed the array, is rejected with WMH_E_ARG.
 *   - Every call on one device shares the array and finds the last call's contents, which it
 *     re-initialises; calls that overlap on one device (other host threads, other streams with
 *     opts->sync = 0) race on it and must be ordered by the caller.
 * Errors: those of wmh_hash, plus WMH_E_ARG for another mode, a plan that does not fit in LDS,
 * or a stream beyond the array; WMH_E_DEVICE when the array's address could not be found.
 */
#define WMH_NOALLOC_SCRATCH_BYTES (16u << 20)
wmh_status wmh_hash_noalloc(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                            const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k,
                            uint64_t seed, uint16_t *sig, void *stream, const wmh_opts *opts);

/*
 * wmh_draws -- the position sequence itself and its component lookup (Algorithm 3's draws,
 * Algorithm 5's ISGREEN lookup), as the hash kernels compute them.  For hash ids
 * j0 <= j < j0 + n_hashes and steps 1 <= t <= depth, with i = (j - j0) * depth + t - 1:
 *   pos[i] = position of step t of hash j,  comp[i] = c(pos[i]),  off[i] = pos[i] - P[comp[i]].
 *   pos, comp, off : device buffers of n_hashes*depth entries (uint64, uint32, uint64); any
 *                    may be NULL.   Requires bounds.  Synchronous.
 * Errors: WMH_E_NO_BOUNDS, WMH_E_ARG (depth = 0 or > 65536, n_hashes = 0, j0 + n_hashes >
 * 2^32), WMH_E_DEVICE.
 */
wmh_status wmh_draws(wmh_ctx *ctx, uint64_t seed, uint32_t j0, uint32_t n_hashes, uint32_t depth,
                     uint64_t *pos, uint32_t *comp, uint64_t *off, void *stream);

/*
 * wmh_estimate -- collision-count estimates for row-aligned pairs (eq. Estimator):
 *   count[i] = #{j < k : A[i*k + j] == B[i*k + j]},  jhat[i] = count[i] / k (IEEE double).
 *   A, B  : device, n_pairs*k uint16 signatures.   count : device, n_pairs uint32 (or NULL).
 *   jhat  : device, n_pairs double (or NULL).       stream : hipStream_t or NULL.
 * Two empty rows (all-zero signatures) give jhat = 1.  Synchronous.
 * Errors: WMH_E_ARG, WMH_E_DEVICE.
 */
wmh_status wmh_estimate(wmh_ctx *ctx, const uint16_t *A, const uint16_t *B, uint64_t n_pairs,
                        uint32_t k, uint32_t *count, double *jhat, void *stream);

/*
 * wmh_estimate_pair -- the estimate for one pair of signatures held in host memory
 * (eq. Estimator):  *count = #{j < k : a[j] == b[j]},  *jhat = *count / k (IEEE double).
 *   a, b : host, k uint16 each (signatures as wmh_hash writes them).   count, jhat : host
 *   outputs (either may be NULL, not both).
 * Needs no context and touches no device; two empty rows (all-zero signatures) give jhat = 1.
 * Errors: WMH_E_ARG (null input, k = 0, both outputs NULL).
 */
wmh_status wmh_estimate_pair(const uint16_t *a, const uint16_t *b, uint32_t k, uint32_t *count,
                             double *jhat);

/*
 * wmh_collisions -- all-pairs collision counts (eq. Estimator's numerator):
 *   counts[a*NB + b] = #{j < k : A[a*k + j] == B[b*k + j]}  (exact uint32).
 *   A : device, NA*k uint16.  B : device, NB*k uint16.  counts : device, NA*NB uint32.
 * Synchronous.  Errors: WMH_E_ARG, WMH_E_DEVICE.
 */
wmh_status wmh_collisions(wmh_ctx *ctx, const uint16_t *A, uint64_t NA, const uint16_t *B,
                          uint64_t NB, uint32_t k, uint32_t *counts, void *stream);

/*
 * wmh_bounds_tables -- host-only: the tables wmh_set_bounds uploads (Sec. 3.1; Algorithm 4).
 *   m, D      : as for wmh_set_bounds (host).
 *   prefix    : host, D+1 uint64 (or NULL): P[0] = 0, P[i+1] = P[i] + m[i].
 *   bucket    : host, n_buckets+1 uint32 (or NULL): T[b] = max{i < D : P[i] <= b << shift}.
 *   shift     : out, log2 of the bucket width; the smallest shift giving at most
 *               2 * 2^ceil(log2 D) buckets (at least 4).
 *   n_buckets : out, ceil(M / 2^shift).   threshold : out, 2^64 mod M.
 * Call first with prefix = bucket = NULL to learn n_buckets.  No device is touched.
 * Errors: WMH_E_ARG, WMH_E_OVERFLOW (M = 0).
 */
wmh_status wmh_bounds_tables(const uint32_t *m, uint32_t D, uint64_t *prefix, uint32_t *bucket,
                             uint32_t *shift, uint64_t *n_buckets, uint64_t *threshold);

/*
 * wmh_last_kernel_ms -- device time of the last wmh_hash call made with opts->profile = 1,
 * from HIP events recorded on the launch stream.  Direct launches: *walk_ms spans the
 * hash-walk kernels (the batched kernel, or every plain launch), *stream_ms the shared-stream
 * build when that call built it (0 when it reused the stream of an earlier call, or had none).
 * hipGraph replays (batched with use_graph): *walk_ms spans the whole graph (counter reset
 * and walk) and *stream_ms is 0.  Indexed path: *walk_ms
 * spans the row kernel, *stream_ms the index build when that call built it (else 0).
 * Split path: *walk_ms spans the walk of the walk rows and the index rows kernel.
 * Requires that call to have completed (opts->sync, or a later synchronization).
 * Errors: WMH_E_ARG (no profiled call yet), WMH_E_DEVICE.
 */
wmh_status wmh_last_kernel_ms(wmh_ctx *ctx, float *walk_ms, float *stream_ms);

/*
 * wmh_last_mode -- the path the last successful wmh_hash on this context took:
 * WMH_MODE_PLAIN, WMH_MODE_BATCHED, WMH_MODE_INDEXED, WMH_MODE_SPLIT or WMH_MODE_PLAIN_SHARED
 * (WMH_MODE_AUTO before any call).
 * Errors: WMH_E_ARG (null).
 */
wmh_status wmh_last_mode(const wmh_ctx *ctx, int32_t *mode);

/*
 * wmh_last_plan -- the schedule of the last successful wmh_hash: plan->mode as wmh_last_mode,
 * and for the batched path the tile plan it ran (rows_per_block, hashes_per_tile,
 * stream_depth, waves_per_block, walk, steps_per_lane; 0 for the other paths); for the indexed
 * path the rows kernel's plan (waves_per_block, index_batch, index_claim; 0 = the launcher's
 * own choice).  Other fields are the defaults.
 * Errors: WMH_E_ARG (null).
 */
wmh_status wmh_last_plan(const wmh_ctx *ctx, wmh_opts *plan);

/* ------------------------------------------------------------------------------------------ */
/* b-bit signatures.  Hash values are geometric with mean 1/s (Theorem 2) and so small with    */
/* high probability (Corollary 1; Table 3 reports 5-9 bits on the paper's data).  Layout of a  */
/* packed row: f = floor(32 / bits) fields per uint32 word, W = ceil(k / f) words; value j is  */
/* in word j / f at bit (j mod f) * bits; unused bits and fields are 0; a value above          */
/* 2^bits - 1 is stored as 2^bits - 1 (saturated: lossless iff bits >= wmh_sig_bits).          */
/* ------------------------------------------------------------------------------------------ */

/* Words per packed row, ceil(k / floor(32 / bits)); 0 if bits is not in [1, 16] or k = 0.
 * Host only. */
uint32_t wmh_pack_words(uint32_t k, uint32_t bits);

/*
 * wmh_sig_bits -- the smallest width that packs these signatures losslessly: the least
 * bits >= 1 with max < 2^bits.  sig: device, N*k uint16.  *bits (host) receives it, *max_value
 * (host, may be NULL) the largest value.  Synchronous.  Errors: WMH_E_ARG, WMH_E_DEVICE.
 */
wmh_status wmh_sig_bits(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                        uint32_t *bits, uint32_t *max_value, void *stream);

/*
 * wmh_pack -- packs N signatures of k values into bits-wide fields (layout above).
 *   sig : device, N*k uint16.   packed : device, N*W uint32.   bits : 1..16.
 *   *n_saturated (host, may be NULL): how many values exceeded 2^bits - 1.  Synchronous.
 * Errors: WMH_E_ARG, WMH_E_DEVICE.
 */
wmh_status wmh_pack(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                    uint32_t bits, uint32_t *packed, uint64_t *n_saturated, void *stream);

/* wmh_unpack -- the inverse: sig (device, N*k uint16) from packed (device, N*W uint32);
 * saturated values come back as 2^bits - 1.  Synchronous.  Errors: WMH_E_ARG, WMH_E_DEVICE. */
wmh_status wmh_unpack(wmh_ctx *ctx, const uint32_t *packed, uint64_t n_rows, uint32_t k,
                      uint32_t bits, uint16_t *sig, void *stream);

/*
 * wmh_packed_collisions -- wmh_collisions on packed rows: counts[a*NB + b] = number of equal
 * fields of A row a and B row b (exact uint32); equals wmh_collisions on the unpacked values.
 * A : device, NA*W uint32.  B : device, NB*W uint32.  counts : device, NA*NB uint32.
 * Synchronous.  Errors: WMH_E_ARG, WMH_E_DEVICE.
 */
wmh_status wmh_packed_collisions(wmh_ctx *ctx, const uint32_t *A, uint64_t NA, const uint32_t *B,
                                 uint64_t NB, uint32_t k, uint32_t bits, uint32_t *counts,
                                 void *stream);

/* wmh_packed_estimate -- wmh_estimate on packed, row-aligned pairs (count and/or jhat, device).
 * Synchronous.  Errors: WMH_E_ARG, WMH_E_DEVICE. */
wmh_status wmh_packed_estimate(wmh_ctx *ctx, const uint32_t *A, const uint32_t *B,
                               uint64_t n_pairs, uint32_t k, uint32_t bits, uint32_t *count,
                               double *jhat, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* (K, L) banding index: the LSH consumer of the signatures (the paper's introduction: the k   */
/* hashes serve indexing for sublinear search).  Band b of a signature is its values at hash    */
/* ids [b*K, (b+1)*K); a database row is a candidate for a query when at least one band is     */
/* equal value for value.  Pairs whose hashes collide independently with probability J are     */
/* candidates with probability 1 - (1 - J^K)^L.                                                */
/* ------------------------------------------------------------------------------------------ */

typedef struct wmh_lsh wmh_lsh;

/*
 * wmh_lsh_build -- indexes N database signatures (device, N*k uint16) under K hashes per band
 * and L bands (K, L >= 1, K*L <= k, L <= 4096, N < 2^32 - 1).  The index copies the bands it
 * uses; sig may be freed afterwards.  Device memory: about N*L*(2K + 4) + 24*L*2^ceil(log2 2N)
 * bytes.  Synchronous.  Errors: WMH_E_ARG, WMH_E_NOMEM, WMH_E_DEVICE.
 */
wmh_status wmh_lsh_build(wmh_ctx *ctx, const uint16_t *sig, uint64_t n_rows, uint32_t k,
                         uint32_t K, uint32_t L, void *stream, wmh_lsh **out);

/*
 * wmh_lsh_query -- candidates of Q query signatures (device, Q*k uint16, the index's k):
 *   out_count[q] (device uint32) = number of distinct database rows sharing a band with query
 *   q, or 0xFFFFFFFF when its band matches (one per band and row) exceed 2048;
 *   out[q*max_out + i] (device uint32), i < min(out_count[q], max_out): those rows in
 *   increasing order.  Synchronous.  Errors: WMH_E_ARG (null, k differs), WMH_E_DEVICE.
 */
wmh_status wmh_lsh_query(wmh_lsh *ix, const uint16_t *query, uint64_t n_queries, uint32_t k,
                         uint32_t max_out, uint32_t *out, uint32_t *out_count, void *stream);

/* Releases the index.  NULL is ignored.  Destroy indexes before their context. */
void wmh_lsh_destroy(wmh_lsh *ix);

/* ------------------------------------------------------------------------------------------ */
/* Fixed-point scaling of real-valued data (Sec. 4, Practical Issues).  The expected step count */
/* is M / sum(x) (Theorem 2); scaling by alpha and rounding up the bounds gives                 */
/* alpha * sum(x) / sum(ceil(alpha * m_i)), which the paper asks to maximize.  sum(x) is a      */
/* common factor, so the best alpha depends on the bounds only.                                 */
/* ------------------------------------------------------------------------------------------ */

/*
 * wmh_choose_scale -- host only.  m: host, D real bounds (finite, >= 0, not all 0).  limit: the
 * largest integer bound allowed (65535 lets the batched walk keep 16-bit rows and 4-byte stream
 * entries; 0 = 2^32 - 1).  Searches alpha <= limit / max(m): the largest such scale and the
 * points n / m_i just below it (where alpha * m_i is an integer) for the `components` largest
 * bounds (0 = 8), `steps` points each (0 = 8), keeping the one with the largest
 * alpha / sum(ceil(alpha * m_i)).
 *   *alpha_out: the scale.   *efficiency (may be NULL): alpha * sum(m) / sum(ceil(alpha * m)),
 *   in (0, 1]: the expected step count grows by 1 / efficiency against unrounded bounds.
 *   m_q (host, D, may be NULL): ceil(alpha * m_i), the integer bounds to pass to wmh_set_bounds.
 * Errors: WMH_E_ARG (null, D = 0, a bound negative or not finite), WMH_E_OVERFLOW (all 0).
 */
wmh_status wmh_choose_scale(const double *m, uint32_t D, uint32_t limit, uint32_t components,
                            uint32_t steps, double *alpha_out, double *efficiency,
                            uint32_t *m_q);

/*
 * wmh_quantize -- real CSR values to the library's fixed point:
 *   out[e] = min(floor(alpha * x[e] + 1/2), m_q[col[e]]) with m_q the context's bounds (set
 *   from wmh_choose_scale's m_q); alpha * x and + 1/2 are IEEE double operations rounded one
 *   at a time, so a host computing the same expression gets the same integers.
 *   x : device, nnz float32 (>= 0; negative values give 0).   col : device, nnz uint32.
 *   out : device, nnz uint32.   *n_clipped (host, may be NULL): values above their bound
 *   (only possible when x exceeded the real bound).  Synchronous.
 * Errors: WMH_E_ARG, WMH_E_NO_BOUNDS, WMH_E_DEVICE.
 */
wmh_status wmh_quantize(wmh_ctx *ctx, const float *x, const uint32_t *col, uint64_t nnz,
                        double alpha, uint32_t *out, uint64_t *n_clipped, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Autotuner of the batched tile plan (scheduling only: every plan gives the same bytes).      */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    uint32_t rows_per_block;   /* R of the fastest plan */
    uint32_t hashes_per_tile;  /* J */
    uint32_t waves_per_block;  /* W */
    uint32_t stream_depth;     /* the planner's shared-stream depth used for every candidate */
    float best_ms;             /* device time of one wmh_hash call with that plan */
    float default_ms;          /* the same with the planner's default plan */
    uint32_t candidates;       /* plans timed */
    int32_t steps_class;       /* floor(log2(mean capped steps per hash)) of the rows */
    int32_t walk;              /* wmh_opts.walk of the fastest plan (1, 2 or 3), or 4 when
                                  the rows go to the component index and the index rows
                                  kernel's plan was tuned instead (waves_per_block,
                                  index_batch, index_claim) */
    uint32_t steps_per_lane;   /* K of the fastest plan */
    uint32_t index_batch;      /* walk 4: keys per round trip of the fastest plan */
    uint32_t index_claim;      /* walk 4: 1 counter, 2 fixed stride */
    uint32_t hash_groups;      /* ballot walk: hash groups of the fastest plan (1 otherwise) */
    int32_t values;            /* wmh_opts.values of the fastest plan: 1 values, 2 coarse
                                  codes (0 for the index rows kernel) */
    uint32_t reserved[2];
} wmh_tune_result;

/*
 * wmh_tune -- times the batched walk on the given rows (device CSR as for wmh_hash) under
 * candidate plans R in {1,2,4,8,16} x W in {4,8,16} x J in {min(k,1024), min(k,512),
 * min(k,256)} with shared windows and K = R, the same with K = 4 for R = 1 and 2, plus R = 4
 * with independent rows and R = 1 with the ballot walk for every W and J (and the ballot walk
 * with its hash ids in 2, 4 and 8 groups for every W), each
 * the best of `reps` (0 = 3) calls after one untimed call, and keeps the
 * fastest in the context under (D, value width, k, step class).  Later wmh_hash calls in the
 * batched, split or auto mode whose plan options are 0 run the plan of their rows' key, or else
 * of the same (D, width, k) at the nearest step class within two (the walk rows of a split
 * have a smaller one).  When the planner of the auto mode sends these rows to the component
 * index, the tuner instead builds the index and times its rows kernel under W in
 * {1,2,4,8,16} (as LDS allows) x keys per trip in {8,16} x row claims by counter or stride,
 * keeps the fastest under the same key for indexed and auto calls whose index options are 0,
 * and reports it with walk = 4.  sig (device, N*k uint16) receives the signatures.
 * Synchronous.  Errors: as wmh_hash, plus WMH_E_ARG when neither a batched plan nor the index
 * fits.
 */
wmh_status wmh_tune(wmh_ctx *ctx, const uint64_t *row_ptr, const uint32_t *col,
                    const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k, uint64_t seed,
                    uint16_t *sig, void *stream, uint32_t reps, wmh_tune_result *out);

/* Writes the context's tuned plans to a text file: a "wmh-tune 6" line, then one line per key
 * "D narrow k steps_class R J W walk K G V ms" (G: hash groups of the ballot walk, V: values
 * as in wmh_opts); for a plan of the index rows kernel walk is 4, R the keys per trip, J the
 * claim (1 counter, 2 stride), K 0, G 1 and V 0.  Errors: WMH_E_ARG. */
wmh_status wmh_tune_save(wmh_ctx *ctx, const char *path);

/* Adds the plans of a file written by wmh_tune_save (replacing equal keys); nothing is added
 * if any line is malformed.  Errors: WMH_E_ARG (missing or malformed file). */
wmh_status wmh_tune_load(wmh_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------------------------ */
/* Serving loop: continuous batching of hash requests on one device.                           */
/* ------------------------------------------------------------------------------------------ */

typedef struct wmh_server wmh_server;

typedef struct {
    uint32_t k;            /* hashes per row, 1 <= k <= 2^24 */
    uint32_t slots;        /* requests on the device at once, each on its own HIP stream;
                              1..64, 0 = 8 */
    uint64_t seed;         /* key of the random sequence */
    uint64_t mem_budget;   /* device bytes for the admitted requests' rows and signatures
                              ((N+1)*8 + nnz*8 + N*k*2 each); 0 = 4 GiB */
    int32_t mode;          /* wmh_mode of every request's walk; 0 = auto (a row split is not
                              available in the loop) */
    uint32_t stream_depth; /* steps of the shared position stream built once at creation;
                              0 = 8192, cut to stay within 1 GiB, and no stream when one cycle
                              of k hash ids exceeds that (steps beyond are drawn in-lane) */
    int32_t build_index;   /* 1: build the component index at creation (auto or indexed mode),
                              so no request waits for it; 0: on the first indexed request */
    uint32_t group_rows;   /* queued requests admitted together into one slot while their rows
                              add up to at most this (one validation pass, one walk or index
                              launch and one copy out for the group; every request's
                              signatures are the same as alone); 0 = 2048, 1 = one request
                              per slot */
    uint32_t reserved[2];
} wmh_server_config;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t queued;       /* requests waiting for admission at the time of the call */
    uint64_t max_queued;   /* largest such backlog seen */
    uint64_t peak_bytes;   /* largest device bytes admitted at once */
    uint64_t hashes;       /* rows * k over completed requests */
    double p50_ms, p99_ms, p999_ms, max_ms, mean_ms; /* arrival -> completion */
    double busy_s;         /* first admission -> last completion */
    double hashes_per_s;   /* hashes / busy_s */
    uint64_t rejected;     /* requests whose rows failed the device check (not in failed) */
    /* Overlap on the device, from HIP event timestamps on each slot's stream: a slot load (a
     * request, or requests admitted together) is on the device from its first copy in to the
     * end of its copy out, and computing from the start of its walk to the end of its copy
     * out (both include time its work waits in the device queues behind other slots' work). */
    uint64_t max_on_device;  /* most completed slot loads (a request, or requests admitted
                                together) on the device at one instant */
    uint64_t max_computing;  /* most completed slot loads computing at one instant */
    double overlap_s;        /* seconds during which at least two slot loads were computing */
    uint64_t loads;          /* completed slot loads (completed / loads: requests per load) */
} wmh_serving_stats;

/*
 * wmh_server_create -- starts a serving loop on ctx's device using ctx's bounds (which must
 * not change while the loop exists).  A worker thread admits queued requests in arrival order
 * whenever a slot is free and the admitted bytes stay within mem_budget (consecutive requests
 * up to group_rows rows together, as one group), runs each group's walk on its slot's stream
 * (so groups overlap on the device), and completes the requests as their results arrive.  A
 * group whose rows fail the device check completes the request with the first bad row with
 * that status and checks each of the others again alone; a group whose slot buffers cannot be
 * allocated is admitted again one request at a time.  Bounds, bucket table and the shared
 * position stream stay device-resident.
 * Errors: WMH_E_ARG, WMH_E_NO_BOUNDS, WMH_E_NOMEM, WMH_E_DEVICE.
 */
wmh_status wmh_server_create(wmh_ctx *ctx, const wmh_server_config *cfg, wmh_server **out);

/*
 * wmh_server_submit -- queues one request of N CSR rows (host buffers: row_ptr N+1, col/val
 * nnz) whose signatures go to sig (host, N*k uint16).  The caller keeps all four buffers valid
 * and unchanged until the request completes.  row_ptr is checked here (WMH_E_ROW_PTR); every
 * entry is checked on the device by wmh_hash's validation pass before any walk, and a request
 * that breaks a rule completes with that status (WMH_E_COL_RANGE, WMH_E_UNSORTED,
 * WMH_E_BOUND) from wmh_server_poll / wmh_server_wait, its sig untouched.  A request larger
 * than mem_budget is WMH_E_NOMEM.
 * arrival_ns is the request's arrival on wmh_server_now_ns()'s clock (0 = now); latency is
 * measured from it, so an open-loop driver that submits late does not hide queueing delay.
 * Each request's signatures are identical to a wmh_hash call on the same rows.
 */
wmh_status wmh_server_submit(wmh_server *srv, const uint64_t *row_ptr, const uint32_t *col,
                             const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint16_t *sig,
                             uint64_t arrival_ns, uint64_t *ticket);

/* Non-blocking completion test; *latency_ms (may be NULL) is set once done. */
wmh_status wmh_server_poll(wmh_server *srv, uint64_t ticket, int *done, double *latency_ms);

/* Blocks until the request completes. */
wmh_status wmh_server_wait(wmh_server *srv, uint64_t ticket, double *latency_ms);

/* Blocks until every submitted request has completed. */
wmh_status wmh_server_drain(wmh_server *srv);

/*
 * wmh_server_reserve -- sizes every slot's device buffers and page-locked staging buffers for
 * requests (or groups of requests) of up to max_rows rows and max_nnz nonzeros, so that
 * admitting them allocates nothing.  Without it a slot grows its buffers (by at least half) when a larger
 * request arrives, and freeing the old ones waits for the device, which delays every request
 * in flight.  Waits until every submitted request has completed.  Errors: WMH_E_ARG,
 * WMH_E_NOMEM (beyond mem_budget or device memory), WMH_E_DEVICE.
 */
wmh_status wmh_server_reserve(wmh_server *srv, uint64_t max_rows, uint64_t max_nnz);

/* Counters and latency percentiles over the completed requests. */
wmh_status wmh_server_stats(wmh_server *srv, wmh_serving_stats *out);

/* Starts the statistics afresh (latencies, counters, overlap), e.g. after a warm-up; requests
 * queued or on the device stay and count as submitted.  Errors: WMH_E_ARG. */
wmh_status wmh_server_reset_stats(wmh_server *srv);

/* The steady clock used for arrival times, in nanoseconds. */
uint64_t wmh_server_now_ns(void);

/*
 * wmh_host_alloc -- pinned (page-locked) host memory of `bytes` bytes for request buffers.
 * wmh_server_submit's copies of rows in and signatures out run as asynchronous DMA from and to
 * such buffers; from pageable buffers the copy in also works, but the loop's worker waits for
 * it.  *ptr receives the buffer (NULL for bytes = 0); release it with wmh_host_free after every
 * request using it has completed.  Errors: WMH_E_ARG (ptr NULL), WMH_E_NOMEM.
 */
wmh_status wmh_host_alloc(size_t bytes, void **ptr);

/* Releases a wmh_host_alloc buffer; NULL is ignored. */
void wmh_host_free(void *ptr);

/* Drains, stops the worker and releases every buffer.  NULL is ignored. */
void wmh_server_destroy(wmh_server *srv);

/* Bounds summary after wmh_set_bounds: D, M, bucket shift and bucket count (any may be NULL). */
wmh_status wmh_bounds_info(const wmh_ctx *ctx, uint32_t *D, uint64_t *M, uint32_t *shift,
                           uint64_t *n_buckets);

/* Human-readable detail of the last failure on this context ("" if none).  Valid until the
 * next call on the context. */
const char *wmh_last_error(const wmh_ctx *ctx);

/* Name of a status code. */
const char *wmh_status_string(wmh_status status);

#ifdef __cplusplus
}
#endif

#endif /* WMH_H */
