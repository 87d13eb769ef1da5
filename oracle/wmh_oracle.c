/*
 * CPU oracle for rejection-sampling weighted minwise hashing over the red-green map
 * (Shrivastava, "Exact Weighted Minwise Hashing in Constant Time", arXiv 1602.08393).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product library never links, includes or calls anything here, and
 * nothing here includes or calls the product library.
 *
 * What it computes, in the paper's order:
 *   - Procedure (Sec. 3.1): bounds m_i, prefix sums M_i, the interval [0, M) cut into D pieces
 *     of size m_i; piece i is green on its first x_i units and red on the rest (eq. redGreen).
 *   - Algorithm 3 / Definition 1: for hash j draw positions r_1, r_2, ... uniformly in [0, M);
 *     the hash is the 1-based index of the first draw that lands in the green region.
 *   - ISGREEN by binary search over the row's sorted, disjoint green intervals (Sec. 3.3, the
 *     O(log d) variant the paper describes before its O(1) hashmaps).
 *   - Estimator (eq. Estimator): collision count over k hashes, divided by k.
 *
 * Readings where the paper leaves a choice open (each is listed in the design notes):
 *   - integer positions: with integer bounds and weights, a uniform real r in [0, M) lies in
 *     [M_i, M_i + x_i) exactly when floor(r) does, so positions are integers p in {0..M-1},
 *     intervals are half-open, and the test is  p - M_i < x_i;
 *   - the consistent random sequence is counter based: step t of hash j takes 64 bits from the
 *     Philox4x32-10 block at counter ((t-1)/2, j, a, 0) under key (seed lo, seed hi), the low
 *     64 bits for odd t and the high 64 bits for even t; a = 0, 1, 2, ... is the redraw index;
 *   - the bounded draw is Lemire's multiply-and-reject, exactly uniform on {0..M-1};
 *   - hash values are 1-based (Definition 1, Theorem 2 gives E[h] = 1/s), capped at 65535
 *     (h = cap when no green draw occurred in the first cap-1 draws), and an empty row hashes
 *     to 0 for every j.
 */
#include <errno.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WO_DEFAULT_CAP 65535u

/* status codes of the oracle (independent of the product's) */
#define WO_OK 0
#define WO_BAD_ARG 1
#define WO_BAD_COL 2     /* column index >= D */
#define WO_UNSORTED 3    /* columns not strictly increasing inside a row */
#define WO_OVER_BOUND 4  /* x_i > m_i */
#define WO_BAD_ROWPTR 5  /* row_ptr decreasing or beyond nnz */
#define WO_NOMEM 6

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as     */
/* 1, 2, 3" (SC'11): ten rounds of two 32x32->64 products with the round multipliers, the      */
/* high halves xored with the other two counter words and the round key; the key advances by   */
/* the Weyl constants between rounds.                                                          */
/* ------------------------------------------------------------------------------------------ */
void wo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prod0 = (uint64_t)mult0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)mult1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------------------------ */
/* Bounded draw (Lemire, "Fast random integer generation in an interval", ACM TOMACS 2019).    */
/* u is a uniform word of `bits` bits (1..64), n the range size, 1 <= n <= 2^bits.  The       */
/* product u*n is split into its high part (the candidate) and its low `bits` bits; the       */
/* candidate is accepted iff the low part is at least 2^bits mod n, which leaves exactly       */
/* floor(2^bits / n) accepted words per value and makes the draw exactly uniform on {0..n-1}.  */
/* Returns 1 and stores the value when accepted, 0 when the word is rejected.                  */
/* ------------------------------------------------------------------------------------------ */
int wo_bounded_draw(uint64_t u, uint64_t n, unsigned bits, uint64_t *value)
{
    if (bits == 0 || bits > 64 || n == 0) return 0;
    unsigned __int128 space = (unsigned __int128)1 << bits;
    if ((unsigned __int128)n > space) return 0;
    unsigned __int128 prod = (unsigned __int128)u * (unsigned __int128)n;
    unsigned __int128 low = prod % space;
    unsigned __int128 high = prod / space;
    unsigned __int128 threshold = space % n;
    if (low < threshold) return 0;
    *value = (uint64_t)high;
    return 1;
}

/* Position of step t (t >= 1) of hash j: a uniform integer in {0..M-1} drawn from the         */
/* counter-based sequence described in the header.  Returns the number of Philox blocks used.  */
uint64_t wo_position(uint64_t seed, uint32_t j, uint32_t t, uint64_t M, uint32_t *blocks_used)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t pair = (t - 1u) >> 1;
    uint32_t half = (t - 1u) & 1u;
    for (uint32_t attempt = 0;; ++attempt) {
        uint32_t ctr[4] = {pair, j, attempt, 0u};
        uint32_t w[4];
        wo_philox4x32_10(ctr, key, w);
        uint64_t u = ((uint64_t)w[2 * half + 1] << 32) | (uint64_t)w[2 * half];
        uint64_t p;
        if (wo_bounded_draw(u, M, 64, &p)) {
            if (blocks_used) *blocks_used = attempt + 1u;
            return p;
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Red-green map of one row: the sorted green intervals [M_i, M_i + x_i) of its nonzeros.      */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    uint64_t *start;   /* M_i of each nonzero component, increasing */
    uint64_t *length;  /* x_i of each nonzero component */
    uint64_t count;
    uint64_t green;    /* sum of x_i: the size of the green region */
} wo_row_map;

/* prefix sums: prefix[0] = 0, prefix[i+1] = prefix[i] + m[i]  (the paper's M_i) */
static void prefix_sums(const uint32_t *m, uint32_t D, uint64_t *prefix)
{
    prefix[0] = 0;
    for (uint32_t i = 0; i < D; ++i) prefix[i + 1] = prefix[i] + (uint64_t)m[i];
}

/* Validates one CSR row and builds its green intervals.  start/length must hold nnz entries. */
static int build_row_map(const uint64_t *prefix, const uint32_t *m, uint32_t D,
                         const uint32_t *col, const uint32_t *val, uint64_t nnz, wo_row_map *map)
{
    map->count = 0;
    map->green = 0;
    for (uint64_t e = 0; e < nnz; ++e) {
        uint32_t c = col[e];
        if (c >= D) return WO_BAD_COL;
        if (e > 0 && col[e - 1] >= c) return WO_UNSORTED;
        if (val[e] > m[c]) return WO_OVER_BOUND;
        if (val[e] == 0) continue; /* an all-red piece has no green interval */
        map->start[map->count] = prefix[c];
        map->length[map->count] = val[e];
        map->count++;
        map->green += val[e];
    }
    return WO_OK;
}

/* ISGREEN: binary search for the last interval starting at or before p, then check that p   */
/* lies inside it.  The intervals are disjoint and sorted because M_{i} + x_i <= M_{i+1}.     */
static int row_is_green(const wo_row_map *map, uint64_t p)
{
    uint64_t lo = 0, hi = map->count; /* find the number of intervals with start <= p */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (map->start[mid] <= p) lo = mid + 1;
        else hi = mid;
    }
    if (lo == 0) return 0;
    return p - map->start[lo - 1] < map->length[lo - 1];
}

/* Source of the draw sequence: either the counter-based generator, or an explicit list of     */
/* positions (used by the exact-enumeration tests; the list length is then the cap).          */
typedef struct {
    const uint64_t *explicit_positions;
    uint64_t seed;
    uint32_t j;
    uint64_t M;
} position_source;

static uint64_t source_position(const position_source *src, uint32_t t)
{
    if (src->explicit_positions) return src->explicit_positions[t - 1];
    return wo_position(src->seed, src->j, t, src->M, NULL);
}

/* Definition 1: the index of the first draw that is green, 0 for an empty row, `cap` when no  */
/* draw before the cap was green.                                                             */
static uint32_t first_green_step(const wo_row_map *map, const position_source *src, uint32_t cap)
{
    if (map->green == 0) return 0;
    for (uint32_t t = 1; t <= cap; ++t) {
        if (row_is_green(map, source_position(src, t))) return t;
    }
    return cap;
}

/* ------------------------------------------------------------------------------------------ */
/* Exported entry points                                                                       */
/* ------------------------------------------------------------------------------------------ */

/* ISGREEN of a single dense vector x (length D) at position p; -1 on invalid input.          */
int wo_is_green_dense(const uint32_t *m, const uint32_t *x, uint32_t D, uint64_t p)
{
    uint64_t *prefix = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint64_t *start = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint64_t *length = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint32_t *cols = malloc(sizeof(uint32_t) * ((size_t)D + 1));
    int result = -1;
    if (!prefix || !start || !length || !cols) goto done;
    prefix_sums(m, D, prefix);
    for (uint32_t i = 0; i < D; ++i) cols[i] = i;
    wo_row_map map = {start, length, 0, 0};
    if (build_row_map(prefix, m, D, cols, x, D, &map) != WO_OK) goto done;
    if (p >= prefix[D]) goto done;
    result = row_is_green(&map, p);
done:
    free(prefix); free(start); free(length); free(cols);
    return result;
}

/* Hash value of one dense vector x for an explicit position sequence (cap = n_positions).    */
/* Returns the hash (0..n_positions) or -1 on invalid input.                                   */
int64_t wo_hash_dense_positions(const uint32_t *m, const uint32_t *x, uint32_t D,
                                const uint64_t *positions, uint32_t n_positions)
{
    uint64_t *prefix = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint64_t *start = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint64_t *length = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    uint32_t *cols = malloc(sizeof(uint32_t) * ((size_t)D + 1));
    int64_t result = -1;
    if (!prefix || !start || !length || !cols || n_positions == 0) goto done;
    prefix_sums(m, D, prefix);
    for (uint32_t i = 0; i < D; ++i) cols[i] = i;
    wo_row_map map = {start, length, 0, 0};
    if (build_row_map(prefix, m, D, cols, x, D, &map) != WO_OK) goto done;
    for (uint32_t t = 0; t < n_positions; ++t)
        if (positions[t] >= prefix[D]) goto done;
    position_source src = {positions, 0, 0, prefix[D]};
    result = first_green_step(&map, &src, n_positions);
done:
    free(prefix); free(start); free(length); free(cols);
    return result;
}

typedef struct {
    const uint32_t *m;
    uint32_t D;
    const uint64_t *prefix;
    const uint64_t *row_ptr;
    const uint32_t *col;
    const uint32_t *val;
    uint64_t row_begin, row_end;
    uint32_t k;
    uint64_t seed;
    uint32_t cap;
    uint16_t *sig;
    uint64_t steps;      /* sum of returned hash values: the membership tests performed */
    int status;
    uint64_t bad_row;
} hash_job;

static void *hash_rows(void *arg)
{
    hash_job *job = (hash_job *)arg;
    uint64_t widest = 0;
    for (uint64_t r = job->row_begin; r < job->row_end; ++r) {
        uint64_t n = job->row_ptr[r + 1] - job->row_ptr[r];
        if (n > widest) widest = n;
    }
    uint64_t *start = malloc(sizeof(uint64_t) * (widest + 1));
    uint64_t *length = malloc(sizeof(uint64_t) * (widest + 1));
    if (!start || !length) {
        job->status = WO_NOMEM;
        free(start); free(length);
        return NULL;
    }
    uint64_t M = job->prefix[job->D];
    for (uint64_t r = job->row_begin; r < job->row_end; ++r) {
        uint64_t first = job->row_ptr[r], nnz = job->row_ptr[r + 1] - first;
        wo_row_map map = {start, length, 0, 0};
        int st = build_row_map(job->prefix, job->m, job->D, job->col + first, job->val + first,
                               nnz, &map);
        if (st != WO_OK) {
            job->status = st;
            job->bad_row = r;
            break;
        }
        for (uint32_t j = 0; j < job->k; ++j) {
            position_source src = {NULL, job->seed, j, M};
            uint32_t h = first_green_step(&map, &src, job->cap);
            job->sig[r * (uint64_t)job->k + j] = (uint16_t)h;
            job->steps += h;
        }
    }
    free(start);
    free(length);
    return NULL;
}

/* Hashes N CSR rows into sig[N*k] (row-major).  cap = 0 selects the default 65535.           */
/* Rows are split over n_threads POSIX threads.  On return *steps_out (if given) holds the sum */
/* of all hash values and *bad_row_out (if given) the first invalid row.                       */
int wo_hash_csr(const uint32_t *m, uint32_t D, const uint64_t *row_ptr, const uint32_t *col,
                const uint32_t *val, uint64_t n_rows, uint64_t nnz, uint32_t k, uint64_t seed,
                uint32_t cap, uint16_t *sig, int n_threads, uint64_t *steps_out,
                uint64_t *bad_row_out)
{
    if (!m || D == 0 || !row_ptr || (!sig && n_rows > 0) || k == 0) return WO_BAD_ARG;
    if (cap == 0) cap = WO_DEFAULT_CAP;
    if (cap > WO_DEFAULT_CAP) return WO_BAD_ARG;
    for (uint64_t r = 0; r < n_rows; ++r) {
        if (row_ptr[r] > row_ptr[r + 1] || row_ptr[r + 1] > nnz) {
            if (bad_row_out) *bad_row_out = r;
            return WO_BAD_ROWPTR;
        }
    }
    uint64_t *prefix = malloc(sizeof(uint64_t) * ((size_t)D + 1));
    if (!prefix) return WO_NOMEM;
    prefix_sums(m, D, prefix);
    if (prefix[D] == 0) {
        free(prefix);
        return WO_BAD_ARG;
    }
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n_rows) n_threads = n_rows ? (int)n_rows : 1;
    hash_job *jobs = calloc((size_t)n_threads, sizeof(hash_job));
    pthread_t *threads = calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !threads) {
        free(prefix); free(jobs); free(threads);
        return WO_NOMEM;
    }
    for (int t = 0; t < n_threads; ++t) {
        hash_job *job = &jobs[t];
        job->m = m; job->D = D; job->prefix = prefix; job->row_ptr = row_ptr;
        job->col = col; job->val = val; job->k = k; job->seed = seed; job->cap = cap;
        job->sig = sig;
        job->row_begin = n_rows * (uint64_t)t / (uint64_t)n_threads;
        job->row_end = n_rows * (uint64_t)(t + 1) / (uint64_t)n_threads;
        job->bad_row = UINT64_MAX;
    }
    int started = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&threads[t], NULL, hash_rows, &jobs[t]) != 0) break;
        started = t;
    }
    hash_rows(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(threads[t], NULL);
    /* rows of threads that could not be started are hashed here, in order */
    for (int t = started + 1; t < n_threads; ++t) hash_rows(&jobs[t]);
    int status = WO_OK;
    uint64_t steps = 0, bad_row = UINT64_MAX;
    for (int t = 0; t < n_threads; ++t) {
        steps += jobs[t].steps;
        if (jobs[t].status != WO_OK && status == WO_OK) {
            status = jobs[t].status;
            bad_row = jobs[t].bad_row;
        }
    }
    if (steps_out) *steps_out = steps;
    if (bad_row_out) *bad_row_out = bad_row;
    free(prefix); free(jobs); free(threads);
    return status;
}

/* Estimator: collisions between two signatures of length k, and count / k.                  */
uint32_t wo_collisions(const uint16_t *a, const uint16_t *b, uint32_t k)
{
    uint32_t count = 0;
    for (uint32_t j = 0; j < k; ++j) count += (a[j] == b[j]);
    return count;
}

double wo_estimate(const uint16_t *a, const uint16_t *b, uint32_t k)
{
    return (double)wo_collisions(a, b, k) / (double)k;
}

/* All-pairs counts: counts[i * nb + q] = collisions between row i of A and row q of B.        */
void wo_collisions_all_pairs(const uint16_t *A, uint64_t na, const uint16_t *B, uint64_t nb,
                             uint32_t k, uint32_t *counts)
{
    for (uint64_t i = 0; i < na; ++i)
        for (uint64_t q = 0; q < nb; ++q)
            counts[i * nb + q] = wo_collisions(A + i * (uint64_t)k, B + q * (uint64_t)k, k);
}
