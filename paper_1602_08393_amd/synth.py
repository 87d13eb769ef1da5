"""Seeded synthetic inputs for red-green weighted minwise hashing.

This module only builds inputs: CSR rows of uint32 fixed-point weights and the per-dimension
integer bounds m_i (the dataset maximum of each dimension, at least 1).  It holds none of the
hashing arithmetic, so both the GPU library's tests and the CPU oracle can take their inputs
from it.

The paper measures on image histograms and HOG features that are not available here; the
workloads below are synthetic stand-ins with the shapes of the five benchmark configurations
(sizes, value distributions, sparsity and degree mix), each drawn from numpy's PCG64 with a fixed
seed (1000 + configuration number).
"""
from __future__ import annotations

import concurrent.futures
import os
from dataclasses import dataclass, field

import numpy as np

U32_MAX = 0xFFFFFFFF


@dataclass
class Dataset:
    """CSR rows plus bounds.  row_ptr u64[N+1], col u32[nnz], val u32[nnz], m u32[D]."""
    name: str
    m: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    k: int
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return int(self.m.shape[0])

    @property
    def n_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def rows(self, index) -> "Dataset":
        """A dataset made of the selected rows (same bounds)."""
        index = np.asarray(index, dtype=np.int64)
        starts = self.row_ptr[index].astype(np.int64)
        ends = self.row_ptr[index + 1].astype(np.int64)
        lengths = ends - starts
        row_ptr = np.zeros(len(index) + 1, dtype=np.uint64)
        row_ptr[1:] = np.cumsum(lengths)
        if len(index):
            gather = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)]) \
                if lengths.sum() else np.zeros(0, dtype=np.int64)
        else:
            gather = np.zeros(0, dtype=np.int64)
        return Dataset(self.name, self.m, row_ptr, self.col[gather].copy(),
                       self.val[gather].copy(), self.k, self.seed, dict(self.meta))

    def head(self, n: int) -> "Dataset":
        return self.rows(np.arange(min(n, self.n_rows)))

    def dense(self) -> np.ndarray:
        X = np.zeros((self.n_rows, self.D), dtype=np.uint32)
        rows = np.repeat(np.arange(self.n_rows), np.diff(self.row_ptr.astype(np.int64)))
        X[rows, self.col] = self.val
        return X


def csr_from_lists(cols_per_row, vals_per_row, D: int, m=None, name="custom", k=64, seed=0):
    lengths = np.array([len(c) for c in cols_per_row], dtype=np.int64)
    row_ptr = np.zeros(len(cols_per_row) + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(lengths)
    col = np.concatenate([np.asarray(c, dtype=np.uint32) for c in cols_per_row]) \
        if len(cols_per_row) and lengths.sum() else np.zeros(0, dtype=np.uint32)
    val = np.concatenate([np.asarray(v, dtype=np.uint32) for v in vals_per_row]) \
        if len(vals_per_row) and lengths.sum() else np.zeros(0, dtype=np.uint32)
    if m is None:
        m = dataset_max_bounds(col, val, D)
    return Dataset(name, np.asarray(m, dtype=np.uint32), row_ptr, col, val, k, seed)


def csr_from_dense(X, m=None, name="dense", k=64, seed=0) -> Dataset:
    X = np.atleast_2d(np.asarray(X, dtype=np.uint32))
    rows, cols = np.nonzero(X)
    row_ptr = np.zeros(X.shape[0] + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(np.bincount(rows, minlength=X.shape[0]))
    col = cols.astype(np.uint32)
    val = X[rows, cols].astype(np.uint32)
    if m is None:
        m = dataset_max_bounds(col, val, X.shape[1])
    return Dataset(name, np.asarray(m, dtype=np.uint32), row_ptr, col, val, k, seed)


def dataset_max_bounds(col: np.ndarray, val: np.ndarray, D: int) -> np.ndarray:
    """m_i = maximum of dimension i over the dataset, with a floor of 1."""
    m = np.ones(D, dtype=np.uint32)
    if len(col):
        np.maximum.at(m, col.astype(np.int64), val.astype(np.uint32))
    return m


def _assemble(col_chunks, val_chunks, lengths, D, name, k, seed, meta, m=None) -> Dataset:
    row_ptr = np.zeros(len(lengths) + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(np.asarray(lengths, dtype=np.int64))
    col = np.concatenate(col_chunks).astype(np.uint32) if col_chunks else np.zeros(0, np.uint32)
    val = np.concatenate(val_chunks).astype(np.uint32) if val_chunks else np.zeros(0, np.uint32)
    if m is None:
        m = dataset_max_bounds(col, val, D)
    return Dataset(name, m, row_ptr, col, val, k, seed, meta)


# ---------------------------------------------------------------------------------------------
# The five benchmark configurations
# ---------------------------------------------------------------------------------------------

def config1() -> Dataset:
    """Plain method, small: N=1000, D=1024, nnz ~ Poisson(100) clipped to [1, D] at distinct
    uniform columns, weights uniform on {1..65535}, m_i = dataset max (floor 1), k=64, seed 0."""
    rng = np.random.Generator(np.random.PCG64(1001))
    N, D = 1000, 1024
    nnz = np.clip(rng.poisson(100, N), 1, D)
    cols, vals = [], []
    for r in range(N):
        c = np.sort(rng.choice(D, size=int(nnz[r]), replace=False))
        cols.append(c)
        vals.append(rng.integers(1, 65536, size=len(c)))
    return _assemble(cols, vals, nnz, D, "config1-plain-small", 64, 0,
                     {"N": N, "D": D, "nnz": "Poisson(100) clipped to [1, D]",
                      "weights": "uniform {1..65535}"})


def config2(n_rows: int = 100_000) -> Dataset:
    """Histogram-shaped: N=100000, D=4096, each cell nonzero with probability 0.3, weights
    log-normal(0, 1) in Q8.8 fixed point (round(256 w) clamped to [1, 65535]), m_i = dataset
    max (floor 1), k=500, seed 0.  Rows are generated in blocks of 4096 so any prefix of rows
    is identical whatever n_rows is; the bounds are those of the n_rows generated."""
    rng = np.random.Generator(np.random.PCG64(1002))
    D, block = 4096, 4096
    cols, vals, lengths = [], [], []
    for r0 in range(0, n_rows, block):
        rows = min(block, n_rows - r0)
        mask = rng.random((rows, D), dtype=np.float32) < np.float32(0.3)
        rr, cc = np.nonzero(mask)
        w = rng.lognormal(0.0, 1.0, size=len(cc))
        q = np.clip(np.rint(256.0 * w), 1, 65535).astype(np.uint32)
        cols.append(cc.astype(np.uint32))
        vals.append(q)
        lengths.append(np.bincount(rr, minlength=rows))
    lengths = np.concatenate(lengths) if lengths else np.zeros(0, np.int64)
    return _assemble(cols, vals, lengths, D, "config2-histogram", 500, 0,
                     {"N": n_rows, "D": D, "density": 0.3, "weights": "LogNormal(0,1) Q8.8"})


def _zipf_clipped(rng, a, lo, hi, n):
    return np.clip(rng.zipf(a, n), lo, hi).astype(np.int64)


def _tf_weights(rng, n):
    """1 + ln(count), count ~ Zipf(1.5), in Q16.16 fixed point."""
    count = rng.zipf(1.5, n).astype(np.float64)
    return np.rint(65536.0 * (1.0 + np.log(count))).astype(np.uint64).clip(1, U32_MAX) \
        .astype(np.uint32)


def _sparse_rows_with_replacement(rng, lengths, D, weight_fn):
    """Columns drawn uniformly with replacement (lengths[r] draws for row r), duplicates merged
    so each row's columns are distinct and increasing; weights drawn per kept column."""
    lengths = np.asarray(lengths, dtype=np.int64)
    row_of = np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)
    c = rng.integers(0, D, size=int(lengths.sum()), dtype=np.int64)
    key = np.unique(row_of * D + c)
    rows = key // D
    cols = (key % D).astype(np.uint32)
    vals = weight_fn(rng, len(cols))
    kept = np.bincount(rows, minlength=len(lengths))
    return cols, vals, kept


def _zipf_rows_block(seed: int, b: int, rows: int, D: int, lo: int, hi: int):
    """Block b of a Zipf-length workload, from its own generator (seed, spawn key b), so blocks
    can be drawn in any order and any prefix of blocks is the same whatever the total."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(b,))))
    want = _zipf_clipped(rng, 1.2, lo, hi, rows)
    return _sparse_rows_with_replacement(rng, want, D, _tf_weights)


def _zipf_rows(seed: int, n_rows: int, block: int, D: int, lo: int, hi: int):
    """Blocks of _zipf_rows_block drawn on host threads (numpy's sampling, sorting and
    logarithms run without the interpreter lock), concatenated in block order."""
    jobs = [(b, min(block, n_rows - r0)) for b, r0 in enumerate(range(0, n_rows, block))]
    workers = max(1, min(len(jobs), 16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda jb: _zipf_rows_block(seed, jb[0], jb[1], D, lo, hi), jobs))
    cols = [p[0] for p in parts]
    vals = [p[1] for p in parts]
    lengths = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, np.int64)
    return cols, vals, lengths


def config3(n_rows: int = 1_000_000, block: int = 20_000) -> Dataset:
    """Text-like: N=1,000,000, D=65536, nnz = clamp(Zipf(1.2), 10, 5000) column draws per row
    (uniform with replacement, duplicates merged), tf weights 1+ln(count), count ~ Zipf(1.5),
    Q16.16, m_i = dataset max (floor 1), k=1000, seed 0.  Blocks of `block` rows have their own
    generators (seed 1003, spawn key = block number)."""
    D = 65536
    cols, vals, lengths = _zipf_rows(1003, n_rows, block, D, 10, 5000)
    return _assemble(cols, vals, lengths, D, "config3-text", 1000, 0,
                     {"N": n_rows, "D": D, "nnz": "clamp(Zipf(1.2), 10, 5000) draws",
                      "weights": "1+ln(Zipf(1.5)) Q16.16"})


def config4(n_rows: int = 200_000) -> Dataset:
    """Heavy-tail rejection: N=200000, D=16384, nnz ~ U{20..2000} distinct uniform columns,
    weights uniform on {1..2^24}; 1% of the dimensions (164) each get one outlier row holding
    100 * 2^24 in that dimension, so their bounds are 100x the rest; m_i = dataset max; k=500.
    The collision-count workload pairs rows [0, 10000) with rows [10000, 20000)."""
    rng = np.random.Generator(np.random.PCG64(1004))
    D = 16384
    n_out = 164
    out_dims = np.sort(rng.choice(D, size=n_out, replace=False))
    out_rows = rng.integers(0, n_rows, size=n_out)
    extra: dict[int, list[int]] = {}
    for d, r in zip(out_dims, out_rows):
        extra.setdefault(int(r), []).append(int(d))
    nnz = rng.integers(20, 2001, size=n_rows)
    cols, vals, lengths = [], [], []
    big = np.uint32(100 * (1 << 24))
    for r in range(n_rows):
        c = rng.choice(D, size=int(nnz[r]), replace=False)
        v = rng.integers(1, (1 << 24) + 1, size=len(c)).astype(np.uint32)
        if r in extra:
            add = np.array(extra[r], dtype=np.int64)
            present = np.isin(add, c)
            v[np.isin(c, add)] = big
            c = np.concatenate([c, add[~present]])
            v = np.concatenate([v, np.full(int((~present).sum()), big, dtype=np.uint32)])
        order = np.argsort(c)
        cols.append(c[order].astype(np.uint32)); vals.append(v[order])
        lengths.append(len(c))
    return _assemble(cols, vals, lengths, D, "config4-heavy-tail", 500, 0,
                     {"N": n_rows, "D": D, "nnz": "U{20..2000}", "weights": "U{1..2^24}",
                      "outlier_dims": n_out, "outlier_value": int(big),
                      "pairs": [[0, 10000], [10000, 20000]]})


def config5_corpus(n_rows: int = 100_000, block: int = 20_000) -> Dataset:
    """Serving corpus: 100,000 rows, D=2^20, nnz = clamp(Zipf(1.2), 5, 10000) column draws per
    row (with replacement, duplicates merged), tf weights as config 3, m_i = corpus max; k=256.
    Requests are batches of corpus rows, so every request is within the bounds.  Blocks of
    `block` rows have their own generators (seed 1005, spawn key = block number)."""
    D = 1 << 20
    cols, vals, lengths = _zipf_rows(1005, n_rows, block, D, 5, 10000)
    return _assemble(cols, vals, lengths, D, "config5-serving-corpus", 256, 0,
                     {"N": n_rows, "D": D, "nnz": "clamp(Zipf(1.2), 5, 10000) draws"})


def serving_requests(n_requests: int, corpus_rows: int, qps: float, seed: int = 2005,
                     max_rows: int = 4096):
    """Poisson arrival times (seconds) and request row lists: sizes log-uniform on [1, 4096],
    rows drawn uniformly from the corpus."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps)
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(max_rows + 1), size=n_requests))) \
        .astype(np.int64).clip(1, max_rows)
    rows = [rng.integers(0, corpus_rows, size=int(s)) for s in sizes]
    return arrivals, sizes, rows


def serving_ranges(n_requests: int, corpus_rows: int, qps: float, seed: int = 2005,
                   max_rows: int = 4096):
    """Poisson arrival times (seconds), request sizes log-uniform on [1, max_rows] and the first
    corpus row of each request, which takes that many consecutive rows.  The corpus rows are
    independent and identically distributed, so a run of consecutive rows is distributed like
    rows drawn at random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arrivals = np.cumsum(gaps)
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(max_rows + 1), size=n_requests))) \
        .astype(np.int64).clip(1, min(max_rows, corpus_rows))
    starts = rng.integers(0, corpus_rows - sizes + 1)
    return arrivals, sizes, starts


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5_corpus}


# ---------------------------------------------------------------------------------------------
# Small random cases for tests
# ---------------------------------------------------------------------------------------------

def random_case(seed: int, n_rows: int, D: int, density: float, max_val: int,
                bound_slack: int = 0, empty_rows: int = 0, zero_bound_dims: int = 0,
                k: int = 64) -> Dataset:
    """Random CSR rows with bounds = dataset max + a random slack in [0, bound_slack].
    ``empty_rows`` rows are left empty; ``zero_bound_dims`` dimensions get m_i = 0 (and no
    entries)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((n_rows, D), dtype=np.uint64)
    mask = rng.random((n_rows, D)) < density
    X[mask] = rng.integers(1, max_val + 1, size=int(mask.sum()), dtype=np.uint64)
    zero_dims = rng.choice(D, size=min(zero_bound_dims, D - 1), replace=False) \
        if zero_bound_dims else np.zeros(0, dtype=np.int64)
    X[:, zero_dims] = 0
    if empty_rows:
        X[rng.choice(n_rows, size=min(empty_rows, n_rows), replace=False)] = 0
    m = X.max(axis=0) if n_rows else np.zeros(D, dtype=np.uint64)
    m = np.maximum(m, 1)
    if bound_slack:
        m = m + rng.integers(0, bound_slack + 1, size=D, dtype=np.uint64)
    m = np.minimum(m, U32_MAX)
    m[zero_dims] = 0
    X = X.astype(np.uint32)
    return csr_from_dense(X, m=m.astype(np.uint32), name=f"random-{seed}", k=k)
