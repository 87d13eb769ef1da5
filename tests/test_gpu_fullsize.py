"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark times.

The whole dataset is hashed on the GPU exactly as ``bench.py`` hashes it (autotuned tile plan,
hipGraph replay, or the planner's choice of path); the oracle then recomputes a sample of rows
one by one — spread over every part of the batch, plus the rows with the longest and shortest
walks and the rows holding the inflated bounds — and the two must agree bit for bit.  Every
row's signature depends only on that row, the bounds and the seed (Sec. 3.1, the consistency
requirement after Definition 1), so a row computed alone by the oracle is the row's exact
expected value inside the full batch.  Properties that hold at any size (batched equals plain
on every row; replays repeat the first call) are checked over all rows.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1602_08393_amd import serve, synth, wmh  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = wmh.Context(0)
    yield c
    c.close()


def say(msg):
    print(f"  {msg}", flush=True)


def row_sums(ds):
    """Sum of each row's weights (u64), for picking the longest and shortest walks."""
    rows = np.repeat(np.arange(ds.n_rows), np.diff(ds.row_ptr.astype(np.int64)))
    return np.bincount(rows, weights=ds.val.astype(np.float64), minlength=ds.n_rows)


def sample_rows(ds, n_random, seed, extra=()):
    """First and last rows, a seeded random spread, the rows with the smallest and largest
    weight sums, and any extra rows, without repeats, in increasing order."""
    n = ds.n_rows
    rng = np.random.Generator(np.random.PCG64(seed))
    sums = row_sums(ds)
    order = np.argsort(sums, kind="stable")
    picks = [np.arange(min(4, n)), np.arange(max(0, n - 4), n),
             rng.integers(0, n, size=n_random), order[:4], order[-4:],
             np.asarray(list(extra), dtype=np.int64)]
    return np.unique(np.concatenate(picks).astype(np.int64))


def assert_rows_equal(got, want, idx, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {want.size} sampled values differ; first "
                             f"at row {idx[r]} hash {j}: gpu {got[r, j]} oracle {want[r, j]}")


def oracle_rows(ds, idx, k, seed=0):
    sub = ds.rows(idx)
    return oracle.hash_csr(sub.m, sub.row_ptr, sub.col, sub.val, k, seed=seed)


def test_histogram_full_size(ctx):
    """N = 100000, D = 4096, k = 500: autotuned batched plan under hipGraph replay, the
    headline configuration of the benchmark; the plain form on all rows."""
    ds = synth.config2()
    k = ds.k
    say(f"histogram full size N={ds.n_rows} D={ds.D} nnz={ds.nnz} k={k}")
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    tuned = ctx.tune(rows, k, 0, reps=1)
    say(f"tuned plan {tuned}")
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device=DEV)
    opts = ctx.make_opts(mode="batched")
    ctx.hash_into(rows, k, 0, sig, opts=opts)
    plan = ctx.last_plan()
    assert plan["rows_per_block"] == tuned["rows_per_block"]
    assert plan["hashes_per_tile"] == tuned["hashes_per_tile"]
    first = sig.clone()
    for _ in range(2):  # graph replays, with eager work between them
        sig.zero_()
        ctx.hash_into(rows, k, 0, sig, opts=opts)
        torch.cuda.synchronize()
        assert torch.equal(sig, first), "replay differs from the first call"
    idx = sample_rows(ds, 40, 11)
    say(f"oracle on {len(idx)} sampled rows")
    got = wmh.sig_to_numpy(sig)
    assert_rows_equal(got[idx], oracle_rows(ds, idx, k), idx, "histogram batched")
    assert got.min() >= 1  # no empty rows in this workload; every hash has a green step
    say("plain form on all rows")
    plain = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="plain"))
    assert np.array_equal(plain, got)
    say("the tuned plan scheduled plainly (a launch per 8192 rows) on all rows")
    shared = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="plain_shared"))
    assert np.array_equal(shared, got)


def test_heavy_tail_full_size(ctx):
    """N = 200000, D = 16384, k = 500 with 1% of bounds inflated 100x: autotuned batched plan,
    the plain form on all rows, and the 10^4 x 10^4 collision counts on sampled pairs."""
    ds = synth.config4()
    k = ds.k
    say(f"heavy tail full size N={ds.n_rows} D={ds.D} nnz={ds.nnz} k={k}")
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    tuned = ctx.tune(rows, k, 0, reps=1)
    say(f"tuned plan {tuned}")
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device=DEV)
    ctx.hash_into(rows, k, 0, sig, opts=ctx.make_opts(mode="batched"))
    plan = ctx.last_plan()
    assert plan["rows_per_block"] == tuned["rows_per_block"]
    got = wmh.sig_to_numpy(sig)
    big = ds.meta["outlier_value"]
    rows_of = np.repeat(np.arange(ds.n_rows), np.diff(ds.row_ptr.astype(np.int64)))
    outlier_rows = np.unique(rows_of[ds.val == big])
    assert len(outlier_rows) > 0
    idx = sample_rows(ds, 40, 12, extra=outlier_rows[:12])
    say(f"oracle on {len(idx)} sampled rows ({min(12, len(outlier_rows))} with outliers)")
    assert_rows_equal(got[idx], oracle_rows(ds, idx, k), idx, "heavy tail batched")
    say("plain form on all rows")
    plain = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="plain"))
    assert np.array_equal(plain, got)
    say("the tuned plan scheduled plainly (a launch per 8192 rows) on all rows")
    shared = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="plain_shared"))
    assert np.array_equal(shared, got)
    say("collision counts, rows [0, 1e4) x [1e4, 2e4)")
    A = sig[0:10000].contiguous()
    B = sig[10000:20000].contiguous()
    counts = ctx.collisions(A, B)
    rng = np.random.Generator(np.random.PCG64(13))
    a_idx = np.concatenate([[0, 9999], rng.integers(0, 10000, 500)])
    b_idx = np.concatenate([[9999, 0], rng.integers(0, 10000, 500)])
    ta = torch.from_numpy(a_idx).to(DEV)
    tb = torch.from_numpy(b_idx).to(DEV)
    sampled = counts[ta, tb].cpu().numpy().view(np.uint32)
    for n, (a, b) in enumerate(zip(a_idx, b_idx)):
        assert sampled[n] == oracle.collisions(got[a], got[10000 + b]), (a, b)


def test_text_like_rows_full_batch(ctx):
    """The first 100000 rows of the text-like workload (D = 65536, k = 1000), hashed in auto
    mode as the benchmark hashes all 1e6 (the planner takes the component index)."""
    ds = synth.config3(n_rows=100_000, block=20_000)
    k = ds.k
    say(f"text-like N={ds.n_rows} D={ds.D} nnz={ds.nnz} k={k}")
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    tuned = ctx.tune(rows, k, 0, reps=1)
    say(f"tuned plan {tuned}")
    assert tuned["walk"] == "index"
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device=DEV)
    opts = ctx.make_opts(mode="auto")  # graph replay of the tuned index rows kernel
    ctx.hash_into(rows, k, 0, sig, opts=opts)
    assert ctx.last_mode() == "indexed"
    plan = ctx.last_plan()
    assert (plan["waves_per_block"], plan["index_batch"], plan["index_claim"]) == \
        (tuned["waves_per_block"], tuned["index_batch"], tuned["index_claim"])
    got = wmh.sig_to_numpy(sig)
    # the rows whose step-order reads left a hash id open past T1 (second pass) or past T2
    # (offset-order pass), by the kernel's own rule (Theorem 2 bounds)
    M = float(ds.m.astype(np.float64).sum())
    rows_of = np.repeat(np.arange(ds.n_rows), np.diff(ds.row_ptr.astype(np.int64)))
    sx = np.bincount(rows_of, weights=ds.val.astype(np.float64), minlength=ds.n_rows)
    sm = np.bincount(rows_of, weights=np.where(ds.val > 0, ds.m[ds.col], 0).astype(np.float64),
                     minlength=ds.n_rows)
    s = np.maximum(sx, 1) / M
    t1 = np.ceil(np.log((1 / 16) / k) / np.log1p(-s))
    t2 = np.ceil(np.log(1e-4 / k) / np.log1p(-s))
    by_steps = (sx > 0) & (t2 < 65534) & (t2 * sm < 65534.0 * sx)
    top = got.max(axis=1)
    second = np.flatnonzero(by_steps & (top > t1))
    third = np.flatnonzero(by_steps & (top > t2))
    say(f"{by_steps.sum()} step-order rows; {len(second)} read again to T2, {len(third)} in "
        f"offset order")
    assert len(second) > 0
    idx = sample_rows(ds, 12, 14, extra=np.concatenate([second[:8], third[:8]]))
    say(f"oracle on {len(idx)} sampled rows")
    assert_rows_equal(got[idx], oracle_rows(ds, idx, k), idx, "text-like auto")
    for _ in range(2):  # graph replays, with eager work between them
        sig.zero_()
        ctx.hash_into(rows, k, 0, sig, opts=opts)
        torch.cuda.synchronize()
        assert np.array_equal(wmh.sig_to_numpy(sig), got), "replay differs from the first call"


def test_text_like_full_million_rows(ctx):
    """All 1e6 rows of the text-like workload (D = 65536, k = 1000), in the benchmark's launch
    configuration (index rows plan tuned on these rows, graph replay); the oracle checks the
    first and last rows, a random spread, the lightest and heaviest rows and rows that ran the
    index's second and offset-order passes."""
    ds = synth.config3()
    k = ds.k
    say(f"text-like full N={ds.n_rows} D={ds.D} nnz={ds.nnz} k={k}")
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device=DEV)
    opts = ctx.make_opts(mode="auto")
    ctx.hash_into(rows, k, 0, sig, opts=opts)  # builds the index
    tuned = ctx.tune(rows, k, 0, reps=1)
    say(f"tuned plan {tuned}")
    ctx.hash_into(rows, k, 0, sig, opts=opts)
    assert ctx.last_mode() == "indexed"
    got = wmh.sig_to_numpy(sig)
    M = float(ds.m.astype(np.float64).sum())
    rows_of = np.repeat(np.arange(ds.n_rows), np.diff(ds.row_ptr.astype(np.int64)))
    sx = np.bincount(rows_of, weights=ds.val.astype(np.float64), minlength=ds.n_rows)
    sm = np.bincount(rows_of, weights=np.where(ds.val > 0, ds.m[ds.col], 0).astype(np.float64),
                     minlength=ds.n_rows)
    s = np.maximum(sx, 1) / M
    t1 = np.ceil(np.log((1 / 16) / k) / np.log1p(-s))
    t2 = np.ceil(np.log(1e-4 / k) / np.log1p(-s))
    by_steps = (sx > 0) & (t2 < 65534) & (t2 * sm < 65534.0 * sx)
    top = got.max(axis=1)
    second = np.flatnonzero(by_steps & (top > t1))
    third = np.flatnonzero(by_steps & (top > t2))
    say(f"{by_steps.sum()} step-order rows; {len(second)} read again to T2, {len(third)} in "
        f"offset order")
    idx = sample_rows(ds, 8, 16, extra=np.concatenate([second[:4], third[:4]]))
    say(f"oracle on {len(idx)} sampled rows")
    assert_rows_equal(got[idx], oracle_rows(ds, idx, k), idx, "text-like 1e6 rows")
    del rows, sig
    torch.cuda.empty_cache()


def test_serving_on_the_large_corpus(ctx):
    """Requests drawn from the first 20000 rows of the D = 2^20 serving corpus (k = 256), in
    page-locked buffers as the benchmark sends them, run through the loop with several slots so
    they overlap; sampled rows of every request equal the oracle, and every request equals
    wmh_hash on the same rows."""
    corpus = synth.config5_corpus(n_rows=20_000)
    k = corpus.k
    say(f"serving corpus N={corpus.n_rows} D={corpus.D} nnz={corpus.nnz} k={k}")
    ctx.set_bounds(corpus.m)
    _, sizes, row_lists = synth.serving_requests(12, corpus.n_rows, qps=1.0, seed=3105,
                                                 max_rows=4096)
    with serve.Server(ctx, k, seed=0, slots=4) as srv:
        reqs = serve.requests_from_corpus(corpus, row_lists, srv, pinned=True)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            srv.wait(r.ticket)
    rng = np.random.Generator(np.random.PCG64(15))
    for n, (rl, r) in enumerate(zip(row_lists, reqs)):
        pick = np.unique(rng.integers(0, len(rl), size=min(3, len(rl))))
        say(f"request {n}: {len(rl)} rows, oracle on {len(pick)}")
        want = oracle_rows(corpus, rl[pick], k)
        assert_rows_equal(r.sig[pick], want, rl[pick], f"serving request {n}")
        sub = corpus.rows(rl)
        direct = wmh.sig_to_numpy(ctx.hash(wmh.upload_dataset(sub, DEV), k, seed=0))
        assert np.array_equal(direct, r.sig), f"request {n} differs from wmh_hash"
