"""GPU parity of the row split (WMH_MODE_SPLIT): the validation pass classes every row by its own
estimated costs, the batched walk takes one class and the component index the other, and the
signatures must equal the oracle's bit for bit whatever the classes (each row's value depends
only on the row, the bounds and the seed, Sec. 3.1)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1602_08393_amd import synth, wmh  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = wmh.Context(0)
    yield c
    c.close()


def gpu_sig(ctx, ds, k, seed, **opts):
    print(f"  gpu: {ds.name} N={ds.n_rows} D={ds.D} k={k} seed={seed} {opts}", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    return wmh.sig_to_numpy(ctx.hash(rows, k, seed=seed, **opts))


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {want.size} differ; first at row {r} hash "
                             f"{j}: gpu {got[r, j]} oracle {want[r, j]}")


def mixed_rows(seed, n_dense, n_sparse, D, k):
    """Rows whose green fractions differ by orders of magnitude: dense rows near their bounds
    (short walks) interleaved with rows of one or two tiny entries (walks of thousands of
    steps), plus an empty row."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(1000, 60000, size=D).astype(np.uint32)
    cols, vals = [], []
    for i in range(n_dense + n_sparse):
        if i % 2 == 0 and len([c for c in cols if len(c) > 4]) < n_dense:
            c = np.sort(rng.choice(D, size=int(rng.integers(D // 3, D // 2)), replace=False))
            v = (m[c] * rng.uniform(0.5, 1.0, size=len(c))).astype(np.uint32)
        else:
            c = np.sort(rng.choice(D, size=int(rng.integers(1, 3)), replace=False))
            v = rng.integers(1, 40, size=len(c)).astype(np.uint32)
        cols.append(c)
        vals.append(v)
    cols.append(np.zeros(0, np.uint32))
    vals.append(np.zeros(0, np.uint32))
    return synth.csr_from_lists(cols, vals, D, m=m, name=f"mixed-{seed}", k=k)


def test_forced_split_random_cases(ctx):
    """Forced split on seeded random datasets (empty rows, zero-bound dimensions, wide values):
    equal to the oracle whichever way the rows fall."""
    for case in range(6):
        rng = np.random.Generator(np.random.PCG64(500 + case))
        ds = synth.random_case(seed=600 + case, n_rows=int(rng.integers(1, 120)),
                               D=int(rng.integers(2, 2500)),
                               density=float(rng.uniform(0.001, 0.4)),
                               max_val=int(rng.choice([255, 65535, 2 ** 24, 2 ** 32 - 1])),
                               bound_slack=int(rng.choice([0, 1000, 10 ** 6])),
                               empty_rows=int(rng.integers(0, 3)),
                               zero_bound_dims=int(rng.integers(0, 3)))
        k = int(rng.integers(1, 200))
        seed = int(rng.integers(0, 2 ** 63))
        want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
        assert_same(gpu_sig(ctx, ds, k, seed, mode="split"), want, f"case {case} split")
        assert ctx.last_mode() in ("split", "batched", "indexed")


def test_split_mixed_rows(ctx):
    """A batch of dense and very sparse rows: the split puts them on different paths (both
    classes non-empty), with the shared and ballot walks and without a graph; auto takes the
    split for this batch."""
    ds = mixed_rows(7, 40, 40, 3000, 200)
    k, seed = 200, 31
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    for opts in (dict(mode="split"), dict(mode="split", use_graph=False),
                 dict(mode="split", walk="ballot"), dict(mode="split", rows_per_block=2),
                 dict(mode="split", stream_depth=None), dict(mode="auto")):
        assert_same(gpu_sig(ctx, ds, k, seed, **opts), want, f"mixed {opts}")
        if opts["mode"] == "split":
            assert ctx.last_mode() == "split", opts
    assert ctx.last_mode() == "split"  # auto chose the split
    # the signatures of the other class are left as they were: a split over rows whose
    # outputs are pre-filled still writes every row
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    sig = torch.full((ds.n_rows, k), 12345, dtype=torch.int16, device=DEV)
    ctx.hash_into(rows, k, seed, sig, opts=ctx.make_opts(mode="split"))
    assert_same(wmh.sig_to_numpy(sig), want, "mixed split into a pre-filled output")


def test_split_heavy_tail_head(ctx):
    """The first 400 rows of the heavy-tail workload under a forced split and under auto."""
    ds = synth.config4(n_rows=2000).head(400)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 500, seed=0)
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="split"), want, "heavy tail head split")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="auto"), want, "heavy tail head auto")


def test_split_heavy_tail_full_size(ctx):
    """All 200000 heavy-tail rows in auto mode (the planner's choice) and forced split: sampled
    rows against the oracle, every row against the batched walk."""
    ds = synth.config4()
    k = ds.k
    print(f"  heavy tail N={ds.n_rows} k={k}", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    walk = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="batched"))
    # the plan tuned on every row serves the walk rows of the split (a nearer step class)
    tuned = ctx.tune(rows, k, 0, reps=1)
    split = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="split"))
    assert ctx.last_mode() == "split"
    plan = ctx.last_plan()
    assert (plan["walk"], plan["rows_per_block"], plan["waves_per_block"]) == \
        (tuned["walk"], tuned["rows_per_block"], tuned["waves_per_block"]), (plan, tuned)
    assert np.array_equal(split, walk)
    auto = wmh.sig_to_numpy(ctx.hash(rows, k, seed=0, mode="auto"))
    assert ctx.last_mode() == "split"  # the planner's choice for this workload
    assert np.array_equal(auto, walk)
    sums = np.bincount(np.repeat(np.arange(ds.n_rows), np.diff(ds.row_ptr.astype(np.int64))),
                       weights=ds.val.astype(np.float64), minlength=ds.n_rows)
    order = np.argsort(sums, kind="stable")
    rng = np.random.Generator(np.random.PCG64(17))
    idx = np.unique(np.concatenate([order[:6], order[-3:], rng.integers(0, ds.n_rows, 20)]))
    sub = ds.rows(idx)
    want = oracle.hash_csr(sub.m, sub.row_ptr, sub.col, sub.val, k, seed=0)
    assert_same(split[idx], want, "heavy tail split, sampled rows")
