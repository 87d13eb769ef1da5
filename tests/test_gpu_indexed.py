"""GPU parity of the component-index path (WMH_MODE_INDEXED) and of the planner's choice.

The index files every draw (j, t <= 65534) under its component; a row's hash j is the
smallest green t among its components' keys, else 65535.  These tests hold it to the oracle's
walk bit for bit: long lists split in sorted chunks, saturated rows, empty rows, explicit
zeros, zero-size pieces, the largest k, index reuse and rebuilds, and the planner's choice.
"""
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


def gpu_sig(ctx, ds, k, seed=0, **opts):
    print(f"  gpu: {ds.name} N={ds.n_rows} D={ds.D} k={k} seed={seed} {opts}", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    return wmh.sig_to_numpy(ctx.hash(rows, k, seed=seed, **opts))


def want_sig(ds, k, seed):
    return oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {want.size} differ; first at row {r} hash "
                             f"{j}: gpu {got[r, j]} oracle {want[r, j]}")


def test_config1_indexed(ctx):
    """D = 1024, k = 64: lists of about 4096 keys, many longer than one sorted chunk."""
    ds = synth.config1()
    got = gpu_sig(ctx, ds, ds.k, 0, mode="indexed")
    assert ctx.last_mode() == "indexed"
    assert_same(got, want_sig(ds, ds.k, 0), "config1 indexed")


CASES = {
    "ragged-empty-zero-dims": (dict(seed=1, n_rows=37, D=300, density=0.2, max_val=60000,
                                    bound_slack=5000, empty_rows=5, zero_bound_dims=20), 70, 11),
    "wide-values": (dict(seed=2, n_rows=29, D=257, density=0.1, max_val=2 ** 32 - 1,
                         bound_slack=0, empty_rows=1), 33, 12),
    "single-dimension": (dict(seed=3, n_rows=50, D=1, density=1.0, max_val=100,
                              bound_slack=300), 65, 13),
    "sparse-slow": (dict(seed=4, n_rows=19, D=2000, density=0.005, max_val=500,
                         bound_slack=60000), 40, 14),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_random_cases_indexed(ctx, name):
    kw, k, seed = CASES[name]
    ds = synth.random_case(k=k, **kw)
    assert_same(gpu_sig(ctx, ds, k, seed, mode="indexed"), want_sig(ds, k, seed),
                f"{name} indexed")


def test_explicit_zero_values_and_saturation(ctx):
    """x = m gives 1 everywhere; one unit of 2^40 saturates at 65535; a row of explicit zeros
    is empty (all 0)."""
    m = np.full(256, 0xFFFFFFFF, dtype=np.uint32)
    cols = [np.arange(256), [3], [200], [5, 9, 77], []]
    vals = [m.copy(), [1], [1], [0, 0, 0], []]
    ds = synth.csr_from_lists(cols, vals, 256, m=m)
    k = 20
    want = want_sig(ds, k, 5)
    assert np.all(want[0] == 1) and np.all(want[1] == 65535) and np.all(want[3] == 0)
    assert_same(gpu_sig(ctx, ds, k, 5, mode="indexed"), want, "saturation indexed")


def test_one_giant_piece(ctx):
    """One piece holds almost all of M: its list has k * 65534 keys in 4096-key chunks."""
    m = np.array([1_000_000_000, 10, 10, 0, 10, 10, 10, 10], dtype=np.uint32)
    rng = np.random.Generator(np.random.PCG64(8))
    cols, vals = [], []
    for r in range(24):
        c = np.sort(rng.choice(8, size=int(rng.integers(1, 6)), replace=False))
        c = c[c != 3]
        v = [int(rng.integers(1, 20000)) if x == 0 else int(rng.integers(0, 11)) for x in c]
        cols.append(c)
        vals.append(v)
    ds = synth.csr_from_lists(cols, vals, 8, m=m)
    k = 48
    assert_same(gpu_sig(ctx, ds, k, 9, mode="indexed"), want_sig(ds, k, 9), "giant piece")


def test_large_dimension_tiny_fraction_auto_picks_index(ctx):
    """D = 2^20, rows of a few hundred nonzeros among bounds near 2^20: s ~ 1e-4..1e-6, where
    the walk needs 10^4..65535 steps per hash.  AUTO takes the index; every mode agrees."""
    D = 1 << 20
    rng = np.random.Generator(np.random.PCG64(10))
    m = rng.integers(1 << 19, 1 << 21, size=D).astype(np.uint32)
    cols, vals = [], []
    for r in range(24):
        c = np.sort(rng.choice(D, size=int(rng.integers(1, 300)), replace=False))
        cols.append(c)
        vals.append(rng.integers(1, m[c].astype(np.int64) + 1))
    cols.append([])
    vals.append([])
    ds = synth.csr_from_lists(cols, vals, D, m=m)
    k = 64
    want = want_sig(ds, k, 3)
    assert (want == 65535).any() and (want < 65535).any()
    got = gpu_sig(ctx, ds, k, 3)
    assert ctx.last_mode() == "indexed"
    assert_same(got, want, "tiny fraction auto")
    assert_same(gpu_sig(ctx, ds, k, 3, mode="plain"), want, "tiny fraction plain")


def test_text_like_rows_k1000(ctx):
    """Rows of the text-like workload (D = 65536, tf weights, k = 1000).  For 12 rows the
    planner does not pay for an index build; once the index exists it uses it."""
    ds = synth.config3(n_rows=2000, block=2000).head(12)
    k = 1000
    want = want_sig(ds, k, 0)
    assert_same(gpu_sig(ctx, ds, k, 0), want, "text-like auto, no index yet")
    assert ctx.last_mode() == "plain"
    assert_same(gpu_sig(ctx, ds, k, 0, mode="indexed"), want, "text-like indexed")
    assert_same(gpu_sig(ctx, ds, k, 0), want, "text-like auto, index built")
    assert ctx.last_mode() == "indexed"


def test_auto_keeps_the_walk_for_dense_rows(ctx):
    ds = synth.config2(n_rows=256)
    got = gpu_sig(ctx, ds, 500, 0)
    assert ctx.last_mode() == "batched"
    assert_same(got, want_sig(ds, 500, 0), "config2 head auto")


def test_index_reuse_and_rebuilds(ctx):
    """The index is kept per (bounds, seed, k) and rebuilt when any of them changes."""
    a = synth.random_case(seed=21, n_rows=30, D=500, density=0.05, max_val=1000,
                          bound_slack=20000, empty_rows=2)
    b = synth.random_case(seed=22, n_rows=30, D=700, density=0.05, max_val=1000,
                          bound_slack=20000)
    for ds, k, seed in [(a, 32, 1), (a, 32, 1), (a, 32, 2), (a, 50, 2), (b, 50, 2), (a, 32, 1)]:
        assert_same(gpu_sig(ctx, ds, k, seed, mode="indexed"), want_sig(ds, k, seed),
                    f"{ds.name} k={k} seed={seed}")


def test_largest_k(ctx):
    """k = 8192 (one wavefront per workgroup, 16-bit hash ids up to 8191)."""
    ds = synth.random_case(seed=23, n_rows=5, D=64, density=0.3, max_val=1000,
                           bound_slack=100000, empty_rows=1)
    k = 8192
    assert_same(gpu_sig(ctx, ds, k, 4, mode="indexed"), want_sig(ds, k, 4), "k=8192")
    rows = wmh.upload_dataset(ds, DEV)
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash(rows, k + 1, seed=4, mode="indexed")
    assert e.value.name == "WMH_E_ARG"


def test_unvalidated_auto_still_plans(ctx):
    ds = synth.config3(n_rows=2000, block=2000).rows(np.arange(20, 26))
    k = 256
    want = want_sig(ds, k, 7)
    assert_same(gpu_sig(ctx, ds, k, 7, mode="indexed"), want, "indexed")
    assert_same(gpu_sig(ctx, ds, k, 7, validate=False), want, "unvalidated auto")
    assert ctx.last_mode() == "indexed"
