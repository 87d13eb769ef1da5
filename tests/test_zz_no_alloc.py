"""wmh_hash_noalloc (the batched walk with its scratch in the library's static device array)
against wmh_hash, bit for bit, through the C-ABI; and its argument checks."""
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


def both(ctx, ds, k, seed=0, **plan):
    """(wmh_hash batched signatures, wmh_hash_noalloc signatures) of ds as numpy uint16."""
    print(f"  noalloc: {ds.name} N={ds.n_rows} D={ds.D} k={k} seed={seed} {plan}", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    want = wmh.sig_to_numpy(ctx.hash(rows, k, seed=seed, mode="batched", **plan))
    sig = torch.full((ds.n_rows, k), -1, dtype=torch.int16, device=DEV)
    ctx.hash_noalloc_into(rows, k, seed, sig, opts=ctx.make_opts(mode="batched", **plan))
    torch.cuda.synchronize()
    return want, wmh.sig_to_numpy(sig)


def test_two_calls_in_a_row_second_smaller(ctx):
    ds = synth.config2(n_rows=3000)
    want, got = both(ctx, ds, 500)
    assert np.array_equal(got, want)
    head = ds.head(16)
    assert np.array_equal(got[:16], oracle.hash_csr(head.m, head.row_ptr, head.col, head.val, 500,
                                                    seed=0))
    assert ctx.last_plan()["mode"] == "batched"
    small = ds.head(700)
    want, got = both(ctx, small, 64, seed=7)
    assert np.array_equal(got, want)


def test_plans_and_empty_rows(ctx):
    ds = synth.random_case(11, 300, 512, 0.05, 1000, empty_rows=5)
    for plan in ({}, {"rows_per_block": 1, "walk": "ballot"},
                 {"rows_per_block": 2, "steps_per_lane": 4}, {"walk": "rows"},
                 {"rows_per_block": 1, "walk": "ballot", "hash_groups": 8},
                 {"stream_depth": None}):
        want, got = both(ctx, ds, 96, seed=3, **plan)
        assert np.array_equal(got, want), plan


def test_coarse_code_ties_without_allocation(ctx):
    """Coarse codes of 2 bits make most tested steps in a row's support tie: the no-allocation
    walk settles them exactly (in-lane draws and the row's CSR value), as wmh_hash and the
    oracle do, with the ballot walk and the shared windows."""
    ds = synth.random_case(23, 200, 2048, 0.05, 1 << 20, bound_slack=1 << 18)
    exact = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 64, seed=9)
    for plan in ({"values": "coarse", "coarse_bits": 2, "walk": "ballot"},
                 {"values": "coarse", "coarse_bits": 2, "rows_per_block": 4}):
        want, got = both(ctx, ds, 64, seed=9, **plan)
        assert np.array_equal(got, want), plan
        assert np.array_equal(got, exact), plan
        assert ctx.last_plan()["coarse_bits"] == 2


def test_stream_shrinks_to_the_static_array(ctx):
    # tiny green fractions: the planner's stream (about 65000 steps x 128 ids x 4 or 8 bytes)
    # is larger than the static array, so the call walks a shorter stream and draws in-lane
    # beyond
    D = 1024
    rng = np.random.Generator(np.random.PCG64(5))
    cols = [np.sort(rng.choice(D, 5, replace=False)) for _ in range(40)]
    vals = [rng.integers(1, 1 << 18, 5, dtype=np.uint64) for _ in range(40)]
    m = np.full(D, 1 << 24, dtype=np.uint32)
    ds = synth.csr_from_lists(cols, vals, D, m=m, name="sparse-green", k=128)
    # bounds above 65535: coarse codes in 4-byte entries (the default), or the exact values in
    # 8-byte entries
    exact = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 128, seed=0)
    for values, entry in (("auto", 4), ("coarse", 4), ("exact", 8)):
        want, got = both(ctx, ds, 128, values=values)
        assert np.array_equal(got, want), values
        assert np.array_equal(got, exact), values
        plan = ctx.last_plan()
        assert plan["values"] == ("coarse" if entry == 4 else "exact")
        assert 0 < plan["stream_depth"] < 65000
        assert plan["stream_depth"] * 128 * entry <= wmh.NOALLOC_SCRATCH_BYTES


def test_rejections_leave_the_output_untouched(ctx):
    ds = synth.config1().head(50)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    sig = torch.full((ds.n_rows, 128), 123, dtype=torch.int16, device=DEV)
    # a stream the caller asks for that does not fit the array (65088 steps x 128 ids x 4 B)
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash_noalloc_into(rows, 128, 0, sig,
                              opts=ctx.make_opts(mode="batched", stream_depth=65000,
                                                 rows_per_block=1, walk="ballot"))
    assert e.value.name == "WMH_E_ARG"
    assert "static scratch" in str(e.value)
    # another mode
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash_noalloc_into(rows, 128, 0, sig, opts=ctx.make_opts(mode="plain"))
    assert e.value.name == "WMH_E_ARG"
    # a value above its bound
    bad = ds.head(50)
    val = bad.val.copy()
    val[3] = int(bad.m[bad.col[3]]) + 1
    bad_rows = wmh.upload_dataset(synth.Dataset(bad.name, bad.m, bad.row_ptr, bad.col, val,
                                                bad.k, bad.seed, bad.meta), DEV)
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash_noalloc_into(bad_rows, 128, 0, sig)
    assert e.value.name == "WMH_E_BOUND"
    torch.cuda.synchronize()
    assert bool((sig == 123).all())
