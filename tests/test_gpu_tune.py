"""GPU tests of the autotuner (wmh_tune): the tuned plan is taken by later calls with the same
key, changes no hash value, and survives a save/load round trip."""
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


@pytest.fixture(scope="module")
def ds():
    return synth.config1()


def _plan_of(res):
    return (res["rows_per_block"], res["hashes_per_tile"], res["waves_per_block"], res["walk"],
            res["steps_per_lane"], res["hash_groups"], res["values"])


def test_tune_then_hash_uses_the_plan(ctx, ds):
    print("  tune config1", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    res = ctx.tune(rows, ds.k, seed=0, reps=2)
    assert res["candidates"] >= 10
    assert 0 < res["best_ms"] <= res["default_ms"]
    assert res["rows_per_block"] in (1, 2, 4, 8, 16)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, ds.k, seed=0)
    for mode in ("batched", "auto"):
        got = wmh.sig_to_numpy(ctx.hash(rows, ds.k, seed=0, mode=mode))
        assert np.array_equal(got, want)
        plan = ctx.last_plan()
        assert plan["mode"] == "batched"
        assert _plan_of(plan) == _plan_of(res)
    # an explicit override wins over the tuned plan
    ctx.hash(rows, ds.k, seed=0, mode="batched", rows_per_block=16, waves_per_block=4)
    assert ctx.last_plan()["rows_per_block"] == 16


def test_other_keys_keep_the_default_plan(ctx):
    other = synth.random_case(seed=31, n_rows=40, D=512, density=0.3, max_val=60000, k=48)
    ctx.set_bounds(other.m)
    rows = wmh.upload_dataset(other, DEV)
    want = oracle.hash_csr(other.m, other.row_ptr, other.col, other.val, 48, seed=2)
    got = wmh.sig_to_numpy(ctx.hash(rows, 48, seed=2, mode="batched"))
    assert np.array_equal(got, want)
    fresh = wmh.Context(0)
    try:
        fresh.set_bounds(other.m)
        fresh.hash(rows, 48, seed=2, mode="batched")
        assert ctx.last_plan() == fresh.last_plan()
    finally:
        fresh.close()


def test_save_and_load(ctx, ds, tmp_path):
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    res = ctx.tune(rows, ds.k, seed=0, reps=1)
    path = tmp_path / "plans.txt"
    ctx.tune_save(str(path))
    assert path.read_text().startswith("wmh-tune 6\n")
    fresh = wmh.Context(0)
    try:
        fresh.set_bounds(ds.m)
        fresh.tune_load(str(path))
        fresh.hash(rows, ds.k, seed=0, mode="batched")
        p = fresh.last_plan()
        assert _plan_of(p) == _plan_of(res)
        bad = tmp_path / "bad.txt"
        bad.write_text("wmh-tune 6\n1024 0 64 4 3 64 8 1 3 1 1 0.5\n")  # R = 3 is not a plan
        with pytest.raises(wmh.WMHError) as e:
            fresh.tune_load(str(bad))
        assert e.value.name == "WMH_E_ARG"
        with pytest.raises(wmh.WMHError):
            fresh.tune_load(str(tmp_path / "missing.txt"))
    finally:
        fresh.close()


def test_wide_bounds_tune_both_value_forms(ctx, tmp_path):
    """Bounds above 16 bits: the tuner times exact 32-bit rows and coarse codes; whichever it
    keeps is taken by later calls, survives a save/load round trip and gives the oracle's
    values."""
    ds = synth.random_case(seed=17, n_rows=96, D=3000, density=0.05, max_val=3_000_000,
                           bound_slack=500_000, k=40)
    print("  tune wide bounds", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    res = ctx.tune(rows, ds.k, seed=5, reps=1)
    assert res["values"] in ("exact", "coarse")
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, ds.k, seed=5)
    got = wmh.sig_to_numpy(ctx.hash(rows, ds.k, seed=5, mode="batched"))
    assert np.array_equal(got, want)
    assert _plan_of(ctx.last_plan()) == _plan_of(res)
    path = tmp_path / "wide.txt"
    ctx.tune_save(str(path))
    fresh = wmh.Context(0)
    try:
        fresh.set_bounds(ds.m)
        fresh.tune_load(str(path))
        assert np.array_equal(wmh.sig_to_numpy(fresh.hash(rows, ds.k, seed=5, mode="batched")),
                              want)
        assert _plan_of(fresh.last_plan()) == _plan_of(res)
    finally:
        fresh.close()


def _sparse_rows():
    """Rows with tiny green fractions (about 2e4 steps per hash): the planner sends them to the
    component index."""
    return synth.random_case(seed=4, n_rows=300, D=2000, density=0.005, max_val=500,
                             bound_slack=60000, k=64)


def test_index_rows_plan_is_tuned_and_taken(ctx, tmp_path):
    ds = _sparse_rows()
    k = ds.k
    print("  tune index rows", flush=True)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    res = ctx.tune(rows, k, seed=3, reps=1)
    assert res["walk"] == "index", res
    assert res["index_batch"] in (8, 16) and res["index_claim"] in (1, 2)
    assert res["candidates"] >= 8 and 0 < res["best_ms"]
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=3)
    for mode in ("indexed", "auto"):
        got = wmh.sig_to_numpy(ctx.hash(rows, k, seed=3, mode=mode))
        assert np.array_equal(got, want)
        plan = ctx.last_plan()
        assert plan["mode"] == "indexed"
        assert (plan["waves_per_block"], plan["index_batch"], plan["index_claim"]) == \
            (res["waves_per_block"], res["index_batch"], res["index_claim"])
    path = tmp_path / "index_plans.txt"
    ctx.tune_save(str(path))
    assert any(line.split()[7] == "4" for line in path.read_text().splitlines()[1:])
    fresh = wmh.Context(0)
    try:
        fresh.set_bounds(ds.m)
        fresh.tune_load(str(path))
        assert np.array_equal(wmh.sig_to_numpy(fresh.hash(rows, k, seed=3, mode="indexed")), want)
        p = fresh.last_plan()
        assert (p["waves_per_block"], p["index_batch"], p["index_claim"]) == \
            (res["waves_per_block"], res["index_batch"], res["index_claim"])
    finally:
        fresh.close()


def test_index_rows_plans_and_graph_replays(ctx):
    """Every index rows plan gives the oracle's values, launched directly and replayed from a
    graph (with eager work between replays)."""
    ds = _sparse_rows()
    k = ds.k
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=8)
    for W in (1, 2, 4, 8, 16):
        for B in (8, 16):
            for C in ("counter", "stride"):
                for graph in (False, True):
                    got = wmh.sig_to_numpy(ctx.hash(rows, k, seed=8, mode="indexed",
                                                    waves_per_block=W, index_batch=B,
                                                    index_claim=C, use_graph=graph))
                    assert np.array_equal(got, want), (W, B, C, graph)
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device=DEV)
    opts = ctx.make_opts(mode="indexed", waves_per_block=4, index_batch=16, index_claim=1)
    for _ in range(4):
        sig.fill_(-1)
        scratch = torch.randn(1 << 16, device=DEV).sum()  # eager work between replays
        ctx.hash_into(rows, k, 8, sig, opts=opts)
        torch.cuda.synchronize()
        assert float(scratch) == float(scratch)
        assert np.array_equal(wmh.sig_to_numpy(sig), want)
    with pytest.raises(wmh.WMHError) as e:  # 32 wavefronts do not fit a workgroup
        ctx.hash(rows, k, seed=8, mode="indexed", waves_per_block=32)
    assert e.value.name == "WMH_E_ARG"
