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
            res["steps_per_lane"])


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
    assert path.read_text().startswith("wmh-tune 3\n")
    fresh = wmh.Context(0)
    try:
        fresh.set_bounds(ds.m)
        fresh.tune_load(str(path))
        fresh.hash(rows, ds.k, seed=0, mode="batched")
        p = fresh.last_plan()
        assert _plan_of(p) == _plan_of(res)
        bad = tmp_path / "bad.txt"
        bad.write_text("wmh-tune 3\n1024 0 64 4 3 64 8 1 3 0.5\n")  # R = 3 is not a plan
        with pytest.raises(wmh.WMHError) as e:
            fresh.tune_load(str(bad))
        assert e.value.name == "WMH_E_ARG"
        with pytest.raises(wmh.WMHError):
            fresh.tune_load(str(tmp_path / "missing.txt"))
    finally:
        fresh.close()
