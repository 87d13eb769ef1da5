"""GPU parity: the HIP library through its C-ABI against the CPU oracle, bit for bit.

Signatures are integers, so the bar is exact equality.  Inputs come from the seeded generators
in paper_1602_08393_amd.synth; the oracle never sees the GPU's outputs except to compare.
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


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, j = bad[0]
        raise AssertionError(f"{what}: {len(bad)} of {want.size} differ; first at row {r} hash "
                             f"{j}: gpu {got[r, j]} oracle {want[r, j]}")


# ---------------------------------------------------------------------------------------------
# A3/A4: the position sequence and the component lookup
# ---------------------------------------------------------------------------------------------

def test_draws_match_oracle_config1(ctx):
    ds = synth.config1()
    ctx.set_bounds(ds.m)
    M = int(ds.m.astype(np.uint64).sum())
    P = np.concatenate([[0], np.cumsum(ds.m.astype(np.uint64))]).astype(np.uint64)
    for seed in (0, 0x0123456789ABCDEF):
        pos, comp, off = ctx.draws(seed, 5, 6, 301)
        for jj in range(6):
            for t in range(1, 302):
                p, _ = oracle.position(seed, 5 + jj, t, M)
                assert int(pos[jj, t - 1]) == p
        c = np.searchsorted(P[:-1], pos, side="right") - 1
        assert np.array_equal(comp, c.astype(np.uint32))
        assert np.array_equal(off, pos - P[c])


def test_draws_redraw_path_at_huge_total(ctx):
    """M = ceil(2^64 / 4097), so 2^64 mod M is close to M and about one word in 4097 is
    rejected and redrawn."""
    D = 1 << 20
    target = -(-(1 << 64) // 4097)
    m = np.full(D, target // D, dtype=np.uint64)
    m[: target - int(m.sum())] += 1
    m = m.astype(np.uint32)
    ctx.set_bounds(m)
    M = int(m.astype(np.uint64).sum())
    assert M == target and ((1 << 64) % M) > 0.99 * M
    depth, nh = 2048, 32
    pos, comp, off = ctx.draws(99, 1000, nh, depth)
    redraws = 0
    for jj in range(nh):
        for t in range(1, depth + 1):
            p, used = oracle.position(99, 1000 + jj, t, M)
            redraws += used > 1
            assert int(pos[jj, t - 1]) == p, (jj, t)
    assert redraws >= 5
    P = np.concatenate([[0], np.cumsum(m.astype(np.uint64))]).astype(np.uint64)
    c = np.searchsorted(P[:-1], pos, side="right") - 1
    assert np.array_equal(comp, c.astype(np.uint32))
    assert np.array_equal(off, pos - P[c])


def test_draws_with_zero_bounds_and_clusters(ctx):
    rng = np.random.Generator(np.random.PCG64(3))
    D = 5000
    m = np.where(rng.random(D) < 0.8, rng.integers(0, 2, D), rng.integers(1, 2 ** 32, D))
    m = m.astype(np.uint32)
    ctx.set_bounds(m)
    P = np.concatenate([[0], np.cumsum(m.astype(np.uint64))]).astype(np.uint64)
    pos, comp, off = ctx.draws(7, 0, 16, 1000)
    c = np.searchsorted(P[:-1], pos, side="right") - 1
    assert np.array_equal(comp, c.astype(np.uint32))
    assert np.all(m[comp] > 0)
    assert np.array_equal(off, pos - P[c])
    assert np.all(off < m[comp].astype(np.uint64))


# ---------------------------------------------------------------------------------------------
# Whole signatures
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("opts", [
    dict(mode="plain"),
    dict(mode="plain", batch_rows=100),
    dict(mode="batched"),
    dict(mode="batched", use_graph=False),
    dict(mode="batched", walk="rows"),
    dict(mode="batched", walk="rows", use_graph=False, hashes_per_tile=17),
    dict(mode="batched", walk="ballot"),
    dict(mode="batched", walk="ballot", use_graph=False, hashes_per_tile=13, waves_per_block=3),
    dict(mode="auto"),
    # the batched walk's kernels scheduled plainly: a launch per batch, a workgroup per tile
    dict(mode="plain_shared"),
    dict(mode="plain_shared", batch_rows=100, walk="ballot"),
    dict(mode="plain_shared", batch_rows=77, walk="rows"),
    dict(mode="plain_shared", batch_rows=33, rows_per_block=4, hashes_per_tile=7),
    # the ballot walk with its hash ids in groups, one tile counter each
    dict(mode="batched", walk="ballot", hash_groups=8),
    dict(mode="batched", walk="ballot", hash_groups=3, use_graph=False, waves_per_block=5),
    dict(mode="plain_shared", walk="ballot", hash_groups=4, batch_rows=300),
])
def test_config1_full(ctx, opts):
    ds = synth.config1()
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, ds.k, seed=0)
    assert_same(gpu_sig(ctx, ds, ds.k, 0, **opts), want, f"config1 {opts}")


BATCHED_PLANS = [
    dict(rows_per_block=1), dict(rows_per_block=2), dict(rows_per_block=4),
    dict(rows_per_block=8), dict(rows_per_block=16),
    dict(rows_per_block=4, hashes_per_tile=7),
    dict(rows_per_block=8, waves_per_block=1), dict(rows_per_block=2, waves_per_block=16),
    dict(rows_per_block=4, stream_depth=None),   # every draw made in-lane
    dict(rows_per_block=4, stream_depth=64),     # stream for the first window only
    # four steps per lane with one or two rows: windows of 256 and 128 steps
    dict(rows_per_block=1, steps_per_lane=4), dict(rows_per_block=2, steps_per_lane=4),
    dict(rows_per_block=1, steps_per_lane=4, stream_depth=None),
    dict(rows_per_block=2, steps_per_lane=4, stream_depth=200, hashes_per_tile=9),
    # independent rows: each row of a block walks its own hash ids
    dict(walk="rows"), dict(walk="rows", hashes_per_tile=7),
    dict(walk="rows", waves_per_block=1), dict(walk="rows", waves_per_block=16),
    dict(walk="rows", stream_depth=None), dict(walk="rows", stream_depth=128),
    # ballot walk: one row per block, first green step from the window's ballot
    dict(walk="ballot"), dict(walk="ballot", hashes_per_tile=7),
    dict(walk="ballot", waves_per_block=1), dict(walk="ballot", waves_per_block=16),
    dict(walk="ballot", stream_depth=None), dict(walk="ballot", stream_depth=64),
    dict(walk="ballot", stream_depth=200, hashes_per_tile=9),
    dict(walk="ballot", hash_groups=2), dict(walk="ballot", hash_groups=8, waves_per_block=4),
    dict(walk="ballot", hash_groups=5, stream_depth=64),
    dict(walk="ballot", hash_groups=8, stream_depth=None),
    # dense rows as 16-bit coarse codes (ties settled from the exact value and offset)
    dict(values="coarse", rows_per_block=1), dict(values="coarse", rows_per_block=2),
    dict(values="coarse", rows_per_block=4), dict(values="coarse", rows_per_block=4,
                                                  hashes_per_tile=7, waves_per_block=3),
    dict(values="coarse", rows_per_block=1, steps_per_lane=4),
    dict(values="coarse", rows_per_block=2, steps_per_lane=4, stream_depth=200),
    dict(values="coarse", rows_per_block=4, stream_depth=None),
    dict(values="coarse", rows_per_block=4, stream_depth=64),
    dict(values="coarse", walk="ballot"), dict(values="coarse", walk="ballot", stream_depth=64),
    dict(values="coarse", walk="ballot", stream_depth=None, hashes_per_tile=9),
    dict(values="exact", rows_per_block=2),
    # codes of 1 to 4 bits: most tested steps in a row's support tie and are settled exactly
    # (in-lane draws, the row's CSR value), in the stream windows and past the stream
    dict(values="coarse", coarse_bits=1, rows_per_block=4),
    dict(values="coarse", coarse_bits=2, rows_per_block=2, steps_per_lane=4),
    dict(values="coarse", coarse_bits=3, rows_per_block=1, steps_per_lane=4, stream_depth=256),
    dict(values="coarse", coarse_bits=1, walk="ballot"),
    dict(values="coarse", coarse_bits=4, walk="ballot", stream_depth=64, hashes_per_tile=5),
    dict(values="coarse", coarse_bits=2, rows_per_block=4, stream_depth=None),
]

CASES = {
    # name: (generator kwargs, k, seed)
    "ragged-empty-zero-dims": (dict(seed=1, n_rows=37, D=300, density=0.2, max_val=60000,
                                    bound_slack=5000, empty_rows=5, zero_bound_dims=20), 70, 11),
    "wide-values": (dict(seed=2, n_rows=29, D=257, density=0.1, max_val=2 ** 32 - 1,
                         bound_slack=0, empty_rows=1), 33, 12),
    "dense-small-D": (dict(seed=3, n_rows=50, D=1, density=1.0, max_val=100, bound_slack=300), 65,
                      13),
    "sparse-slow": (dict(seed=4, n_rows=19, D=2000, density=0.005, max_val=500,
                         bound_slack=60000), 40, 14),
    # bounds a little above 2^16, where the default coarse codes cover two to four integers
    # each (ties stay rare: the plans with few code bits below make them frequent)
    "coarse-near-16-bits": (dict(seed=5, n_rows=45, D=400, density=0.1, max_val=70000,
                                 bound_slack=60000, empty_rows=2), 60, 15),
    "coarse-dense-few-dims": (dict(seed=6, n_rows=23, D=5, density=0.8, max_val=131000,
                                   bound_slack=3), 70, 16),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_random_cases_all_plans(ctx, name):
    kw, k, seed = CASES[name]
    ds = synth.random_case(k=k, **kw)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    assert_same(gpu_sig(ctx, ds, k, seed, mode="plain"), want, f"{name} plain")
    for plan in BATCHED_PLANS:
        got = gpu_sig(ctx, ds, k, seed, mode="batched", **plan)
        assert_same(got, want, f"{name} batched {plan}")
    # the same plans scheduled plainly, in batches of 10 rows (a ragged last batch)
    for plan in BATCHED_PLANS[::3]:
        got = gpu_sig(ctx, ds, k, seed, mode="plain_shared", batch_rows=10, **plan)
        assert_same(got, want, f"{name} plain_shared {plan}")


def test_stream_kept_between_calls(ctx):
    """The shared position stream is built once per (seed, k, depth, bounds) and reused: calls
    that alternate seeds, k, depth and bounds each give the oracle's values, graph replays and
    direct launches alike; a call on a second stream reuses the stream the first one built."""
    ds = synth.random_case(seed=31, n_rows=41, D=700, density=0.05, max_val=9000,
                           bound_slack=500, empty_rows=1, k=50)
    rows = None
    for seed, k, opts in ((3, 50, {}), (4, 50, {}), (3, 50, {}), (3, 20, {}),
                          (3, 50, dict(stream_depth=1000)), (3, 50, dict(use_graph=False)),
                          (4, 50, dict(use_graph=False, stream_depth=1000)), (3, 50, {})):
        ctx.set_bounds(ds.m)
        rows = wmh.upload_dataset(ds, DEV)
        got = wmh.sig_to_numpy(ctx.hash(rows, k, seed=seed, mode="batched", rows_per_block=4,
                                        **opts))
        want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
        assert_same(got, want, f"seed {seed} k {k} {opts}")
    # new bounds with the same seed and k: the stream is rebuilt
    m2 = ds.m.copy()
    m2[::3] += 7
    ctx.set_bounds(m2)
    got = wmh.sig_to_numpy(ctx.hash(rows, 50, seed=3, mode="batched", rows_per_block=4))
    assert_same(got, oracle.hash_csr(m2, ds.row_ptr, ds.col, ds.val, 50, seed=3), "new bounds")
    # asynchronous calls on two streams (ordered, as calls sharing a context must be): the
    # second reuses the stream the first one built
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    out_a = torch.empty((ds.n_rows, 50), dtype=torch.int16, device=DEV)
    out_b = torch.empty_like(out_a)
    ctx.hash_into(rows, 50, 8, out_a, stream=a.cuda_stream,
                  opts=ctx.make_opts(mode="batched", rows_per_block=4, sync=False))
    b.wait_stream(a)
    ctx.hash_into(rows, 50, 8, out_b, stream=b.cuda_stream,
                  opts=ctx.make_opts(mode="batched", rows_per_block=4, sync=False))
    torch.cuda.synchronize()
    want = oracle.hash_csr(m2, ds.row_ptr, ds.col, ds.val, 50, seed=8)
    assert_same(wmh.sig_to_numpy(out_a), want, "stream a")
    assert_same(wmh.sig_to_numpy(out_b), want, "stream b")


def test_two_plane_rows_with_wide_entries(ctx):
    """Four rows of 16-bit values with D * 4 > 65536: the rows sit in two LDS planes of row
    pairs (the second plane starts past byte 65536) and the stream entries are wide (8 bytes),
    for both batched walks and with every draw made in-lane."""
    ds = synth.random_case(seed=21, n_rows=23, D=16500, density=0.004, max_val=30000,
                           bound_slack=3000, empty_rows=2, k=37)
    assert int(ds.m.max()) <= 0xFFFF and ds.D * 4 > 65536
    k = 37
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=9)
    for opts in (dict(rows_per_block=4), dict(rows_per_block=4, stream_depth=None),
                 dict(rows_per_block=4, hashes_per_tile=5, waves_per_block=4),
                 dict(walk="rows"), dict(rows_per_block=2, steps_per_lane=4),
                 dict(walk="ballot"), dict(walk="ballot", stream_depth=None)):
        assert_same(gpu_sig(ctx, ds, k, 9, mode="batched", **opts), want, f"D=16500 {opts}")


def _random_plan(rng):
    """One random plan among every option the batched path takes."""
    w = rng.random()
    walk = "rows" if w < 0.2 else "ballot" if w < 0.4 else "shared"
    plan = dict(mode="batched", walk=walk)
    if walk == "shared":
        R = int(rng.choice([1, 2, 4, 8, 16]))
        plan["rows_per_block"] = R
        if R < 4 and rng.random() < 0.5:
            plan["steps_per_lane"] = 4
    if rng.random() < 0.5:
        plan["hashes_per_tile"] = int(rng.integers(1, 300))
    if rng.random() < 0.5:
        plan["waves_per_block"] = int(rng.choice([1, 2, 4, 8, 16]))
    d = rng.random()
    if d < 0.2:
        plan["stream_depth"] = None
    elif d < 0.6:
        plan["stream_depth"] = int(rng.integers(1, 3000))
    if rng.random() < 0.3:
        plan["use_graph"] = False
    c = rng.random()
    if c < 0.3:
        plan["values"] = "coarse"
        if c < 0.15:
            plan["coarse_bits"] = int(rng.integers(1, 16))
    elif c < 0.45:
        plan["values"] = "exact"
    return plan


@pytest.mark.parametrize("case", range(12))
def test_random_datasets_random_plans(ctx, case):
    """Seeded random datasets (row count, dimension, density, value width, slack, empty rows,
    zero-bound dimensions, k) against the oracle, each under the plain walk, auto mode and
    three random batched plans."""
    rng = np.random.Generator(np.random.PCG64(1000 + case))
    n_rows = int(rng.integers(1, 160))
    D = int(rng.integers(1, 3000))
    max_val = int(rng.choice([3, 255, 65535, 2 ** 20, 2 ** 32 - 1]))
    ds = synth.random_case(seed=2000 + case, n_rows=n_rows, D=D,
                           density=float(rng.uniform(0.002, 0.5)), max_val=max_val,
                           bound_slack=int(rng.choice([0, 10, 5000,
                                                       min(2 ** 32 - 1 - max_val, 300 * max_val)])),
                           empty_rows=int(rng.integers(0, 3)),
                           zero_bound_dims=int(rng.integers(0, 5)) if D > 5 else 0)
    k = int(rng.integers(1, 300))
    seed = int(rng.integers(0, 2 ** 63))
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    assert_same(gpu_sig(ctx, ds, k, seed, mode="plain"), want, f"case {case} plain")
    assert_same(gpu_sig(ctx, ds, k, seed, mode="auto"), want, f"case {case} auto")
    for _ in range(3):
        plan = _random_plan(rng)
        try:
            got = gpu_sig(ctx, ds, k, seed, **plan)
        except wmh.WMHError as e:  # a plan that does not fit this dimension in LDS
            assert e.name == "WMH_E_ARG", (case, plan, e)
            continue
        assert_same(got, want, f"case {case} {plan}")


def test_packed_entries_at_the_offset_limit(ctx):
    """D = 16384 with four rows of 16-bit values: packed entries whose LDS offset c * 4 reaches
    65532, the largest that fits their 16-bit field."""
    ds = synth.random_case(seed=41, n_rows=10, D=16384, density=0.01, max_val=60000,
                           bound_slack=5, empty_rows=1, k=45)
    assert int(ds.m.max()) <= 0xFFFF
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 45, seed=12)
    for opts in (dict(rows_per_block=4), dict(rows_per_block=4, use_graph=False),
                 dict(walk="rows"), dict(walk="ballot")):
        assert_same(gpu_sig(ctx, ds, 45, 12, mode="batched", **opts), want, f"D=16384 {opts}")


def test_coarse_codes_at_their_limits(ctx):
    """Coarse codes at the packed entry's limit (one row of 16-bit codes per block, D = 32768:
    LDS offsets up to 65534); one dimension more and the planner keeps the exact 32-bit rows
    (asking for codes is then an argument error), as it does for code widths above 15 bits."""
    k = 29
    for D, fits in ((32768, True), (32769, False)):
        ds = synth.random_case(seed=47, n_rows=9, D=D, density=0.003, max_val=2 ** 20,
                               bound_slack=1000, empty_rows=1, k=k)
        want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=5)
        assert_same(gpu_sig(ctx, ds, k, 5, mode="batched", walk="ballot"), want, f"D={D} auto")
        assert ctx.last_plan()["values"] == ("coarse" if fits else "exact")
        if fits:
            for opts in (dict(values="coarse", walk="ballot"),
                         dict(values="coarse", rows_per_block=1, coarse_bits=2),
                         dict(values="coarse", walk="ballot", coarse_bits=1, stream_depth=None)):
                assert_same(gpu_sig(ctx, ds, k, 5, mode="batched", **opts), want, f"D={D} {opts}")
            with pytest.raises(wmh.WMHError) as e:
                gpu_sig(ctx, ds, k, 5, mode="batched", values="coarse", coarse_bits=16)
            assert e.value.name == "WMH_E_ARG"
        else:
            with pytest.raises(wmh.WMHError) as e:
                gpu_sig(ctx, ds, k, 5, mode="batched", values="coarse", walk="ballot")
            assert e.value.name == "WMH_E_ARG"


def test_many_hash_ids(ctx):
    """k above 65536: hash ids past 16 bits in the draws, the stream index and many hash
    tiles per row block."""
    ds = synth.random_case(seed=43, n_rows=3, D=40, density=0.6, max_val=900, bound_slack=0,
                           k=70001)
    k = 70001
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=13)
    for opts in (dict(mode="batched"), dict(mode="batched", hashes_per_tile=4096),
                 dict(mode="batched", walk="ballot", hashes_per_tile=4096),
                 dict(mode="batched", walk="ballot", hash_groups=8),
                 dict(mode="plain")):
        assert_same(gpu_sig(ctx, ds, k, 13, **opts), want, f"k={k} {opts}")


def test_full_rows_hash_to_one_and_saturation(ctx):
    """x = m gives h = 1 everywhere; s = 1/2^40 saturates every hash at 65535."""
    m = np.full(256, 0xFFFFFFFF, dtype=np.uint32)
    X = np.zeros((6, 256), dtype=np.uint32)
    X[0] = m
    X[1, 3] = 1
    X[2, 200] = 1
    X[3, :] = m
    X[3, 7] = 0
    ds = synth.csr_from_dense(X, m=m)
    k = 20
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=5)
    assert np.all(want[0] == 1) and np.all(want[1] == 65535)
    for opts in (dict(mode="plain"), dict(mode="batched", rows_per_block=4),
                 dict(mode="batched", rows_per_block=1), dict(mode="batched", rows_per_block=16),
                 dict(mode="batched", rows_per_block=8, stream_depth=70000),
                 dict(mode="batched", rows_per_block=2, stream_depth=128),
                 dict(mode="batched", walk="rows"),
                 dict(mode="batched", walk="rows", stream_depth=None),
                 dict(mode="batched", rows_per_block=1, steps_per_lane=4),
                 dict(mode="batched", rows_per_block=2, steps_per_lane=4, stream_depth=None),
                 dict(mode="batched", walk="ballot"),
                 dict(mode="batched", walk="ballot", stream_depth=70000),
                 dict(mode="batched", walk="ballot", stream_depth=None),
                 dict(mode="batched", walk="ballot", hash_groups=8)):
        assert_same(gpu_sig(ctx, ds, k, 5, **opts), want, f"saturation {opts}")


def test_large_dimension_sparse_rows(ctx):
    """D = 2^20 (dense rows do not fit in LDS): the sparse plain path; includes the redraw
    path of the bounded draw (M near 2^52)."""
    D = 1 << 20
    rng = np.random.Generator(np.random.PCG64(8))
    m = np.full(D, 0xFFFFFFFF, dtype=np.uint32)
    cols, vals = [], []
    for r in range(12):
        c = np.sort(rng.choice(D, size=int(rng.integers(1, 3000)), replace=False))
        cols.append(c)
        vals.append(m[c] - rng.integers(0, 2 ** 20, size=len(c)).astype(np.uint32))
    ds = synth.csr_from_lists(cols, vals, D, m=m)
    k = 24
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=3)
    assert_same(gpu_sig(ctx, ds, k, 3), want, "D=2^20 auto")
    assert_same(gpu_sig(ctx, ds, k, 3, mode="plain"), want, "D=2^20 plain")


def test_config2_head(ctx):
    ds = synth.config2(n_rows=512)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 500, seed=0)
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="plain"), want, "config2 head plain")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="batched"), want, "config2 head batched")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="batched", walk="rows"), want,
                "config2 head independent rows")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="batched", walk="ballot"), want,
                "config2 head ballot walk")


@pytest.fixture(scope="module")
def config4():
    return synth.config4()


def test_config4_head_full_bounds(ctx, config4):
    ds = config4.head(300)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, 500, seed=0)
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="batched"), want, "config4 head batched")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="batched", walk="ballot"), want,
                "config4 head ballot walk")
    assert_same(gpu_sig(ctx, ds, 500, 0, mode="plain"), want, "config4 head plain")


def test_prefix_property_and_determinism(ctx):
    ds = synth.config1().head(200)
    a = gpu_sig(ctx, ds, 64, 9, mode="batched")
    b = gpu_sig(ctx, ds, 500, 9, mode="batched")
    c = gpu_sig(ctx, ds, 500, 9, mode="batched", rows_per_block=16, hashes_per_tile=33)
    d = gpu_sig(ctx, ds, 500, 9, mode="plain", batch_rows=17)
    assert np.array_equal(a, b[:, :64])
    assert np.array_equal(b, c) and np.array_equal(b, d)
    for _ in range(3):
        assert np.array_equal(gpu_sig(ctx, ds, 500, 9, mode="batched"), b)


# ---------------------------------------------------------------------------------------------
# Validation, errors, empty input
# ---------------------------------------------------------------------------------------------

def _rows(rp, col, val):
    return wmh.upload_rows(np.array(rp, np.uint64), np.array(col, np.uint32),
                           np.array(val, np.uint32), DEV)


@pytest.mark.parametrize("rp,col,val,status", [
    ([0, 2, 3], [0, 5, 1], [1, 1, 1], "WMH_E_COL_RANGE"),
    ([0, 2, 3], [1, 1, 1], [1, 1, 1], "WMH_E_UNSORTED"),
    ([0, 2, 3], [2, 1, 1], [1, 1, 1], "WMH_E_UNSORTED"),
    ([0, 2, 3], [0, 1, 2], [1, 9, 1], "WMH_E_BOUND"),
    ([0, 2, 1], [0, 1, 2], [1, 1, 1], "WMH_E_ROW_PTR"),
    ([0, 2, 4], [0, 1, 2], [1, 1, 1], "WMH_E_ROW_PTR"),
])
def test_validation_errors_leave_output_untouched(ctx, rp, col, val, status):
    m = np.array([5, 5, 5, 5], dtype=np.uint32)
    ctx.set_bounds(m)
    rows = _rows(rp, col, val)
    rows.nnz = 3
    for mode in ("plain", "batched"):
        sig = torch.full((2, 8), 0x5A5A, dtype=torch.int16, device=DEV)
        with pytest.raises(wmh.WMHError) as e:
            ctx.hash_into(rows, 8, 0, sig, opts=ctx.make_opts(mode=mode))
        assert e.value.name == status, ctx.last_error()
        assert torch.all(sig == 0x5A5A)
        assert "row" in ctx.last_error()


def test_large_dimension_validation(ctx):
    """Bounds too large for LDS (D = 70000: the validation pass gathers them from memory):
    values at their bound, between a small block neighbour's bound and their own, and small
    ones pass and hash as the oracle does in every mode that holds such rows (plain walk,
    index, auto); a value one above its bound fails with WMH_E_BOUND at the right row, as do a
    column out of range and unsorted columns, and the output stays untouched."""
    rng = np.random.Generator(np.random.PCG64(70))
    D = 70000
    m = rng.integers(1000, 200000, size=D).astype(np.uint32)
    m[::7] = 5  # small bounds between large ones
    ctx.set_bounds(m)
    N, k, seed = 40, 32, 11
    cols, vals = [], []
    for r in range(N):
        c = np.sort(rng.choice(D, size=int(rng.integers(1, 300)), replace=False)).astype(np.uint32)
        kind = r % 3
        if kind == 0:
            v = m[c]  # at the bound
        elif kind == 1:
            v = np.maximum(1, m[c] // 2)
        else:
            v = np.minimum(m[c], 5)
        cols.append(c)
        vals.append(v.astype(np.uint32))
    ds = synth.csr_from_lists(cols, vals, D)
    ds.m[:] = m
    want = oracle.hash_csr(m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    # (no batched plan holds 70000 dense components in LDS)
    for mode in ("plain", "indexed", "auto"):
        assert_same(gpu_sig(ctx, ds, k, seed, mode=mode), want, f"D={D} {mode}")

    big = np.flatnonzero(m > 10000)
    c_bad = int(big[len(big) // 2])
    bad_cols = [c.copy() for c in cols]
    bad_vals = [v.copy() for v in vals]
    bad_cols[17] = np.array([c_bad], np.uint32)
    bad_vals[17] = np.array([int(m[c_bad]) + 1], np.uint32)
    for cc, vv, status, row in (
            (bad_cols, bad_vals, "WMH_E_BOUND", 17),
            ([np.array([3, D], np.uint32)] + cols[1:], [np.array([1, 1], np.uint32)] + vals[1:],
             "WMH_E_COL_RANGE", 0),
            (cols[:5] + [np.array([9, 4], np.uint32)] + cols[6:],
             vals[:5] + [np.array([1, 1], np.uint32)] + vals[6:], "WMH_E_UNSORTED", 5)):
        bad = synth.csr_from_lists(cc, vv, D, m=m)
        rows = wmh.upload_dataset(bad, DEV)
        for mode in ("plain", "indexed", "auto"):
            sig = torch.full((N, k), 0x5A5A, dtype=torch.int16, device=DEV)
            with pytest.raises(wmh.WMHError) as e:
                ctx.hash_into(rows, k, seed, sig, opts=ctx.make_opts(mode=mode))
            assert e.value.name == status, ctx.last_error()
            assert f"row {row}" in ctx.last_error(), ctx.last_error()
            assert torch.all(sig == 0x5A5A)


def test_empty_rows_and_empty_batch(ctx):
    m = np.array([3, 4], dtype=np.uint32)
    ds = synth.csr_from_dense(np.zeros((5, 2), dtype=np.uint32), m=m)
    for mode in ("plain", "batched"):
        assert np.all(gpu_sig(ctx, ds, 10, 0, mode=mode) == 0)
    rows = wmh.upload_rows(np.zeros(1, np.uint64), np.zeros(0, np.uint32),
                           np.zeros(0, np.uint32), DEV)
    ctx.hash_into(rows, 10, 0, torch.empty(0, dtype=torch.int16, device=DEV))


@pytest.mark.parametrize("D", [19456, 19457, 311296, 311297])
def test_validation_bound_modes(ctx, D):
    """The validation pass takes the bounds from LDS up to D = 19456, from a per-block table
    of their minima and means (blocks of 32 components) up to D = 311296, and from memory above:
    at both edges, values at their bound, at the block's smallest bound and between it and
    their own hash as the oracle does under the plain walk and auto, and a value one above its
    bound fails with WMH_E_BOUND at its row in both modes, the output untouched."""
    rng = np.random.Generator(np.random.PCG64(D))
    m = rng.integers(50, 100000, size=D).astype(np.uint32)
    m[::5] = 7  # small bounds beside large ones in every block
    N, k, seed = 24, 24, 3
    cols, vals = [], []
    for r in range(N):
        c = np.sort(rng.choice(D, size=int(rng.integers(1, 400)), replace=False)).astype(np.uint32)
        kind = r % 3
        v = m[c] if kind == 0 else np.minimum(m[c], 7) if kind == 1 else np.maximum(1, m[c] // 3)
        cols.append(c)
        vals.append(v.astype(np.uint32))
    ds = synth.csr_from_lists(cols, vals, D, m=m, name=f"modes-{D}", k=k)
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    for mode in ("plain", "auto"):
        assert_same(gpu_sig(ctx, ds, k, seed, mode=mode), want, f"D={D} {mode}")
    big = np.flatnonzero(m > 1000)
    c_bad = int(big[len(big) // 2])
    bad = synth.csr_from_lists(cols[:9] + [np.array([c_bad], np.uint32)] + cols[10:],
                               vals[:9] + [np.array([int(m[c_bad]) + 1], np.uint32)] + vals[10:],
                               D, m=m)
    ctx.set_bounds(m)
    rows = wmh.upload_dataset(bad, DEV)
    for mode in ("plain", "auto"):
        sig = torch.full((N, k), 0x5A5A, dtype=torch.int16, device=DEV)
        with pytest.raises(wmh.WMHError) as e:
            ctx.hash_into(rows, k, seed, sig, opts=ctx.make_opts(mode=mode))
        assert e.value.name == "WMH_E_BOUND", ctx.last_error()
        assert "row 9" in ctx.last_error(), ctx.last_error()
        assert torch.all(sig == 0x5A5A)


def test_largest_dimension(ctx):
    """D at its largest, 2^26, with the last bound at 2^32 - 1 (the last piece, the end of the
    prefix P and of the bucket table): a row of 2^20 + 2 nonzeros spread over the whole range,
    a row holding only the last component (green fraction about 1/18), an empty row and a row
    too light to find a green step (every hash saturates) equal the oracle under the plain
    walk, the component index (lists of 2^26 components) and auto; no batched plan holds such
    rows, and D = 2^26 + 1 is refused."""
    D = 1 << 26
    rng = np.random.Generator(np.random.PCG64(77))
    m = rng.integers(1, 1000, size=D, dtype=np.uint32)
    m[D - 1] = 0xFFFFFFFF
    c0 = np.unique(np.concatenate([rng.choice(D - 1, size=1 << 20, replace=False),
                                   [0, D - 1]])).astype(np.uint32)
    c3 = np.array([0, 1, 2, D - 3, D - 2], np.uint32)
    ds = synth.csr_from_lists(
        [c0, np.array([D - 1], np.uint32), np.zeros(0, np.uint32), c3],
        [m[c0] // 2 + 1, np.array([1 << 31], np.uint32), np.zeros(0, np.uint32), m[c3]],
        D, m=m, name="largest-D", k=16)
    k, seed = 16, 21
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=seed)
    assert np.all(want[3] == 65535) and np.all(want[2] == 0) and want[1].max() < 1000
    for mode in ("plain", "indexed", "auto"):
        assert_same(gpu_sig(ctx, ds, k, seed, mode=mode), want, f"D=2^26 {mode}")
    rows = wmh.upload_dataset(ds, DEV)
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash(rows, k, seed=seed, mode="batched")
    assert e.value.name == "WMH_E_ARG"
    with pytest.raises(wmh.WMHError) as e:
        ctx.set_bounds(np.ones(D + 1, dtype=np.uint32))
    assert e.value.name == "WMH_E_ARG"


def test_largest_k(ctx):
    """k at its largest, 2^24, on a row with x = m in every dimension: every position is green,
    so every hash is 1 (Def. 1), under the plain walk, the batched walk and auto.  The batched
    planner keeps no shared stream here (one cycle of 2^24 hash ids would exceed its 1 GiB), so
    every step is drawn in-lane.  One more hash id is refused."""
    m = np.array([5, 1, 300, 7, 65535], dtype=np.uint32)
    ds = synth.csr_from_dense(m[None, :].copy(), m=m)
    k = 1 << 24
    for mode in ("plain", "batched", "auto"):
        got = gpu_sig(ctx, ds, k, 3, mode=mode)
        assert got.shape == (1, k), mode
        assert np.all(got == 1), (mode, np.flatnonzero(got != 1)[:5])
        if mode == "batched":
            assert ctx.last_plan()["stream_depth"] == 0, ctx.last_plan()
    rows = wmh.upload_dataset(ds, DEV)
    with pytest.raises(wmh.WMHError) as e:
        ctx.hash(rows, k + 1)
    assert e.value.name == "WMH_E_ARG"


def test_bad_arguments(ctx):
    fresh = wmh.Context(0)
    rows = _rows([0, 1], [0], [1])
    with pytest.raises(wmh.WMHError) as e:
        fresh.hash(rows, 4)
    assert e.value.name == "WMH_E_NO_BOUNDS"
    with pytest.raises(wmh.WMHError) as e:
        fresh.set_bounds(np.zeros(3, dtype=np.uint32))
    assert e.value.name == "WMH_E_OVERFLOW"
    fresh.set_bounds(np.array([2], dtype=np.uint32))
    with pytest.raises(wmh.WMHError) as e:
        fresh.hash(rows, 0)
    assert e.value.name == "WMH_E_ARG"
    fresh.close()


# ---------------------------------------------------------------------------------------------
# A8: estimator and all-pairs collision counts
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("na,nb,k", [(1, 1, 1), (3, 5, 7), (64, 64, 64), (70, 129, 33),
                                     (200, 150, 500)])
def test_collisions_random_signatures(ctx, na, nb, k):
    rng = np.random.Generator(np.random.PCG64(na * 1000 + nb))
    A = rng.integers(0, 4, size=(na, k)).astype(np.uint16)
    B = rng.integers(0, 4, size=(nb, k)).astype(np.uint16)
    A[:, ::5] = 65535
    B[:, ::7] = 65535
    want = oracle.collisions_all_pairs(A, B)
    tA = torch.from_numpy(A.view(np.int16)).to(DEV)
    tB = torch.from_numpy(B.view(np.int16)).to(DEV)
    got = ctx.collisions(tA, tB).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    n = min(na, nb)
    count, jhat = ctx.estimate(tA[:n].contiguous(), tB[:n].contiguous())
    count = count.cpu().numpy().view(np.uint32)
    jhat = jhat.cpu().numpy()
    for i in range(n):
        assert count[i] == oracle.collisions(A[i], B[i])
        assert jhat[i] == oracle.estimate(A[i], B[i])


def test_collisions_on_real_signatures(ctx, config4):
    ds = config4.head(96)
    sig = gpu_sig(ctx, ds, 500, 0)
    A, B = sig[:40], sig[40:]
    want = oracle.collisions_all_pairs(A, B)
    got = ctx.collisions(torch.from_numpy(A.view(np.int16)).to(DEV),
                         torch.from_numpy(B.view(np.int16)).to(DEV)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
