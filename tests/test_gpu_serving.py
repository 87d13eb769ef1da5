"""GPU tests of the serving loop (wmh_server_*): every request's signatures equal the oracle's
and wmh_hash's on the same rows, a request gives the same bytes alone and in a concurrent mix,
admission respects the memory budget, and bad requests are refused at submission."""
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


@pytest.fixture(scope="module")
def corpus():
    return synth.config1()


def _rows(rng, n_corpus, sizes):
    return [rng.integers(0, n_corpus, size=s) for s in sizes]


def _oracle_sig(ds, rows, k, seed):
    sub = ds.rows(rows)
    return oracle.hash_csr(sub.m, sub.row_ptr, sub.col, sub.val, k, seed=seed)


@pytest.mark.parametrize("mode,slots", [("auto", 4), ("plain", 2), ("batched", 1),
                                        ("indexed", 3)])
def test_requests_match_oracle(ctx, corpus, mode, slots):
    k, seed = 48, 21
    print(f"  serving {mode} slots={slots}", flush=True)
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(5))
    row_lists = _rows(rng, corpus.n_rows, [1, 7, 64, 130, 3, 257])
    with serve.Server(ctx, k, seed=seed, slots=slots, mode=mode) as srv:
        reqs = serve.requests_from_corpus(corpus, row_lists, srv)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            assert srv.wait(r.ticket) >= 0
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["hashes"] == sum(len(x) for x in row_lists) * k
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    for rows, r in zip(row_lists, reqs):
        assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, seed))


def test_index_built_at_creation(ctx, corpus):
    """build_index: the loop builds the component index before its first request; requests
    in auto and indexed mode equal the oracle."""
    k, seed = 40, 5
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(16))
    row_lists = _rows(rng, corpus.n_rows, [1, 33, 250])
    for mode in ("auto", "indexed"):
        print(f"  serving {mode} with the index built at creation", flush=True)
        with serve.Server(ctx, k, seed=seed, slots=2, mode=mode, build_index=True) as srv:
            reqs = serve.requests_from_corpus(corpus, row_lists, srv, pinned=True)
            for r in reqs:
                srv.submit(r)
            for r in reqs:
                srv.wait(r.ticket)
        for rows, r in zip(row_lists, reqs):
            assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, seed))


def test_alone_and_in_the_mix_are_identical(ctx, corpus):
    k, seed = 64, 0
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(6))
    probe_rows = rng.integers(0, corpus.n_rows, size=300)
    others = _rows(rng, corpus.n_rows, [500, 1, 40, 999, 77, 300, 2, 600])
    with serve.Server(ctx, k, seed=seed, slots=4) as srv:
        alone = serve.requests_from_corpus(corpus, [probe_rows], srv)[0]
        srv.submit(alone)
        srv.wait(alone.ticket)
        # the mix from page-locked buffers (asynchronous copies), the lone request from pageable
        mix = serve.requests_from_corpus(corpus, others[:4] + [probe_rows] + others[4:], srv,
                                         pinned=True)
        for r in mix:
            srv.submit(r)
        srv.drain()
        for r in mix:
            srv.wait(r.ticket)
    assert np.array_equal(alone.sig, mix[4].sig)
    # and equal to a direct wmh_hash of the same rows
    sub = corpus.rows(probe_rows)
    direct = wmh.sig_to_numpy(ctx.hash(wmh.upload_dataset(sub, DEV), k, seed=seed))
    assert np.array_equal(alone.sig, direct)


def test_memory_budget_queues_requests(ctx, corpus):
    k = 32
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(7))
    row_lists = _rows(rng, corpus.n_rows, [200] * 6)
    with serve.Server(ctx, k, slots=4, mem_budget=1) as probe:
        big = serve.requests_from_corpus(corpus, row_lists[:1], probe)[0]
        with pytest.raises(wmh.WMHError) as e:
            probe.submit(big)
        assert e.value.name == "WMH_E_NOMEM"
    # a budget that holds only one of these requests at a time: the rest wait in the queue
    with serve.Server(ctx, k, slots=4) as sizer:
        reqs = serve.requests_from_corpus(corpus, row_lists, sizer)
    sizes = [(r.n_rows + 1) * 8 + len(r.col) * 8 + r.n_rows * k * 2 for r in reqs]
    budget = int(max(sizes) * 1.3)
    with serve.Server(ctx, k, slots=4, mem_budget=budget) as srv:
        for r in reqs:
            srv.submit(r)
        srv.drain()
        st = srv.stats()
        for r in reqs:
            srv.wait(r.ticket)
    assert st["completed"] == len(reqs)
    assert st["peak_bytes"] <= budget
    assert st["max_queued"] >= 1
    for rows, r in zip(row_lists, reqs):
        assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, 0))


def test_bad_requests_are_refused(ctx, corpus):
    """row_ptr is checked at submission; the entries on the device, before any walk: such a
    request completes with the rule's status and leaves its signatures untouched, and the loop
    goes on serving the requests around it."""
    ctx.set_bounds(corpus.m)
    k = 8
    with serve.Server(ctx, k, slots=2) as srv:
        broken = srv.make_request(np.array([0, 3, 2], np.uint64), np.array([1, 2, 3], np.uint32),
                                  np.array([1, 1, 1], np.uint32))
        with pytest.raises(wmh.WMHError) as e:
            srv.submit(broken)
        assert e.value.name == "WMH_E_ROW_PTR"
        good_rows = [np.arange(0, 5), np.arange(5, 9)]
        good = serve.requests_from_corpus(corpus, good_rows, srv)
        unsorted = srv.make_request(np.array([0, 2], np.uint64), np.array([5, 3], np.uint32),
                                    np.array([1, 1], np.uint32))
        over = srv.make_request(np.array([0, 1], np.uint64), np.array([0], np.uint32),
                                np.array([int(corpus.m[0]) + 1], np.uint32))
        far = srv.make_request(np.array([0, 1], np.uint64), np.array([corpus.D], np.uint32),
                               np.array([1], np.uint32))
        for r in (unsorted, over, far):
            r.sig[:] = 777
        for r in (good[0], unsorted, over, far, good[1]):
            srv.submit(r)
        for r, name in ((unsorted, "WMH_E_UNSORTED"), (over, "WMH_E_BOUND"),
                        (far, "WMH_E_COL_RANGE")):
            with pytest.raises(wmh.WMHError) as e:
                srv.wait(r.ticket)
            assert e.value.name == name
            assert np.all(r.sig == 777)
        for rows, r in zip(good_rows, good):
            srv.wait(r.ticket)
            assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, 0))
        st = srv.stats()
        assert st["rejected"] == 3 and st["failed"] == 0 and st["completed"] == 2
        # bounds cannot change under a live serving loop
        with pytest.raises(wmh.WMHError) as e:
            ctx.set_bounds(corpus.m)
        assert e.value.name == "WMH_E_ARG"
        empty = srv.make_request(np.zeros(1, np.uint64), np.zeros(0, np.uint32),
                                 np.zeros(0, np.uint32))
        srv.wait(srv.submit(empty))
    ctx.set_bounds(corpus.m)


def test_large_dimension_requests(ctx):
    """D = 2^20 (dense rows do not fit in LDS): the loop picks the plain walk or the component
    index per request; both ways the bytes equal the oracle's."""
    D = 1 << 20
    rng = np.random.Generator(np.random.PCG64(9))
    cols, vals = [], []
    for _ in range(40):
        c = np.sort(rng.choice(D, size=int(rng.integers(1, 400)), replace=False))
        cols.append(c)
        vals.append(rng.integers(1, 1000, size=len(c)))
    ds = synth.csr_from_lists(cols, vals, D)
    ds.m[:] = np.maximum(ds.m, 50)
    k = 16
    ctx.set_bounds(ds.m)
    with serve.Server(ctx, k, seed=4, slots=3) as srv:
        row_lists = [np.arange(0, 10), np.arange(10, 40), np.array([3, 3, 7])]
        reqs = serve.requests_from_corpus(ds, row_lists, srv)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            srv.wait(r.ticket)
    for rows, r in zip(row_lists, reqs):
        assert np.array_equal(r.sig, _oracle_sig(ds, rows, k, 4))


def test_requests_overlap_on_the_device(ctx):
    """A burst of slow requests (tiny green fractions, about 2e4 steps per hash) on four slots:
    the device timestamps of their walks overlap, and each result equals wmh_hash's."""
    ds = synth.random_case(seed=4, n_rows=240, D=2000, density=0.005, max_val=500,
                           bound_slack=60000)
    k, seed = 64, 17
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, DEV)
    want = wmh.sig_to_numpy(ctx.hash(rows, k, seed=seed, mode="batched"))
    parts = [np.arange(i, ds.n_rows, 8) for i in range(8)]
    print(f"  serving overlap: {len(parts)} requests of {len(parts[0])} rows", flush=True)
    # one request per slot load, so that the requests themselves overlap
    with serve.Server(ctx, k, seed=seed, slots=4, mode="batched", group_rows=1) as srv:
        reqs = serve.requests_from_corpus(ds, parts, srv, pinned=True)
        for r in reqs:
            srv.submit(r)
        srv.drain()
        for r in reqs:
            srv.wait(r.ticket)
        st = srv.stats()
    assert st["completed"] == len(parts) and st["failed"] == 0
    assert st["max_on_device"] >= 2 and st["max_computing"] >= 2 and st["overlap_s"] > 0, st
    for idx, r in zip(parts, reqs):
        assert np.array_equal(r.sig, want[idx])
    # the counters start afresh after a reset
    with serve.Server(ctx, k, seed=seed, slots=2, mode="batched") as srv:
        r = serve.requests_from_corpus(ds, parts[:1], srv)[0]
        srv.submit(r)
        srv.wait(r.ticket)
        srv.reset_stats()
        st = srv.stats()
    assert st["completed"] == 0 and st["max_computing"] == 0 and st["p50_ms"] == 0


def test_reserved_buffers(ctx, corpus):
    """wmh_server_reserve sizes the slots for the largest request up front: requests up to it,
    and a larger one after it (the slot then grows), all equal the oracle; a reservation beyond
    the memory budget is refused."""
    k, seed = 32, 9
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(23))
    row_lists = _rows(rng, corpus.n_rows, [300, 5, 299, 1, 120])
    rp = corpus.row_ptr.astype(np.int64)
    max_nnz = max(int((rp[r + 1] - rp[r]).sum()) for r in row_lists)
    print(f"  serving with reserved buffers: 300 rows, {max_nnz} nonzeros", flush=True)
    with serve.Server(ctx, k, seed=seed, slots=3, mode="batched", mem_budget=64 << 20) as srv:
        srv.reserve(300, max_nnz)
        reqs = serve.requests_from_corpus(corpus, row_lists, srv, pinned=True)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            srv.wait(r.ticket)
        bigger = serve.requests_from_corpus(corpus, [np.arange(700)], srv)[0]
        srv.submit(bigger)
        srv.wait(bigger.ticket)
        with pytest.raises(wmh.WMHError) as e:
            srv.reserve(10 ** 6, 10 ** 8)
        assert e.value.name == "WMH_E_NOMEM"
    for rows, r in zip(row_lists, reqs):
        assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, seed))
    assert np.array_equal(bigger.sig, _oracle_sig(corpus, np.arange(700), k, seed))


def test_wide_bounds_take_coarse_codes_in_the_loop(ctx):
    """Bounds above 16 bits: the loop's batched walk runs on coarse codes (and on exact rows
    when asked), and every request equals the oracle."""
    ds = synth.random_case(seed=61, n_rows=300, D=900, density=0.05, max_val=5_000_000,
                           bound_slack=100_000, empty_rows=3, k=36)
    k, seed = 36, 13
    ctx.set_bounds(ds.m)
    rng = np.random.Generator(np.random.PCG64(62))
    row_lists = _rows(rng, ds.n_rows, [1, 40, 299, 7])
    print("  serving wide bounds (coarse codes)", flush=True)
    with serve.Server(ctx, k, seed=seed, slots=3, mode="batched") as srv:
        reqs = serve.requests_from_corpus(ds, row_lists, srv, pinned=True)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            srv.wait(r.ticket)
    for rows, r in zip(row_lists, reqs):
        assert np.array_equal(r.sig, _oracle_sig(ds, rows, k, seed))


def _offset_request(srv, req, lead, trail, D):
    """The same rows with `lead` entries before them and `trail` after them in col and val
    (out-of-range columns and huge values, which no check or walk may read): row_ptr starts at
    `lead` and ends before the trailing entries."""
    junk_c = np.full(lead, D + 7, np.uint32), np.full(trail, D + 9, np.uint32)
    junk_v = np.full(lead, 0xFFFFFFFF, np.uint32), np.full(trail, 0xFFFFFFFF, np.uint32)
    return srv.make_request(req.row_ptr + np.uint64(lead),
                            np.concatenate([junk_c[0], req.col, junk_c[1]]),
                            np.concatenate([junk_v[0], req.val, junk_v[1]]))


def test_grouped_requests_equal_alone(ctx, corpus):
    """Requests queued behind a busy slot are admitted together, their rows end to end: each
    request's signatures equal the oracle's on its own rows, also for requests whose row_ptr
    starts past 0 and ends before the last entry, and for requests of empty rows."""
    k, seed = 32, 9
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(19))
    row_lists = [rng.integers(0, corpus.n_rows, size=2000)] + _rows(
        rng, corpus.n_rows, rng.integers(1, 21, size=40))
    with serve.Server(ctx, k, seed=seed, slots=1) as srv:
        reqs = serve.requests_from_corpus(corpus, row_lists, srv)
        reqs = [_offset_request(srv, r, i % 4, (i * 3) % 5, corpus.D) if i % 3 == 1 else r
                for i, r in enumerate(reqs)]
        empty = srv.make_request(np.zeros(4, np.uint64), np.zeros(0, np.uint32),
                                 np.zeros(0, np.uint32))
        reqs.insert(20, empty)
        row_lists.insert(20, None)
        print(f"  serving groups: {len(reqs)} requests on one slot", flush=True)
        for r in reqs:
            srv.submit(r)
        srv.drain()
        for r in reqs:
            srv.wait(r.ticket)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
    assert st["loads"] < st["completed"] // 4, st
    for rows, r in zip(row_lists, reqs):
        if rows is None:
            want = oracle.hash_csr(corpus.m, np.zeros(4, np.uint64), np.zeros(0, np.uint32),
                                   np.zeros(0, np.uint32), k, seed=seed)
        else:
            want = _oracle_sig(corpus, rows, k, seed)
        assert np.array_equal(r.sig, want)


def test_group_rows_limit(ctx, corpus):
    """group_rows bounds the rows admitted together: with 8, requests of three rows go at
    most two to a load; with 1, one each."""
    k, seed = 16, 2
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(23))
    row_lists = _rows(rng, corpus.n_rows, [3] * 24)
    for group_rows, most in ((8, 2), (1, 1)):
        print(f"  serving group_rows={group_rows}", flush=True)
        with serve.Server(ctx, k, seed=seed, slots=1, group_rows=group_rows) as srv:
            reqs = serve.requests_from_corpus(corpus, row_lists, srv)
            for r in reqs:
                srv.submit(r)
            srv.drain()
            for r in reqs:
                srv.wait(r.ticket)
            st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["loads"] * most >= len(reqs), st
        for rows, r in zip(row_lists, reqs):
            assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, seed))


def test_bad_request_inside_a_group(ctx, corpus):
    """A group whose rows fail the check: the request holding the first bad row completes
    with its rule's status, a second bad request with its own after being checked alone, and
    every good request of the group with the oracle's signatures."""
    k, seed = 24, 6
    ctx.set_bounds(corpus.m)
    rng = np.random.Generator(np.random.PCG64(29))
    row_lists = [rng.integers(0, corpus.n_rows, size=1500)] + _rows(
        rng, corpus.n_rows, rng.integers(1, 13, size=16))
    with serve.Server(ctx, k, seed=seed, slots=1) as srv:
        good = serve.requests_from_corpus(corpus, row_lists, srv)
        far = srv.make_request(np.array([0, 1, 2], np.uint64), np.array([3, corpus.D], np.uint32),
                               np.array([1, 1], np.uint32))
        unsorted = srv.make_request(np.array([0, 2], np.uint64), np.array([5, 3], np.uint32),
                                    np.array([1, 1], np.uint32))
        for r in (far, unsorted):
            r.sig[:] = 777
        order = good[:6] + [far] + good[6:11] + [unsorted] + good[11:]
        print(f"  serving a group with bad requests: {len(order)} requests", flush=True)
        for r in order:
            srv.submit(r)
        for r, name in ((far, "WMH_E_COL_RANGE"), (unsorted, "WMH_E_UNSORTED")):
            with pytest.raises(wmh.WMHError) as e:
                srv.wait(r.ticket)
            assert e.value.name == name
            assert np.all(r.sig == 777)
        for r in good:
            srv.wait(r.ticket)
        st = srv.stats()
    assert st["rejected"] == 2 and st["failed"] == 0 and st["completed"] == len(good)
    for rows, r in zip(row_lists, good):
        assert np.array_equal(r.sig, _oracle_sig(corpus, rows, k, seed))


def test_largest_k_request(ctx):
    """A serving loop at k = 2^24 keeps no shared stream (one cycle of its hash ids would exceed
    the stream's 1 GiB) and draws every step in-lane: rows with x = m in every dimension hash to
    1 everywhere (Def. 1), and a later request is served the same way."""
    m = np.array([5, 1, 300, 7, 65535], dtype=np.uint32)
    ds = synth.csr_from_dense(np.stack([m, m, m]), m=m)
    ctx.set_bounds(m)
    k = 1 << 24
    with serve.Server(ctx, k, seed=3, slots=2, mode="batched") as srv:
        reqs = serve.requests_from_corpus(ds, [np.array([0, 2]), np.array([1])], srv)
        for r in reqs:
            srv.submit(r)
        for r in reqs:
            assert srv.wait(r.ticket) >= 0
    for r, n in zip(reqs, (2, 1)):
        assert r.sig.shape == (n, k)
        assert np.all(r.sig == 1)
