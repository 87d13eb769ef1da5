"""GPU parity of the (K, L) banding index: candidate rows of every query equal the oracle's,
in order, including rows equal to the query, empty results, repeated database rows and the
overflow flag."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lsh  # noqa: E402
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


def dev16(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)).to(DEV)


def check(ctx, db, q, K, L, max_out=256):
    print(f"  lsh N={db.shape[0]} Q={q.shape[0]} k={db.shape[1]} K={K} L={L}", flush=True)
    want = lsh.candidates(db, q, K, L)
    ix = ctx.lsh_index(dev16(db), K, L)
    try:
        out, cnt = ix.query(dev16(q), max_out)
    finally:
        ix.close()
    out = out.cpu().numpy().view(np.uint32)
    cnt = cnt.cpu().numpy().view(np.uint32)
    for i, w in enumerate(want):
        assert cnt[i] == len(w), (i, cnt[i], len(w))
        n = min(len(w), max_out)
        assert list(out[i, :n]) == w[:n]


@pytest.mark.parametrize("K,L", [(1, 1), (2, 5), (4, 8), (5, 12), (1, 64), (3, 70)])
def test_random_small_alphabet(ctx, K, L):
    rng = np.random.Generator(np.random.PCG64(K * 100 + L))
    k = K * L + 3
    alphabet = 30 if K == 1 else 3  # keeps a query's band matches below the 2048 buffer
    db = rng.integers(0, alphabet, size=(300, k)).astype(np.uint16)
    db[50] = db[10]  # repeated row
    q = rng.integers(0, alphabet, size=(37, k)).astype(np.uint16)
    q[0] = db[10]
    q[1] = 7  # matches nothing
    check(ctx, db, q, K, L, max_out=64)


def test_real_signatures(ctx):
    ds = synth.config1()
    ctx.set_bounds(ds.m)
    sig = wmh.sig_to_numpy(ctx.hash(wmh.upload_dataset(ds, DEV), ds.k, seed=0))
    check(ctx, sig[100:], sig[:100], K=2, L=32)


def test_overflow_flag(ctx):
    db = np.zeros((3000, 4), dtype=np.uint16)
    q = np.zeros((2, 4), dtype=np.uint16)
    q[1] = 5
    ix = ctx.lsh_index(dev16(db), 1, 1)
    try:
        out, cnt = ix.query(dev16(q), 16)
    finally:
        ix.close()
    cnt = cnt.cpu().numpy().view(np.uint32)
    assert cnt[0] == 0xFFFFFFFF and cnt[1] == 0


def test_bad_parameters(ctx):
    db = dev16(np.zeros((5, 8), dtype=np.uint16))
    with pytest.raises(wmh.WMHError) as e:
        ctx.lsh_index(db, 3, 3)
    assert e.value.name == "WMH_E_ARG"
