"""GPU quantization of real values (Sec. 4, Practical Issues) against the oracle, bit for bit,
then the quantized rows hashed on the GPU against the oracle's hashes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import scale  # noqa: E402
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


@pytest.mark.parametrize("limit", [65535, 0, 1000])
def test_quantize_then_hash(ctx, limit):
    print(f"  quantize limit={limit}", flush=True)
    rng = np.random.Generator(np.random.PCG64(limit + 5))
    N, D = 60, 700
    mask = rng.random((N, D)) < 0.1
    X = np.zeros((N, D), dtype=np.float32)
    X[mask] = rng.lognormal(0.0, 1.5, size=int(mask.sum())).astype(np.float32)
    X[3] = 0.0  # an empty row
    rows, cols = np.nonzero(X)
    row_ptr = np.zeros(N + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(np.bincount(rows, minlength=N))
    x = X[rows, cols]
    m = np.maximum(X.max(axis=0).astype(np.float64), 1e-3)
    alpha, eff, m_q = wmh.choose_scale(m, limit=limit)
    assert eff > 0.5
    want, want_clip = scale.quantize(x, cols, m_q, alpha)
    ctx.set_bounds(m_q)
    got, clipped = ctx.quantize(torch.from_numpy(x).to(DEV),
                                torch.from_numpy(cols.astype(np.uint32).view(np.int32)).to(DEV),
                                alpha)
    got = got.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want) and clipped == want_clip == 0
    ds = synth.Dataset("quantized", m_q, row_ptr, cols.astype(np.uint32), got, 64)
    sig = wmh.sig_to_numpy(ctx.hash(wmh.upload_dataset(ds, DEV), 64, seed=1))
    assert np.array_equal(sig, oracle.hash_csr(m_q, row_ptr, ds.col, got, 64, seed=1))
    assert np.all(sig[3] == 0)


def test_values_above_the_bound_are_clipped(ctx):
    m = np.array([10.0, 20.0])
    alpha, _, m_q = wmh.choose_scale(m, limit=1000)
    ctx.set_bounds(m_q)
    x = np.array([5.0, 30.0, 20.0], dtype=np.float32)
    col = np.array([0, 1, 1], dtype=np.uint32)
    got, clipped = ctx.quantize(torch.from_numpy(x).to(DEV),
                                torch.from_numpy(col.view(np.int32)).to(DEV), alpha)
    want, want_clip = scale.quantize(x, col, m_q, alpha)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    assert clipped == want_clip == 1
