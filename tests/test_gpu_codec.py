"""GPU parity of the b-bit signature codec: packed words, unpacked values, the lossless width,
and collision counts on packed rows, all against the oracle's field-by-field definition."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import codec  # noqa: E402
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


def to_dev(a: np.ndarray):
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint16): np.int16, np.dtype(np.uint32): np.int32}[a.dtype]
    return torch.from_numpy(a.view(view)).to(DEV)


def u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def random_sig(seed, n, k, p=0.02):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.geometric(p, size=(n, k)).clip(0, 65535).astype(np.uint16)
    s[rng.random((n, k)) < 0.01] = 65535
    return s


@pytest.mark.parametrize("n,k,bits", [(1, 1, 1), (3, 7, 5), (10, 64, 8), (33, 500, 9),
                                      (5, 1000, 3), (17, 77, 16), (64, 31, 11), (2, 32, 1)])
def test_pack_unpack(ctx, n, k, bits):
    print(f"  pack n={n} k={k} bits={bits}", flush=True)
    sig = random_sig(n * 100 + k, n, k)
    want, want_sat = codec.pack(sig, bits)
    got, sat = ctx.pack(to_dev(sig), bits)
    assert np.array_equal(u32(got), want)
    assert sat == want_sat
    back = wmh.sig_to_numpy(ctx.unpack(got, k, bits))
    assert np.array_equal(back, codec.unpack(want, k, bits))


def test_sig_bits(ctx):
    for top in (0, 1, 2, 5, 63, 64, 1000, 40000, 65535):
        sig = np.zeros((3, 50), dtype=np.uint16)
        sig[1, 17] = top
        b, m = ctx.sig_bits(to_dev(sig))
        assert m == top and b == codec.lossless_bits(sig)


@pytest.mark.parametrize("na,nb,k,bits", [(1, 1, 1, 1), (3, 5, 7, 5), (64, 64, 64, 8),
                                          (70, 129, 33, 9), (65, 1, 500, 16),
                                          (130, 67, 1000, 3), (40, 40, 96, 7)])
def test_packed_collisions(ctx, na, nb, k, bits):
    print(f"  packed collisions {na}x{nb} k={k} bits={bits}", flush=True)
    A = random_sig(na + 7 * k, na, k, p=0.2)
    B = random_sig(nb + 11 * k, nb, k, p=0.2)
    B[: min(na, nb)] = np.where(np.random.Generator(np.random.PCG64(3)).random(
        (min(na, nb), k)) < 0.5, A[: min(na, nb)], B[: min(na, nb)])
    pa, _ = codec.pack(A, bits)
    pb, _ = codec.pack(B, bits)
    want = codec.packed_collisions(pa, pb, k, bits)
    got = u32(ctx.packed_collisions(to_dev(pa), to_dev(pb), k, bits))
    assert np.array_equal(got, want)
    n = min(na, nb)
    count, jhat = ctx.packed_estimate(to_dev(pa[:n]), to_dev(pb[:n]), k, bits)
    assert np.array_equal(u32(count), np.diag(want[:n, :n]))
    assert np.allclose(jhat.cpu().numpy(), np.diag(want[:n, :n]) / k, rtol=0, atol=0)


def test_real_signatures_lossless(ctx):
    ds = synth.config1()
    ctx.set_bounds(ds.m)
    sig = ctx.hash(wmh.upload_dataset(ds, DEV), ds.k, seed=0)
    bits, top = ctx.sig_bits(sig)
    assert bits <= 9  # mean step count ~20 here
    packed, sat = ctx.pack(sig, bits)
    assert sat == 0
    assert torch.equal(ctx.unpack(packed, ds.k, bits), sig)
    A, B = packed[:300].contiguous(), packed[300:700].contiguous()
    direct = ctx.collisions(sig[:300].contiguous(), sig[300:700].contiguous())
    assert torch.equal(ctx.packed_collisions(A, B, ds.k, bits), direct)
    want = oracle.collisions_all_pairs(wmh.sig_to_numpy(sig[:300]), wmh.sig_to_numpy(sig[300:700]))
    assert np.array_equal(u32(direct), want)


def test_bad_widths(ctx):
    sig = to_dev(np.zeros((2, 8), dtype=np.uint16))
    for bits in (0, 17):
        with pytest.raises(wmh.WMHError) as e:
            ctx.pack(sig, bits)
        assert e.value.name == "WMH_E_ARG"
