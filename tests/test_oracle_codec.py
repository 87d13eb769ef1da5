"""Pins of the b-bit codec oracle against what the definition fixes: exhaustive round trips at
every width, saturation counted directly, collision counts equal to the C oracle's uint16
comparison when the width is lossless, the word count, and the minimal lossless width."""
import numpy as np
import pytest

import oracle
from oracle import codec


@pytest.mark.parametrize("bits", range(1, 17))
def test_every_value_round_trips(bits):
    top = (1 << bits) - 1
    values = np.arange(0, min(top, 65535) + 1, dtype=np.uint16)
    if len(values) > 4099:  # sample wide widths: both ends and a stride through the middle
        values = np.unique(np.concatenate([values[:1500], values[-1500:], values[::37]]))
    k = len(values)
    packed, sat = codec.pack(values[None, :], bits)
    assert sat == 0
    assert packed.shape == (1, -(-k // (32 // bits)))
    assert np.array_equal(codec.unpack(packed, k, bits)[0], values)


def test_layout_of_one_row():
    # 5-bit fields: six per word, the seventh value starts the second word
    packed, _ = codec.pack(np.array([[1, 2, 3, 4, 5, 6, 7]], dtype=np.uint16), 5)
    w0, w1 = int(packed[0, 0]), int(packed[0, 1])
    assert [(w0 >> (5 * i)) & 31 for i in range(6)] == [1, 2, 3, 4, 5, 6]
    assert w0 >> 30 == 0 and w1 == 7


def test_saturation():
    rng = np.random.Generator(np.random.PCG64(1))
    sig = rng.integers(0, 65536, size=(5, 77)).astype(np.uint16)
    for bits in (3, 7, 9, 15):
        top = (1 << bits) - 1
        packed, sat = codec.pack(sig, bits)
        assert sat == int((sig.astype(np.int64) > top).sum())
        assert np.array_equal(codec.unpack(packed, 77, bits), np.minimum(sig, top))


def test_collisions_equal_uint16_collisions_when_lossless(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(2))
    A = rng.geometric(0.05, size=(7, 45)).clip(1, 65535).astype(np.uint16)
    B = A.copy()
    B[::2, ::3] = rng.geometric(0.05, size=B[::2, ::3].shape).clip(1, 65535)
    bits = codec.lossless_bits(np.concatenate([A, B]))
    pa, sa = codec.pack(A, bits)
    pb, sb = codec.pack(B, bits)
    assert sa == 0 and sb == 0
    want = oracle.collisions_all_pairs(A, B)
    assert np.array_equal(codec.packed_collisions(pa, pb, 45, bits), want)
    # one bit less saturates and can only add collisions
    if bits > 1:
        qa, _ = codec.pack(A, bits - 1)
        qb, _ = codec.pack(B, bits - 1)
        assert np.all(codec.packed_collisions(qa, qb, 45, bits - 1) >= want)


def test_minimal_lossless_width():
    for top in (0, 1, 2, 3, 31, 32, 1000, 65535):
        sig = np.array([[0, top]], dtype=np.uint16)
        b = codec.lossless_bits(sig)
        assert top < (1 << b) and (b == 1 or top >= (1 << (b - 1)))
        assert codec.pack(sig, b)[1] == 0
        if b > 1:
            assert codec.pack(sig, b - 1)[1] == 1


def test_word_count():
    for bits in range(1, 17):
        f = 32 // bits
        for k in (1, f - 1 or 1, f, f + 1, 500, 1000):
            assert codec.pack_words(k, bits) == (k + f - 1) // f
    with pytest.raises(ValueError):
        codec.pack_words(10, 17)
