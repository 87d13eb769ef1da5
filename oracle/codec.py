"""CPU oracle of the b-bit signature codec.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Hash values are geometric with mean 1/s (Theorem 2), hence small with high probability
(Corollary 1), and the paper stores them in a few bits each (Table 3: 5-9 bits on its data).
The stored form written out here, field by field:

* a row of k values packs into W = ceil(k / f) uint32 words, f = floor(32 / b) fields a word;
* value j goes to word j // f, bits [(j mod f) * b, (j mod f) * b + b); other bits are 0;
* a value above 2^b - 1 is stored as 2^b - 1 (saturated);
* two packed rows collide on hash j when their stored values at j are equal.

Plain loops over fields, no word-level tricks: the GPU counts equal fields with a carry-free
test on xored words; this module unpacks and compares.
"""
from __future__ import annotations

import numpy as np


def fields_per_word(bits: int) -> int:
    if not 1 <= bits <= 16:
        raise ValueError("bits must be in [1, 16]")
    return 32 // bits


def pack_words(k: int, bits: int) -> int:
    f = fields_per_word(bits)
    return -(-k // f)


def lossless_bits(sig: np.ndarray) -> int:
    """Smallest b >= 1 with every value < 2^b."""
    top = int(np.max(sig)) if np.size(sig) else 0
    return max(1, top.bit_length())


def pack(sig: np.ndarray, bits: int) -> tuple[np.ndarray, int]:
    """(packed uint32 [N, W], number of saturated values)."""
    sig = np.atleast_2d(np.asarray(sig, dtype=np.uint16))
    n, k = sig.shape
    f = fields_per_word(bits)
    top = (1 << bits) - 1
    out = np.zeros((n, pack_words(k, bits)), dtype=np.uint64)
    saturated = 0
    for r in range(n):
        for j in range(k):
            v = int(sig[r, j])
            if v > top:
                saturated += 1
                v = top
            out[r, j // f] |= v << ((j % f) * bits)
    return out.astype(np.uint32), saturated


def unpack(packed: np.ndarray, k: int, bits: int) -> np.ndarray:
    packed = np.atleast_2d(np.asarray(packed, dtype=np.uint32))
    n = packed.shape[0]
    f = fields_per_word(bits)
    top = (1 << bits) - 1
    out = np.zeros((n, k), dtype=np.uint16)
    for r in range(n):
        for j in range(k):
            out[r, j] = (int(packed[r, j // f]) >> ((j % f) * bits)) & top
    return out


def packed_collisions(A: np.ndarray, B: np.ndarray, k: int, bits: int) -> np.ndarray:
    """counts[a, b] = number of hashes j whose stored values agree (all pairs)."""
    ua = unpack(A, k, bits)
    ub = unpack(B, k, bits)
    counts = np.zeros((ua.shape[0], ub.shape[0]), dtype=np.uint32)
    for a in range(ua.shape[0]):
        counts[a] = (ub == ua[a]).sum(axis=1)
    return counts
