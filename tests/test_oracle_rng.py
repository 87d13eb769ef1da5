"""Pins for the oracle's random sequence: Philox4x32-10 and the bounded draw.

The paper only asks for a consistent uniform sequence shared by every vector (Sec. 3.1, the
consistency paragraph after Definition 1).  The readings fixed here: Philox4x32-10 as the
counter-based generator and Lemire's multiply-and-reject as the exactly uniform bounded draw.
"""
import os
from collections import Counter

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            words = [int(w, 16) for w in line.split()]
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expected", _kat_rows())
def test_philox_known_answers(oracle_lib, ctr, key, expected):
    assert oracle_lib.philox4x32_10(ctr, key) == tuple(expected)


@pytest.mark.parametrize("bits", [8, 12])
def test_bounded_draw_exhaustive_small_words(oracle_lib, bits):
    """At a reduced word width every value of {0..n-1} must come from exactly
    floor(2^bits / n) accepted words and 2^bits mod n words must be rejected."""
    space = 1 << bits
    for n in list(range(1, 70)) + [space - 1, space, space // 2 + 1, 3 * space // 4 + 3]:
        counts = Counter()
        rejected = 0
        for u in range(space):
            v = oracle_lib.bounded_draw(u, n, bits)
            if v is None:
                rejected += 1
            else:
                assert 0 <= v < n
                counts[v] += 1
        assert rejected == space % n, (n, rejected)
        assert set(counts) == set(range(n))
        assert set(counts.values()) == {space // n}, n


def test_bounded_draw_exhaustive_16bit_selected(oracle_lib):
    space = 1 << 16
    for n in (1, 3, 1000, 40000, 65535):
        counts = np.zeros(n, dtype=np.int64)
        rejected = 0
        for u in range(space):
            v = oracle_lib.bounded_draw(u, n, 16)
            if v is None:
                rejected += 1
            else:
                counts[v] += 1
        assert rejected == space % n
        assert counts.min() == counts.max() == space // n


def test_bounded_draw_64bit_matches_integer_definition(oracle_lib):
    """At 64 bits: value = floor(u n / 2^64), accepted iff (u n mod 2^64) >= 2^64 mod n."""
    rng = np.random.Generator(np.random.PCG64(7))
    space = 1 << 64
    ns = [1, 2, 3, (1 << 32) - 1, 1 << 32, (1 << 57) + 1, (1 << 63) + 1, space - 1, 66411476]
    for n in ns:
        for _ in range(200):
            u = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
            got = oracle_lib.bounded_draw(u, n, 64)
            prod = u * n
            want = prod >> 64 if (prod % space) >= space % n else None
            assert got == want


def test_position_layout_pairs_of_steps(oracle_lib):
    """Step t of hash j uses the Philox block at counter ((t-1)//2, j, 0, 0): its low 64 bits
    for odd t, its high 64 bits for even t (when the first block is accepted)."""
    seed = 0x0123456789ABCDEF
    key = (seed & 0xFFFFFFFF, seed >> 32)
    M = 66411476
    for j in (0, 1, 7, 499, 123456):
        for t in (1, 2, 3, 4, 99, 100, 65535):
            w = oracle_lib.philox4x32_10(((t - 1) // 2, j, 0, 0), key)
            half = (t - 1) & 1
            u = (w[2 * half + 1] << 32) | w[2 * half]
            expect = oracle_lib.bounded_draw(u, M, 64)
            got, used = oracle_lib.position(seed, j, t, M)
            assert used == 1 and got == expect


def test_position_redraw_uses_next_attempt_counter(oracle_lib):
    """With M = 2^57 + 1 about 1 word in 128 is rejected; a rejected step redraws from the block
    at counter ((t-1)//2, j, a, 0) for a = 1, 2, ..., same half."""
    M = (1 << 57) + 1
    seed = 5
    key = (seed, 0)
    found = 0
    for j in range(4):
        for t in range(1, 2000):
            p, used = oracle_lib.position(seed, j, t, M)
            assert 0 <= p < M
            if used > 1:
                found += 1
                half = (t - 1) & 1
                for a in range(used):
                    w = oracle_lib.philox4x32_10(((t - 1) // 2, j, a, 0), key)
                    u = (w[2 * half + 1] << 32) | w[2 * half]
                    v = oracle_lib.bounded_draw(u, M, 64)
                    if a < used - 1:
                        assert v is None
                    else:
                        assert v == p
    assert found > 20  # about 8000 / 128 expected


@pytest.mark.parametrize("M", [1, 2, 5, 17, 1000])
def test_positions_uniform(oracle_lib, M):
    counts = np.zeros(M, dtype=np.int64)
    n = 0
    for j in range(40):
        for t in range(1, 1 + max(50, 30 * M // 40)):
            p, _ = oracle_lib.position(2024, j, t, M)
            counts[p] += 1
            n += 1
    if M == 1:
        assert counts[0] == n
        return
    chi2, pval = stats.chisquare(counts)
    assert pval > 1e-6, (M, chi2)


def test_hash_ids_and_seeds_change_the_sequence(oracle_lib):
    M = 10 ** 9
    a = [oracle_lib.position(0, 0, t, M)[0] for t in range(1, 50)]
    b = [oracle_lib.position(0, 1, t, M)[0] for t in range(1, 50)]
    c = [oracle_lib.position(1, 0, t, M)[0] for t in range(1, 50)]
    d = [oracle_lib.position(1 << 32, 0, t, M)[0] for t in range(1, 50)]
    assert len({tuple(a), tuple(b), tuple(c), tuple(d)}) == 4
    assert len(set(a)) == len(a)
