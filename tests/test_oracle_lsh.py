"""Pins of the banding oracle: brute force over all pairs and bands on small inputs, and the
banding probability 1 - (1 - J^K)^L on pairs whose hashes agree independently with
probability J, within a binomial confidence interval."""
import math

import numpy as np
import pytest

from oracle import lsh


def test_matches_brute_force():
    rng = np.random.Generator(np.random.PCG64(4))
    db = rng.integers(0, 3, size=(40, 12)).astype(np.uint16)
    q = rng.integers(0, 3, size=(9, 12)).astype(np.uint16)
    q[0] = db[7]
    for K, L in [(1, 1), (2, 3), (3, 4), (4, 2), (6, 2), (12, 1)]:
        got = lsh.candidates(db, q, K, L)
        for i in range(q.shape[0]):
            want = [r for r in range(db.shape[0])
                    if any(np.array_equal(db[r, b * K:(b + 1) * K], q[i, b * K:(b + 1) * K])
                           for b in range(L))]
            assert got[i] == want
        assert 7 in got[0]


@pytest.mark.parametrize("J,K,L", [(0.5, 3, 5), (0.8, 5, 4), (0.3, 2, 10)])
def test_banding_probability(J, K, L):
    rng = np.random.Generator(np.random.PCG64(int(J * 100) + K + L))
    n, k = 4000, K * L
    q = rng.integers(0, 1 << 15, size=(1, k)).astype(np.uint16)
    same = rng.random((n, k)) < J
    db = np.where(same, q, q + 1 + rng.integers(0, 100, size=(n, k))).astype(np.uint16)
    hits = len(lsh.candidates(db, q, K, L)[0])
    p = lsh.candidate_probability(J, K, L)
    sd = math.sqrt(n * p * (1 - p))
    assert abs(hits - n * p) < 6 * sd + 1


def test_bad_parameters():
    with pytest.raises(ValueError):
        lsh.candidates(np.zeros((2, 4), np.uint16), np.zeros((1, 4), np.uint16), 3, 2)
