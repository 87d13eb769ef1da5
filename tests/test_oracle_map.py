"""Pins for the oracle's red-green map, its ISGREEN and its step count.

Checked against brute force: an explicit per-position colour array built from the Procedure
(Sec. 3.1, eq. redGreen) -- piece i covers m_i consecutive positions, the first x_i green --
with no prefix sums and no search.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from paper_1602_08393_amd import synth


def colour_array(m, x):
    colours = []
    for mi, xi in zip(m, x):
        colours += [True] * int(xi) + [False] * (int(mi) - int(xi))
    return colours


def brute_hash(colours, positions):
    """1-based index of the first green position; len(positions) if none; 0 for no green."""
    if not any(colours):
        return 0
    for t, p in enumerate(positions, start=1):
        if colours[p]:
            return t
    return len(positions)


def _random_vectors(rng, D, max_m, zero_bounds=True):
    m = rng.integers(0 if zero_bounds else 1, max_m + 1, size=D)
    if m.sum() == 0:
        m[rng.integers(0, D)] = 1
    x = np.array([rng.integers(0, mi + 1) for mi in m])
    return m.astype(np.uint32), x.astype(np.uint32)


def test_is_green_exhaustive_against_colour_array(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(300):
        D = int(rng.integers(1, 9))
        m, x = _random_vectors(rng, D, 6)
        colours = colour_array(m, x)
        for p in range(len(colours)):
            assert oracle_lib.is_green_dense(m, x, p) == int(colours[p]), (m, x, p)


def test_is_green_extremes(oracle_lib):
    m = np.array([3, 0, 5, 1, 0, 2], dtype=np.uint32)
    full = m.copy()
    none = np.zeros_like(m)
    for p in range(int(m.sum())):
        assert oracle_lib.is_green_dense(m, full, p) == 1
        assert oracle_lib.is_green_dense(m, none, p) == 0
    # p outside [0, M) and x above the bound are rejected
    assert oracle_lib.is_green_dense(m, full, int(m.sum())) == -1
    bad = full.copy()
    bad[0] = 4
    assert oracle_lib.is_green_dense(m, bad, 0) == -1


def test_hash_from_explicit_positions_matches_brute_force(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(12))
    for _ in range(400):
        D = int(rng.integers(1, 7))
        m, x = _random_vectors(rng, D, 5)
        M = int(m.sum())
        colours = colour_array(m, x)
        cap = int(rng.integers(1, 8))
        positions = rng.integers(0, M, size=cap)
        assert oracle_lib.hash_dense_positions(m, x, positions) == brute_hash(colours, positions)


def test_hash_csr_matches_brute_force_on_generator_positions(oracle_lib):
    """The full oracle (generator positions, default cap) against the colour array walked with
    the same positions, for random tiny rows including empty rows and zero-bound dimensions."""
    for seed in range(6):
        ds = synth.random_case(seed, n_rows=12, D=7, density=0.4, max_val=9, bound_slack=3,
                               empty_rows=2, zero_bound_dims=1, k=24)
        M = int(ds.m.astype(np.uint64).sum())
        X = ds.dense()
        sig = oracle_lib.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, ds.k, seed=seed + 100,
                                  threads=2)
        for r in range(ds.n_rows):
            colours = colour_array(ds.m, X[r])
            for j in range(ds.k):
                want = 0
                if any(colours):
                    t = 1
                    while True:
                        p, _ = oracle_lib.position(seed + 100, j, t, M)
                        if colours[p] or t == 65535:
                            want = t
                            break
                        t += 1
                assert sig[r, j] == want, (seed, r, j)


def test_small_cap_saturates(oracle_lib):
    """With cap H the value is H exactly when the first H-1 draws are all red."""
    m = np.array([1000, 1000], dtype=np.uint32)
    x = np.array([1, 0], dtype=np.uint32)     # s = 1/2000
    sig = oracle_lib.hash_dense(m, x[None, :], k=400, seed=3, cap=5)
    assert set(np.unique(sig)) <= {1, 2, 3, 4, 5}
    assert (sig == 5).mean() > 0.95
    sig_full = oracle_lib.hash_dense(m, x[None, :], k=400, seed=3)
    # below the cap the two agree; at the cap the uncapped value is >= cap
    small = sig[0] < 5
    assert np.array_equal(sig[0][small], sig_full[0][small])
    assert np.all(sig_full[0][~small] >= 5)


def test_exact_enumeration_of_collision_probability(oracle_lib):
    """Over every position sequence of length H (each equally likely), the fraction of
    sequences on which x and y get the same value equals the capped closed form, and as H grows
    that closed form approaches the generalized Jaccard (Theorem 1)."""
    cases = [
        ([2, 1, 3], [1, 1, 2], [2, 0, 3]),
        ([1, 1, 1, 1], [1, 0, 1, 0], [1, 1, 0, 0]),      # binary case: J = |x & y| / |x | y|
        ([3, 2], [3, 0], [0, 2]),                         # disjoint supports
        ([4, 1], [2, 1], [4, 1]),                         # x <= y
        ([2, 0, 3], [1, 0, 1], [1, 0, 1]),                # identical, with a zero-bound piece
    ]
    for m, x, y in cases:
        m = np.array(m, dtype=np.uint32)
        x = np.array(x, dtype=np.uint32)
        y = np.array(y, dtype=np.uint32)
        M = int(m.sum())
        for H in (1, 2, 3, 4):
            hits = 0
            pmf_x = Fraction(0)
            total = M ** H
            values_x = {}
            for seq in itertools.product(range(M), repeat=H):
                hx = oracle_lib.hash_dense_positions(m, x, seq)
                hy = oracle_lib.hash_dense_positions(m, y, seq)
                hits += hx == hy
                values_x[hx] = values_x.get(hx, 0) + 1
            got = Fraction(hits, total)
            assert got == oracle_lib.capped_collision(x, y, M, H), (m, x, y, H)
            # step-count law of x (Theorem 2, truncated at H): Pr(h = t) = (1-s)^(t-1) s
            s = Fraction(int(x.sum()), M)
            for t in range(1, H):
                assert Fraction(values_x.get(t, 0), total) == (1 - s) ** (t - 1) * s
            assert Fraction(values_x.get(H, 0), total) == (1 - s) ** (H - 1)
        J = oracle_lib.jaccard(x, y)
        assert abs(float(oracle_lib.capped_collision(x, y, M, 400)) - float(J)) < 1e-12
