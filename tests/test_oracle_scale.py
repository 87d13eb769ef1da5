"""Pins of the fixed-point scaling oracle (Sec. 4, Practical Issues) against what the arithmetic
and the objective fix, independent of the oracle's own formulas:

* ``quantize``: exact rational round-half-up where alpha * x and alpha * x + 1/2 are exact in
  IEEE double (dyadic inputs, ties at .5 included), the same rounding within the double
  product's error bound for arbitrary inputs, negative values to 0, and the clip to the bound of
  the value's own column, counted.
* ``objective``: values worked out by hand, and the bound alpha / sum(ceil(alpha m)) <= 1 / sum(m)
  with equality exactly where every alpha * m_i is an integer.
* ``best_breakpoint``: values worked out by hand, the closed form 1 / sum(m) when alpha = 1 is
  allowed, and a dense sweep of alpha over small rationals that never finds a larger objective.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import scale


def _exact_round_half_up(alpha: float, x: float) -> int:
    r = Fraction(alpha) * Fraction(float(x))
    return max(0, math.floor(r + Fraction(1, 2)))


def test_quantize_ties_round_up():
    # alpha * x lands exactly on .5: floor(v + 1/2) rounds up (half-to-even would give 0, 2, 4)
    x = np.array([1.0, 3.0, 5.0, 7.0, 9.0], dtype=np.float32)
    col = np.zeros(5, dtype=np.uint32)
    got, clipped = scale.quantize(x, col, np.array([1000]), 0.5)
    assert got.tolist() == [1, 2, 3, 4, 5] and clipped == 0
    # just below and above a tie
    x = np.array([2.9921875, 3.0078125], dtype=np.float32)  # 3 -+ 2^-7, dyadic
    got, _ = scale.quantize(x, np.zeros(2, dtype=np.uint32), np.array([1000]), 0.5)
    assert got.tolist() == [1, 2]


@pytest.mark.parametrize("seed", range(4))
def test_quantize_dyadic_inputs_are_exact(seed):
    # alpha = a / 2^e and x = b / 2^f with few significant bits: the product is below 2^24 with
    # no bit under 2^-22, so the double product and the added half are exact, and the result must
    # be the exact rational round-half-up
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 4000
    alpha = float(rng.integers(1, 1 << 10)) / float(1 << int(rng.integers(0, 11)))
    b = rng.integers(0, 1 << 14, size=n)
    f = rng.integers(0, 13, size=n)
    x = (b / np.exp2(f)).astype(np.float32)
    assert np.all(x.astype(np.float64) == b / np.exp2(f))  # representable in float32
    col = rng.integers(0, 7, size=n).astype(np.uint32)
    m_q = np.full(7, 1 << 31, dtype=np.int64)
    got, clipped = scale.quantize(x, col, m_q, alpha)
    want = [_exact_round_half_up(alpha, v) for v in x]
    assert clipped == 0
    assert got.tolist() == want


@pytest.mark.parametrize("seed", range(3))
def test_quantize_general_inputs_within_the_rounding_bound(seed):
    # arbitrary alpha and x: the double product is within half an ulp of alpha * x, so the result
    # equals the exact rational round-half-up unless alpha * x + 1/2 lies within that error of an
    # integer (checked to differ by at most 1 there)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    n = 20000
    alpha = float(rng.uniform(0.01, 3000.0))
    x = rng.lognormal(0.0, 2.0, size=n).astype(np.float32)
    got, _ = scale.quantize(x, np.zeros(n, dtype=np.uint32), np.array([1 << 62]), alpha)
    decided = 0
    for q, v in zip(got.tolist(), x):
        r = Fraction(alpha) * Fraction(float(v)) + Fraction(1, 2)
        want = math.floor(r)
        frac = r - want
        tol = Fraction(abs(float(r)) * 2.0 ** -50 + 2.0 ** -60)
        if tol < frac < 1 - tol:
            assert q == want
            decided += 1
        else:
            assert abs(q - want) <= 1
    assert decided >= n - 5


def test_quantize_negative_to_zero_and_clip_by_column():
    x = np.array([-3.0, -0.25, 0.0, 0.2, 10.0, 10.0, 11.0, 4.0], dtype=np.float32)
    col = np.array([0, 0, 0, 0, 0, 1, 1, 2], dtype=np.uint32)
    m_q = np.array([7, 12, 3])
    got, clipped = scale.quantize(x, col, m_q, 1.0)
    # 10 -> 10 clipped to column 0's bound 7; 11 -> 11 within column 1's 12; 4 -> clipped to 3
    assert got.tolist() == [0, 0, 0, 0, 7, 10, 11, 3]
    assert clipped == 2


def test_objective_hand_values():
    # alpha / sum(ceil(alpha * m_i))
    assert scale.objective(Fraction(1), [1, 2]) == Fraction(1, 3)
    assert scale.objective(Fraction(1, 2), [1, 2]) == Fraction(1, 4)       # 1/2 / (1 + 1)
    assert scale.objective(Fraction(3, 2), [1, 2]) == Fraction(3, 10)      # 3/2 / (2 + 3)
    assert scale.objective(Fraction(2, 3), [2, 3]) == Fraction(1, 6)       # 2/3 / (2 + 2)
    assert scale.objective(Fraction(1, 10), [5, 5, 30]) == Fraction(1, 50)  # 1/10 / (1 + 1 + 3)


@pytest.mark.parametrize("seed", range(5))
def test_objective_bound_and_equality(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    m = [int(v) for v in rng.integers(1, 40, size=int(rng.integers(1, 6)))]
    top = Fraction(1, sum(m))
    for q in range(1, 25):
        for p in range(1, 3 * q):
            a = Fraction(p, q)
            got = scale.objective(a, m)
            assert got <= top
            integral = all((a * mi).denominator == 1 for mi in m)
            assert (got == top) == integral


def test_best_breakpoint_hand_values():
    # one bound: alpha = 1/3 makes 3 alpha an integer, so the best is 1/3
    assert scale.best_breakpoint([3], 2) == Fraction(1, 3)
    # m = (2, 3), alpha <= 2/3: the candidates 1/3, 1/2, 2/3 (and every alpha between) reach at
    # most 1/6, below 1 / sum(m) = 1/5
    assert scale.best_breakpoint([2, 3], 2) == Fraction(1, 6)
    # alpha = 1 allowed (limit >= max m): every alpha * m_i is an integer, the bound 1/sum(m)
    assert scale.best_breakpoint([2, 3], 3) == Fraction(1, 5)
    assert scale.best_breakpoint([4, 7, 1], 50) == Fraction(1, 12)


@pytest.mark.parametrize("seed", range(8))
def test_best_breakpoint_beats_a_dense_sweep(seed):
    # every alpha = p / q <= limit / max(m) with q <= 48: none has a larger objective, and the
    # best found is attained (it equals the sweep's maximum when the sweep contains the argmax)
    rng = np.random.Generator(np.random.PCG64(50 + seed))
    m = [int(v) for v in rng.integers(1, 13, size=int(rng.integers(1, 5)))]
    limit = int(rng.integers(2, 30))
    amax = Fraction(limit, max(m))
    best = scale.best_breakpoint(m, limit)
    assert best <= Fraction(1, sum(m))
    sweep_max = Fraction(0)
    for q in range(1, 49):
        for p in range(1, int(amax * q) + 1):
            sweep_max = max(sweep_max, scale.objective(Fraction(p, q), m))
    assert sweep_max <= best
    # the argmax is n / m_i or amax; all of these have denominators <= 12 here, or amax's
    if max(m) <= 48:
        assert sweep_max == best
