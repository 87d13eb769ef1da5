"""CPU oracle of the fixed-point scaling step (Sec. 4, Practical Issues).  TEST INFRASTRUCTURE
ONLY (see ``oracle/__init__``).

* ``quantize``: x_q = floor(alpha * x + 1/2) with both operations IEEE double rounded one at a
  time (numpy does not fuse them), negative results to 0, capped at the integer bound
  ceil(alpha * m) of the value's column.
* ``objective``: the paper's alpha * sum(x) / sum(ceil(alpha * m_i)) without the common factor
  sum(x), in exact rationals.
* ``best_breakpoint``: brute force over every alpha = n / m_i <= alpha_max (integer bounds),
  where the objective peaks.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def quantize(x: np.ndarray, col: np.ndarray, m_q: np.ndarray, alpha: float):
    prod = np.multiply(np.float64(alpha), np.asarray(x, dtype=np.float32).astype(np.float64))
    v = np.floor(np.maximum(np.add(prod, 0.5), 0.0))
    cap = np.asarray(m_q, dtype=np.float64)[np.asarray(col, dtype=np.int64)]
    clipped = int((v > cap).sum())
    return np.minimum(v, cap).astype(np.uint32), clipped


def objective(alpha, m) -> Fraction:
    a = Fraction(alpha)
    total = sum((a * Fraction(int(mi))).__ceil__() for mi in m)
    return a / total


def best_breakpoint(m, limit: int) -> Fraction:
    top = max(int(v) for v in m)
    amax = Fraction(limit, top)
    best = objective(amax, m)
    for mi in m:
        mi = int(mi)
        if mi == 0:
            continue
        n = 1
        while Fraction(n, mi) <= amax:
            best = max(best, objective(Fraction(n, mi), m))
            n += 1
    return best
