"""CPU oracle of (K, L) banding over signatures.  TEST INFRASTRUCTURE ONLY (see
``oracle/__init__``).

Band b of a signature is its values at hash ids [b*K, (b+1)*K).  A database row is a candidate
for a query when some band is equal value for value; candidates are reported once each, in
increasing row order.  Plain dictionaries from band tuples to rows: no hashing of the values.
"""
from __future__ import annotations

import numpy as np


def candidates(db: np.ndarray, queries: np.ndarray, K: int, L: int) -> list[list[int]]:
    db = np.asarray(db, dtype=np.uint16)
    queries = np.asarray(queries, dtype=np.uint16)
    if K < 1 or L < 1 or K * L > db.shape[1]:
        raise ValueError("need K, L >= 1 and K * L <= k")
    tables = []
    for b in range(L):
        table: dict[tuple, list[int]] = {}
        for r in range(db.shape[0]):
            table.setdefault(tuple(db[r, b * K:(b + 1) * K].tolist()), []).append(r)
        tables.append(table)
    out = []
    for q in range(queries.shape[0]):
        found: set[int] = set()
        for b in range(L):
            found.update(tables[b].get(tuple(queries[q, b * K:(b + 1) * K].tolist()), []))
        out.append(sorted(found))
    return out


def candidate_probability(J: float, K: int, L: int) -> float:
    """Probability that a pair whose hashes agree independently with probability J shares a
    band."""
    return 1.0 - (1.0 - J ** K) ** L
