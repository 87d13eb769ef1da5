"""CPU oracle for red-green weighted minwise hashing (arXiv 1602.08393).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product library never imports it and it never
imports the product library: the two share no code.

The arithmetic lives in ``wmh_oracle.c`` (plain C, one thread per row range).  This module loads
it through ctypes and adds the exact rational quantities the tests compare against:

* ``jaccard``            -- generalized Jaccard, eq. 1 (exact ``Fraction``).
* ``capped_collision``   -- probability that two rows collide when the step count is capped at H.
  A collision happens at step t < H when the first t-1 draws miss both green regions and draw t
  hits both; every pair that reaches step H collides.  This tends to eq. 1 as H grows
  (Theorem 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwmh_oracle.so")
SOURCE = os.path.join(_HERE, "wmh_oracle.c")
DEFAULT_CAP = 65535

STATUS_NAMES = {0: "ok", 1: "bad argument", 2: "column >= D", 3: "columns not increasing",
                4: "value above bound", 5: "bad row_ptr", 6: "out of memory"}


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc into ``oracle/libwmh_oracle.so``."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-pthread",
           SOURCE, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u16p = ctypes.POINTER(ctypes.c_uint16)
        L.wo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.wo_philox4x32_10.restype = None
        L.wo_bounded_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint, u64p]
        L.wo_bounded_draw.restype = ctypes.c_int
        L.wo_position.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint64, u32p]
        L.wo_position.restype = ctypes.c_uint64
        L.wo_is_green_dense.argtypes = [u32p, u32p, ctypes.c_uint32, ctypes.c_uint64]
        L.wo_is_green_dense.restype = ctypes.c_int
        L.wo_hash_dense_positions.argtypes = [u32p, u32p, ctypes.c_uint32, u64p, ctypes.c_uint32]
        L.wo_hash_dense_positions.restype = ctypes.c_int64
        L.wo_hash_csr.argtypes = [u32p, ctypes.c_uint32, u64p, u32p, u32p, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_uint32, u16p, ctypes.c_int, u64p, u64p]
        L.wo_hash_csr.restype = ctypes.c_int
        L.wo_collisions.argtypes = [u16p, u16p, ctypes.c_uint32]
        L.wo_collisions.restype = ctypes.c_uint32
        L.wo_estimate.argtypes = [u16p, u16p, ctypes.c_uint32]
        L.wo_estimate.restype = ctypes.c_double
        L.wo_collisions_all_pairs.argtypes = [u16p, ctypes.c_uint64, u16p, ctypes.c_uint64,
                                              ctypes.c_uint32, u32p]
        L.wo_collisions_all_pairs.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleError(RuntimeError):
    def __init__(self, status: int, row: int | None = None):
        self.status = status
        self.row = row
        super().__init__(f"oracle status {status} ({STATUS_NAMES.get(status, '?')}), row {row}")


# ---------------------------------------------------------------------------------------------
# Thin wrappers
# ---------------------------------------------------------------------------------------------

def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> tuple[int, int, int, int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().wo_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                           _ptr(out, ctypes.c_uint32))
    return tuple(int(v) for v in out)


def bounded_draw(u: int, n: int, bits: int = 64) -> int | None:
    """Lemire's bounded draw at word width ``bits``; None when the word is rejected."""
    v = ctypes.c_uint64(0)
    ok = lib().wo_bounded_draw(ctypes.c_uint64(u), ctypes.c_uint64(n), bits, ctypes.byref(v))
    return int(v.value) if ok else None


def position(seed: int, j: int, t: int, M: int) -> tuple[int, int]:
    """(position of step t of hash j, Philox blocks used)."""
    used = ctypes.c_uint32(0)
    p = lib().wo_position(ctypes.c_uint64(seed), j, t, ctypes.c_uint64(M), ctypes.byref(used))
    return int(p), int(used.value)


def is_green_dense(m: np.ndarray, x: np.ndarray, p: int) -> int:
    m = np.ascontiguousarray(m, dtype=np.uint32)
    x = np.ascontiguousarray(x, dtype=np.uint32)
    return lib().wo_is_green_dense(_ptr(m, ctypes.c_uint32), _ptr(x, ctypes.c_uint32), len(m),
                                   ctypes.c_uint64(p))


def hash_dense_positions(m: np.ndarray, x: np.ndarray, positions: Sequence[int]) -> int:
    m = np.ascontiguousarray(m, dtype=np.uint32)
    x = np.ascontiguousarray(x, dtype=np.uint32)
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    return int(lib().wo_hash_dense_positions(_ptr(m, ctypes.c_uint32), _ptr(x, ctypes.c_uint32),
                                             len(m), _ptr(pos, ctypes.c_uint64), len(pos)))


def hash_csr(m, row_ptr, col, val, k: int, seed: int = 0, cap: int = 0,
             threads: int | None = None, return_steps: bool = False):
    """Signatures uint16 [N, k] of CSR rows (row_ptr u64 [N+1], col u32, val u32)."""
    m = np.ascontiguousarray(m, dtype=np.uint32)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    val = np.ascontiguousarray(val, dtype=np.uint32)
    n = len(row_ptr) - 1
    sig = np.zeros((n, k), dtype=np.uint16)
    if threads is None:
        threads = os.cpu_count() or 1
    steps = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    nnz = len(col)
    if len(val) != nnz:
        raise ValueError("col and val differ in length")
    col_p = _ptr(col, ctypes.c_uint32) if nnz else ctypes.POINTER(ctypes.c_uint32)()
    val_p = _ptr(val, ctypes.c_uint32) if nnz else ctypes.POINTER(ctypes.c_uint32)()
    st = lib().wo_hash_csr(_ptr(m, ctypes.c_uint32), len(m), _ptr(row_ptr, ctypes.c_uint64),
                           col_p, val_p, n, nnz, k, ctypes.c_uint64(seed), cap,
                           _ptr(sig, ctypes.c_uint16), int(threads), ctypes.byref(steps),
                           ctypes.byref(bad))
    if st != 0:
        raise OracleError(st, int(bad.value))
    return (sig, int(steps.value)) if return_steps else sig


def hash_dense(m, X, k: int, seed: int = 0, cap: int = 0, threads: int = 1):
    """Signatures of the rows of a dense matrix X [N, D] (a convenience over ``hash_csr``)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.uint32))
    rows, cols = np.nonzero(X)
    counts = np.bincount(rows, minlength=X.shape[0])
    row_ptr = np.zeros(X.shape[0] + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(counts)
    return hash_csr(m, row_ptr, cols.astype(np.uint32), X[rows, cols].astype(np.uint32), k,
                    seed=seed, cap=cap, threads=threads)


def collisions(a: np.ndarray, b: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint16)
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return int(lib().wo_collisions(_ptr(a, ctypes.c_uint16), _ptr(b, ctypes.c_uint16), len(a)))


def estimate(a: np.ndarray, b: np.ndarray) -> float:
    a = np.ascontiguousarray(a, dtype=np.uint16)
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return float(lib().wo_estimate(_ptr(a, ctypes.c_uint16), _ptr(b, ctypes.c_uint16), len(a)))


def collisions_all_pairs(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint16)
    B = np.ascontiguousarray(B, dtype=np.uint16)
    out = np.zeros((A.shape[0], B.shape[0]), dtype=np.uint32)
    lib().wo_collisions_all_pairs(_ptr(A, ctypes.c_uint16), A.shape[0], _ptr(B, ctypes.c_uint16),
                                  B.shape[0], A.shape[1], _ptr(out, ctypes.c_uint32))
    return out


# ---------------------------------------------------------------------------------------------
# Exact quantities from the paper's mathematics
# ---------------------------------------------------------------------------------------------

def jaccard(x: Sequence[int], y: Sequence[int]) -> Fraction:
    """Generalized Jaccard, eq. 1, as an exact fraction (0/0 taken as 0)."""
    num = sum(min(int(a), int(b)) for a, b in zip(x, y))
    den = sum(max(int(a), int(b)) for a, b in zip(x, y))
    return Fraction(num, den) if den else Fraction(0)


def capped_collision(x: Sequence[int], y: Sequence[int], M: int, cap: int) -> Fraction:
    """Pr(h(x) == h(y)) for non-empty x, y when the step count is capped at ``cap``.

    Each draw is uniform on {0..M-1}.  Let a = sum(min)/M (green for both) and
    n = 1 - sum(max)/M (green for neither).  A collision at step t < cap needs t-1 draws green
    for neither and then one green for both: a * n^(t-1).  Pairs that reach step ``cap`` both
    get the value ``cap``: probability n^(cap-1).

    The sum over t < cap is geometric: a (1 - n^(cap-1)) / (1 - n).  Exact for cap <= 64; a
    float for larger caps (where the exact fraction would have enormous terms).
    """
    both = sum(min(int(p), int(q)) for p, q in zip(x, y))
    either = sum(max(int(p), int(q)) for p, q in zip(x, y))
    if either == 0:
        raise ValueError("both vectors empty")
    if cap <= 64:
        a = Fraction(both, M)
        n = 1 - Fraction(either, M)
        return a * (1 - n ** (cap - 1)) / (1 - n) + n ** (cap - 1)
    a = both / M
    n = 1.0 - either / M
    tail = n ** (cap - 1)
    return a * (1.0 - tail) / (1.0 - n) + tail
