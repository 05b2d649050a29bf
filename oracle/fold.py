"""CPU oracle for the float map-reduce of Section 4.2. TEST INFRASTRUCTURE ONLY.

Only the tests and the benchmark may import this module. Section 4.2 compares map-reduce
implementations on two sums over i = 1..n, each term mapped from its index and the terms
added:

  kind 0: the sum of sqrt(i)
  kind 1: the sum of (-1)^(i+1) / i   (the alternating harmonic series, whose limit is ln 2)

Each term is the IEEE double nearest to its exact value (numpy's sqrt and division are
correctly rounded), and the terms are added with ``math.fsum``, which returns the double
nearest to their exact sum. So the oracle is the sum of the rounded terms, rounded once.

Pins (tests/test_oracle_fold.py): exact rational / 50-digit decimal sums for small n; the
alternating series' error term (the limit ln 2 with the Euler-transform tail); the
Euler-Maclaurin expansion of the square-root sum (zeta(-1/2) constant); S(n) - S(n-1) = term n.
"""
from __future__ import annotations

import math

import numpy as np

SQRT, ALT_HARMONIC = 0, 1
_CHUNK = 1 << 20


def terms(kind: int, i0: int, i1: int) -> np.ndarray:
    """Terms i0..i1-1 (1-based indices) as doubles."""
    i = np.arange(i0, i1, dtype=np.float64)
    if kind == SQRT:
        return np.sqrt(i)
    if kind == ALT_HARMONIC:
        sign = np.where((np.arange(i0, i1) & 1) == 1, 1.0, -1.0)
        return sign / i
    raise ValueError(f"unknown kind {kind}")


def fold_sum(kind: int, n: int) -> float:
    """The double nearest to the exact sum of the rounded terms 1..n (0.0 for n = 0)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    parts = []
    for a in range(1, n + 1, _CHUNK):
        parts.append(terms(kind, a, min(n + 1, a + _CHUNK)))
    if not parts:
        return 0.0
    return math.fsum(np.concatenate(parts))


def abs_sum(kind: int, n: int) -> float:
    """Sum of the terms' magnitudes (for error bounds)."""
    if n <= 0:
        return 0.0
    total = 0.0
    for a in range(1, n + 1, _CHUNK):
        total += float(np.abs(terms(kind, a, min(n + 1, a + _CHUNK))).sum())
    return total
