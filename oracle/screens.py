"""Screening statistics, plain CPU definitions -- TEST INFRASTRUCTURE ONLY.

Same import rule as the rest of ``oracle/``: only tests, ``smoke()`` and
``bench.py``'s cpu_baseline leg use it.  Each function is the textbook
definition written out word by word, with no blocking or reordering.
"""
from __future__ import annotations

import numpy as np


def gap_counts(x: np.ndarray, lo: int, hi: int, bins: int) -> np.ndarray:
    """Gap test (Knuth, TAOCP Vol. 2, Sec. 3.3.2 D), counting the gaps
    between consecutive hits: word j is a hit when lo <= x[j] < hi; for
    consecutive hits j < j' the gap j' - j - 1 is counted in bin
    min(gap, bins - 1).  The run before the first hit is not counted."""
    counts = np.zeros(bins, dtype=np.uint64)
    prev = -1
    for j, v in enumerate(np.asarray(x, dtype=np.uint32).tolist()):
        if lo <= v < hi:
            if prev >= 0:
                counts[min(j - prev - 1, bins - 1)] += 1
            prev = j
    return counts


def weight_class(v: int) -> int:
    """Hamming-weight class of a 32-bit word: popcount <= 14, 15..17, >= 18."""
    w = bin(int(v)).count("1")
    return 0 if w <= 14 else (1 if w <= 17 else 2)


def hwd_counts(x: np.ndarray) -> np.ndarray:
    """Hamming-weight dependency table: (class of word j, class of word j+1)
    for every j, a 3x3 table of counts."""
    t = np.zeros((3, 3), dtype=np.uint64)
    xs = np.asarray(x, dtype=np.uint32).tolist()
    for a, b in zip(xs[:-1], xs[1:]):
        t[weight_class(a), weight_class(b)] += 1
    return t


def gap_probabilities(lo: int, hi: int, bins: int) -> np.ndarray:
    """Probability of each gap bin for independent uniform 32-bit words:
    p (1-p)^r for r < bins-1, (1-p)^(bins-1) for the last bin."""
    p = (hi - lo) / 2.0 ** 32
    r = np.arange(bins - 1)
    return np.concatenate([p * (1 - p) ** r, [(1 - p) ** (bins - 1)]])


def weight_class_probabilities() -> np.ndarray:
    """Class probabilities of a uniform 32-bit word (binomial(32, 1/2))."""
    from math import comb
    w = np.array([comb(32, k) for k in range(33)], dtype=np.float64) / 2.0 ** 32
    return np.array([w[:15].sum(), w[15:18].sum(), w[18:].sum()])
