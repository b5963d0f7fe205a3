"""Pins of the screening-statistic oracle (oracle/screens.py): hand-worked
sequences, brute force over all splits of a short sequence, and the
probabilities' normalisation and a closed form."""
from __future__ import annotations

from math import comb

import numpy as np

from oracle import screens


def test_gap_hand_example():
    lo, hi = 100, 200
    H, M = 150, 5                      # a hit and a miss
    x = np.array([M, H, M, M, H, H] + [M] * 70 + [H, M], dtype=np.uint32)
    # hits at 1, 4, 5, 76: gaps 2, 0, 70 -> bins 2, 0, 3 (last bin >= 3)
    assert screens.gap_counts(x, lo, hi, 4).tolist() == [1, 0, 1, 1]
    # boundaries: lo is a hit, hi is not
    # hits at 0, 1, 3 (200 is outside): gaps 0 and 1
    assert screens.gap_counts(np.array([100, 199, 200, 100], np.uint32), 100, 200, 3).tolist() == [1, 1, 0]


def test_gap_total_is_hits_minus_one():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 2 ** 32, 5000, dtype=np.uint64).astype(np.uint32)
    lo, hi = 1 << 30, 1 << 31
    hits = int(((x >= lo) & (x < hi)).sum())
    assert int(screens.gap_counts(x, lo, hi, 16).sum()) == hits - 1


def test_hwd_hand_example():
    x = np.array([0, 0xFFFF, 0xFFFFFFFF, 0x7FFF], dtype=np.uint32)   # weights 0, 16, 32, 15
    t = screens.hwd_counts(x)
    expect = np.zeros((3, 3), np.uint64)
    expect[0, 1] = expect[1, 2] = expect[2, 1] = 1
    assert np.array_equal(t, expect)
    assert [screens.weight_class(v) for v in (0x3FFF, 0x7FFF, 0x1FFFF, 0x3FFFF)] == [0, 1, 1, 2]


def test_hwd_brute_force_marginals():
    rng = np.random.default_rng(2)
    x = rng.integers(0, 2 ** 32, 3000, dtype=np.uint64).astype(np.uint32)
    t = screens.hwd_counts(x)
    cls = np.array([screens.weight_class(v) for v in x])
    for c in range(3):
        assert int(t[c].sum()) == int((cls[:-1] == c).sum())
        assert int(t[:, c].sum()) == int((cls[1:] == c).sum())


def test_probabilities():
    p = screens.gap_probabilities(0, 1 << 30, 8)      # p = 1/4
    assert abs(p.sum() - 1) < 1e-12
    assert abs(p[0] - 0.25) < 1e-15 and abs(p[-1] - 0.75 ** 7) < 1e-15
    w = screens.weight_class_probabilities()
    assert abs(w.sum() - 1) < 1e-12
    assert abs(w[1] - (comb(32, 15) + comb(32, 16) + comb(32, 17)) / 2 ** 32) < 1e-15
