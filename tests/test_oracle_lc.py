"""Linear-complexity pins (the MT family's outputs obey a GF(2) linear
recurrence, paper Sec. 3.1 and Sec. 4.2).

Berlekamp-Massey itself is first pinned against brute force and against
sequences whose complexity is known; then every output bit of the oracle's
streams must have linear complexity <= mexp, with the connection polynomial
predicting held-out bits exactly.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from oracle_helpers import random_row


def _brute_force_lc(s):
    """Smallest L such that some length-L LFSR generates s (exhaustive)."""
    n = len(s)
    for L in range(0, n + 1):
        for taps in itertools.product((0, 1), repeat=L):
            if all(s[k] == (sum(taps[i] * s[k - 1 - i] for i in range(L)) & 1)
                   for k in range(L, n)):
                return L
    return n


def _predicts(bits, conn, start, stop):
    L = len(conn) - 1
    c = conn[1:].astype(np.int64)
    for k in range(start, stop):
        if L and (int(np.dot(c, bits[k - 1::-1][:L].astype(np.int64))) & 1) != bits[k]:
            return False
        if not L and bits[k] != 0:
            return False
    return True


def test_bm_matches_brute_force_on_short_sequences():
    rng = np.random.default_rng(0)
    for n in range(1, 13):
        for _ in range(12):
            s = rng.integers(0, 2, n).astype(np.uint8)
            L, conn = oracle.berlekamp_massey(s)
            assert L == _brute_force_lc(list(s)), (n, s)
            assert _predicts(s, conn, L, n)


@pytest.mark.parametrize("taps,deg", [((31, 3), 31), ((7, 1), 7), ((89, 38), 89)])
def test_bm_recovers_primitive_lfsr(taps, deg):
    # s_k = s_{k-a} ^ s_{k-b}: x^a + x^b + 1 primitive -> LC = a
    a, b = taps
    rng = np.random.default_rng(deg)
    s = list(rng.integers(0, 2, a))
    while not any(s):
        s = list(rng.integers(0, 2, a))
    for k in range(a, 4 * a + 64):
        s.append(s[k - a] ^ s[k - b])
    s = np.array(s, dtype=np.uint8)
    L, conn = oracle.berlekamp_massey(s)
    assert L == deg
    expect = np.zeros(deg + 1, dtype=np.uint8)
    expect[0] = expect[a] = expect[b] = 1
    assert np.array_equal(conn, expect)


def test_bm_random_sequence_is_about_half_length():
    rng = np.random.default_rng(3)
    s = rng.integers(0, 2, 5000).astype(np.uint8)
    L, _ = oracle.berlekamp_massey(s)
    assert abs(L - 2500) <= 20


def _bit_sequences(row, seed_value, n_total):
    n_words = int(row[0]) // 32 + 1
    u, _ = oracle.generate(row, oracle.seed(seed_value, n_words), n_total)
    return u


@pytest.mark.parametrize("mexp,bits", [(3217, range(32)), (11213, (0, 13, 31)),
                                       (23209, (5, 31)), (44497, (0,))])
def test_linear_complexity_at_most_mexp(mexp, bits):
    rng = np.random.default_rng(mexp + 77)
    row, _ = random_row(rng, mexp)
    K = 1024
    window = 2 * mexp + 64
    u = _bit_sequences(row, 1, window + K)
    for b in bits:
        s = ((u >> np.uint32(b)) & 1).astype(np.uint8)
        L, conn = oracle.berlekamp_massey(s[:window])
        assert L <= mexp, (b, L)
        assert _predicts(s, conn, window, window + K), b


def test_nonlinear_table_exceeds_mexp():
    """Negative control: a non-linear recursion table destroys the bound."""
    rng = np.random.default_rng(2)
    row, _ = random_row(rng, 3217)
    row[5:21] = rng.integers(0, 2**32, 16, dtype=np.uint64).astype(np.uint32)
    u = _bit_sequences(row, 1, 2 * 3217 + 2000)
    L, _ = oracle.berlekamp_massey(((u >> np.uint32(7)) & 1).astype(np.uint8))
    assert L > 3217
