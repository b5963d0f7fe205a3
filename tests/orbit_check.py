"""Test-side check, with the oracle, of whether a polynomial annihilates the
word sequence of a given state (used to pick states that a stream's
jump-ahead polynomial does not cover)."""
from __future__ import annotations

import numpy as np

import oracle


def raw_words(row, state, n_words, length):
    """x_0 .. x_{length-1}: the state followed by the words the recurrence
    appends, read off the oracle's state after every N outputs."""
    out = [np.array(state, dtype=np.uint32)]
    st = np.array(state, dtype=np.uint32)
    have = n_words
    while have < length:
        _, st = oracle.generate(row, st, n_words, False)
        out.append(st.copy())
        have += n_words
    return np.concatenate(out)[:length]


def annihilates(row, coeff_words, degree, state, checks=64):
    """True when y_t = XOR_{i: p_i = 1} x_{t+i} vanishes for t = 1..checks,
    p given as packed coefficient words (bit i of word i/32)."""
    n_words = int(row[0]) // 32 + 1
    x = raw_words(row, state, n_words, 1 + degree + checks + 1)
    bits = np.unpackbits(np.asarray(coeff_words, dtype=np.uint32).view(np.uint8),
                         bitorder="little")[: degree + 1]
    taps = np.flatnonzero(bits)
    for t in range(1, checks + 1):
        y = np.bitwise_xor.reduce(x[t + taps])
        if y != 0:
            return False
    return True
