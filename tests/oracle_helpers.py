"""Test-side construction of parameter rows from basis words (input building
only; no generator arithmetic)."""
from __future__ import annotations

import numpy as np

PARAM_WORDS = 53


def span(basis):
    out = []
    for i in range(16):
        acc = 0
        for b in range(4):
            if (i >> b) & 1:
                acc ^= int(basis[b])
        out.append(acc)
    return out


def row_from_basis(mexp, pos, sh1, sh2, rec_basis, tmp_basis, flt_basis=None,
                   mask=None):
    n_words = mexp // 32 + 1
    if mask is None:
        mask = (0xFFFFFFFF << (32 * n_words - mexp)) & 0xFFFFFFFF
    rec = span(rec_basis)
    tmp = span(tmp_basis)
    if flt_basis is None:
        flt = [0x3F800000 | (t >> 9) for t in tmp]
    else:
        flt = [0x3F800000 | v for v in span([b & 0x7FFFFF for b in flt_basis])]
    return np.array([mexp, pos, sh1, sh2, mask] + rec + tmp + flt, dtype=np.uint32)


def random_row(rng, mexp, pos=None, sh1=None, sh2=None, independent_float=True):
    n_words = mexp // 32 + 1
    pos = int(rng.integers(1, n_words - 1)) if pos is None else pos
    sh1 = int(rng.integers(0, 32)) if sh1 is None else sh1
    sh2 = int(rng.integers(0, 32)) if sh2 is None else sh2
    rb = [int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)]
    tb = [int(v) for v in rng.integers(0, 2**32, 4, dtype=np.uint64)]
    fb = [int(v) for v in rng.integers(0, 2**23, 4, dtype=np.uint64)] if independent_float else None
    return row_from_basis(mexp, pos, sh1, sh2, rb, tb, fb), (rb, tb, fb)


def random_state(rng, n_words):
    return rng.integers(0, 2**32, n_words, dtype=np.uint64).astype(np.uint32)


def mantissa(f32: np.ndarray) -> np.ndarray:
    """Exact 23-bit integer m with f = m * 2^-23 (f in [0, 1))."""
    m = np.asarray(f32, dtype=np.float64) * float(1 << 23)
    mi = m.astype(np.uint32)
    assert np.all(mi.astype(np.float64) == m), "f32 output is not a multiple of 2^-23"
    return mi
