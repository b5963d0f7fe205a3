"""An independent GF(2)-matrix formulation of the MTGP32 output map.

Used only to pin the oracle.  Instead of bitwise word operations it builds
32x32 matrices over GF(2) from what each operation *is*: the period mask is a
diagonal matrix, a logical shift is a shifted identity, a GF(2)-linear
16-entry table is the 32x4 matrix of its four basis words applied to the low
four bits, and XOR is matrix addition.  Words are column vectors of bits
(bit i = (w >> i) & 1).  The recurrence is then iterated one word at a time
with matrix-vector products mod 2.

It only models linear tables (tables that are spans of four basis words),
which is the structure of MTGP's precomputed tables (paper Sec. 3.1).
"""
from __future__ import annotations

import numpy as np

W = 32


def word_to_bits(w: int) -> np.ndarray:
    return np.array([(int(w) >> i) & 1 for i in range(W)], dtype=np.uint8)


def bits_to_word(v: np.ndarray) -> int:
    return int(sum(int(v[i] & 1) << i for i in range(W)))


def identity() -> np.ndarray:
    return np.eye(W, dtype=np.uint8)


def shift_left(s: int) -> np.ndarray:
    """(x << s): output bit i takes input bit i - s."""
    m = np.zeros((W, W), dtype=np.uint8)
    for i in range(s, W):
        m[i, i - s] = 1
    return m


def shift_right(s: int) -> np.ndarray:
    """(x >> s): output bit i takes input bit i + s."""
    m = np.zeros((W, W), dtype=np.uint8)
    for i in range(0, W - s):
        m[i, i + s] = 1
    return m


def diagonal(mask: int) -> np.ndarray:
    return np.diag(word_to_bits(mask)).astype(np.uint8)


def basis_matrix(basis, width: int = W) -> np.ndarray:
    """Column b (b < 4) holds the bits of basis[b]; other columns are zero,
    so M @ y picks up basis[b] for each set bit b among y's low four bits."""
    m = np.zeros((W, W), dtype=np.uint8)
    for b in range(4):
        m[:, b] = word_to_bits(int(basis[b]) & ((1 << width) - 1))
    return m


def mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return (a.astype(np.int64) @ b.astype(np.int64) % 2).astype(np.uint8)


def add(*ms) -> np.ndarray:
    out = np.zeros_like(ms[0])
    for m in ms:
        out ^= m
    return out


class Model:
    """Matrix model of one parameter set given by its basis words."""

    def __init__(self, n_words: int, pos: int, sh1: int, sh2: int, mask: int,
                 rec_basis, tmp_basis, flt_basis=None):
        self.N, self.pos = n_words, pos
        I = identity()
        left = add(I, shift_left(sh1))                 # X -> X ^ (X << sh1)
        self.A_old = mul(left, diagonal(mask))         # oldest word, masked
        self.A_next = left                             # the adjacent word
        self.A_tap = shift_right(sh2)                  # pos-tap >> sh2
        self.G = add(I, basis_matrix(rec_basis))       # Y -> Y ^ rec[Y & 15]
        fold = mul(add(I, shift_right(8)), add(I, shift_right(16)))
        self.E_u32 = mul(basis_matrix(tmp_basis), fold)
        self.E_f32 = None
        if flt_basis is not None:
            self.E_f32 = mul(basis_matrix(flt_basis, 23), fold)
        self.S9 = shift_right(9)

    def run(self, state_words, count: int):
        """Returns (u32 outputs, f32 mantissas (or None), final state words)."""
        N, pos = self.N, self.pos
        x = [word_to_bits(w) for w in state_words]
        u32, man = [], []
        for j in range(count):
            y = add(mul(self.A_old, x[j][:, None])[:, 0],
                    mul(self.A_next, x[j + 1][:, None])[:, 0],
                    mul(self.A_tap, x[j + pos][:, None])[:, 0])
            xn = mul(self.G, y[:, None])[:, 0]
            x.append(xn)
            h = x[j + pos - 1]
            u32.append(bits_to_word(add(xn, mul(self.E_u32, h[:, None])[:, 0])))
            if self.E_f32 is not None:
                man.append(bits_to_word(add(mul(self.S9, xn[:, None])[:, 0],
                                            mul(self.E_f32, h[:, None])[:, 0])))
        final = [bits_to_word(v) for v in x[count:count + N]]
        return (np.array(u32, dtype=np.uint32),
                None if self.E_f32 is None else np.array(man, dtype=np.uint32),
                np.array(final, dtype=np.uint32))
