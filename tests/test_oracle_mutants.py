"""The oracle's pins must catch plausible mistakes.

Each case compiles a copy of the oracle source with one planted mistake (a
dropped term, a wrong shift direction, an off-by-one tap, a wrong constant)
and checks that the GF(2)-matrix model or the numpy seeding pin rejects it.
Mistakes are planted on the CPU only, in temporary copies.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from gf2_model import Model
from oracle_helpers import random_row, random_state

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "mtgp_oracle.c")

MUTANTS = [
    ("X ^= X << p->sh1;", "X ^= X >> p->sh1;"),
    ("X ^= X << p->sh1;", ""),
    ("uint32_t Y = X ^ (tap >> p->sh2);", "uint32_t Y = X ^ (tap << p->sh2);"),
    ("uint32_t X = (oldest & p->mask) ^ next;", "uint32_t X = oldest ^ next;"),
    ("uint32_t X = (oldest & p->mask) ^ next;", "uint32_t X = (oldest & p->mask);"),
    ("return Y ^ p->rec[Y & 0xFu];", "return Y ^ p->rec[(Y >> 28) & 0xFu];"),
    ("return Y ^ p->rec[Y & 0xFu];", "return X ^ p->rec[Y & 0xFu];"),
    ("x[n] = recursion(p, x[j], x[j + 1], x[j + pos]);",
     "x[n] = recursion(p, x[j], x[j + 1], x[j + pos - 1]);"),
    ("x[n] = recursion(p, x[j], x[j + 1], x[j + pos]);",
     "x[n] = recursion(p, x[j + 1], x[j], x[j + pos]);"),
    ("uint32_t t = temper_index(x[j + pos - 1]);", "uint32_t t = temper_index(x[j + pos]);"),
    ("H ^= H >> 8;", ""),
    ("H ^= H >> 16;", "H ^= H >> 15;"),
    ("out[j] = x[n] ^ p->tmp[t];", "out[j] = x[n] ^ p->tmp[t ^ 1];"),
    ("uint32_t bits = (x[n] >> 9) ^ p->flt[t];", "uint32_t bits = (x[n] >> 8) ^ p->flt[t];"),
    ("uint32_t bits = (x[n] >> 9) ^ p->flt[t];", "uint32_t bits = (x[n] >> 9) ^ p->tmp[t];"),
    ("x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + (uint32_t)i;",
     "x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + (uint32_t)(i - 1);"),
    ("x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + (uint32_t)i;",
     "x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 29)) + (uint32_t)i;"),
    ("memcpy(state, x + count, (size_t)N * sizeof(uint32_t));",
     "memcpy(state, x + count + 1, (size_t)(N - 1) * sizeof(uint32_t));"),
]


def _build_mutant(d, idx, old, new):
    src = open(SRC).read()
    assert old in src, old
    mutated = src.replace(old, new, 1)
    path = os.path.join(d, "m%d.c" % idx)
    so = os.path.join(d, "m%d.so" % idx)
    with open(path, "w") as f:
        f.write(mutated)
    subprocess.run(["gcc", "-O1", "-w", "-shared", "-fPIC", "-o", so, path], check=True)
    lib = ctypes.CDLL(so)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_generate.argtypes = [u32p, u32p, ctypes.c_uint64, ctypes.c_int, u32p]
    lib.oracle_seed.argtypes = [ctypes.c_uint32, ctypes.c_int, u32p]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _pins_pass(lib) -> bool:
    """Run the seeding pin and the matrix-model pin on the mutant."""
    for seed in (1, 5489):
        x = np.zeros(351, dtype=np.uint32)
        lib.oracle_seed(seed, 351, _p(x))
        if not np.array_equal(x, np.random.RandomState(seed).get_state()[1][:351].astype(np.uint32)):
            return False
    rng = np.random.default_rng(99)
    for mexp in (89, 3217):
        row, (rb, tb, fb) = random_row(rng, mexp, independent_float=True)
        n_words = mexp // 32 + 1
        state = random_state(rng, n_words)
        count = 3 * n_words + 50
        mu, mm, ms = Model(n_words, int(row[1]), int(row[2]), int(row[3]), int(row[4]),
                           rb, tb, fb).run(state, count)
        for as_float in (0, 1):
            st = state.copy()
            out = np.zeros(count, dtype=np.uint32)
            lib.oracle_generate(_p(row), _p(st), count, as_float, _p(out))
            if not np.array_equal(st, ms):
                return False
            if as_float == 0 and not np.array_equal(out, mu):
                return False
            if as_float == 1:
                f = out.view(np.float32).astype(np.float64) * (1 << 23)
                if not np.array_equal(f, mm.astype(np.float64)):
                    return False
    return True


def test_unmutated_source_passes():
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(d, 999, "#include <stdint.h>", "#include <stdint.h>")
        assert _pins_pass(lib)


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_planted_mistake_is_caught(idx):
    old, new = MUTANTS[idx]
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(d, idx, old, new)
        assert not _pins_pass(lib), "planted mistake survived: %r -> %r" % (old, new)
