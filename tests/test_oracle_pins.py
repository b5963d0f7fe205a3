"""Pins of the CPU oracle against things other than itself.

* Seeding: numpy's legacy MT19937 initialisation and C++'s
  std::mersenne_twister_engine use the same initialisation recurrence.
* Recurrence + tempering: an independent GF(2)-matrix formulation
  (tests/gf2_model.py), iterated word by word, over many parameter sets,
  including the edge cases pos = 1, pos = N-2, sh1 = 0, sh2 = 0.
* Structural invariants: GF(2)-linearity of the output map, the zero state,
  mask semantics, continuation, the float identities.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from gf2_model import Model
from oracle_helpers import mantissa, random_row, random_state, row_from_basis


# ---------------------------------------------------------------- seeding --

@pytest.mark.parametrize("seed", [0, 1, 5489, 0xDEADBEEF, 0xFFFFFFFF])
@pytest.mark.parametrize("n_words", [3, 101, 351, 624])
def test_seed_matches_numpy_mt19937_init(seed, n_words):
    ref = np.random.RandomState(seed).get_state()[1][:n_words].astype(np.uint32)
    assert np.array_equal(oracle.seed(seed, n_words), ref)


_MT_SRC = r"""
#include <iostream>
#include <random>
#include <cstdint>
int main(int argc, char** argv) {
  uint32_t seed = (uint32_t)std::stoul(argv[1]);
  std::mersenne_twister_engine<uint32_t, 32, NW, 1, 19, 0x9908b0dfu, 11,
      0xffffffffu, 7, 0x9d2c5680u, 15, 0xefc60000u, 18, 1812433253u> e(seed);
  std::cout << e << std::endl;
}
"""


@pytest.mark.parametrize("n_words", [101, 351, 726, 1391])
def test_seed_matches_std_mersenne_twister_engine(n_words):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "mt.cpp")
        exe = os.path.join(d, "mt")
        with open(src, "w") as f:
            f.write(_MT_SRC)
        subprocess.run([gxx, "-O1", "-std=c++17", "-DNW=%d" % n_words, src, "-o", exe],
                       check=True)
        for seed in (0, 1, 4357, 2**32 - 1):
            txt = subprocess.run([exe, str(seed)], check=True, capture_output=True,
                                 text=True).stdout.split()
            # operator<< prints x_0..x_{n-1} then the position index.
            words = np.array([int(t) for t in txt[:n_words]], dtype=np.uint64).astype(np.uint32)
            assert np.array_equal(oracle.seed(seed, n_words), words)


# ------------------------------------------------ GF(2) matrix formulation --

def _model_from(row, bases):
    rb, tb, fb = bases
    mexp, pos, sh1, sh2, mask = (int(v) for v in row[:5])
    if fb is None:
        # derived float table: flt = 0x3F800000 | tmp >> 9, i.e. basis tb >> 9
        fb = [int(b) >> 9 for b in tb]
    return Model(mexp // 32 + 1, pos, sh1, sh2, mask, rb, tb, fb)


CASES = [
    # (mexp, pos, sh1, sh2, independent float table)
    (65, 1, 1, 1, True),          # N = 3: the smallest state
    (89, 1, 13, 7, False),
    (127, 2, 5, 31, True),        # pos = N-2
    (127, 1, 0, 0, True),         # sh1 = 0 and sh2 = 0
    (3217, None, None, None, True),
    (3217, 1, 31, 17, False),     # pos = 1
    (3217, 99, 2, 0, True),       # pos = N-2
    (11213, None, None, None, False),
    (11213, 349, None, None, True),
    (23209, None, None, None, True),
    (44497, None, None, None, True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_oracle_matches_gf2_matrix_model(case):
    mexp, pos, sh1, sh2, indep = CASES[case]
    rng = np.random.default_rng(1000 + case)
    row, bases = random_row(rng, mexp, pos, sh1, sh2, independent_float=indep)
    n_words = mexp // 32 + 1
    state = random_state(rng, n_words)
    count = 5000 if n_words < 400 else 1800   # always several state lengths deep
    model = _model_from(row, bases)
    mu, mm, mstate = model.run(state, count)
    ou, ostate = oracle.generate(row, state, count, as_float=False)
    of, _ = oracle.generate(row, state, count, as_float=True)
    assert np.array_equal(ou, mu)
    assert np.array_equal(ostate, mstate)
    assert np.array_equal(mantissa(of), mm)


# --------------------------------------------------------------- invariants --

@pytest.mark.parametrize("mexp", [3217, 11213, 44497])
def test_output_map_is_gf2_linear(mexp):
    rng = np.random.default_rng(mexp)
    row, _ = random_row(rng, mexp)
    n_words = mexp // 32 + 1
    s1, s2 = random_state(rng, n_words), random_state(rng, n_words)
    count = 3 * n_words + 17
    u1, t1 = oracle.generate(row, s1, count)
    u2, t2 = oracle.generate(row, s2, count)
    u12, t12 = oracle.generate(row, s1 ^ s2, count)
    assert np.array_equal(u12, u1 ^ u2)
    assert np.array_equal(t12, t1 ^ t2)
    f1, _ = oracle.generate(row, s1, count, True)
    f2, _ = oracle.generate(row, s2, count, True)
    f12, _ = oracle.generate(row, s1 ^ s2, count, True)
    assert np.array_equal(mantissa(f12), mantissa(f1) ^ mantissa(f2))


def test_zero_state_gives_zero_output():
    rng = np.random.default_rng(7)
    row, _ = random_row(rng, 11213)
    z = np.zeros(351, dtype=np.uint32)
    u, st = oracle.generate(row, z, 4000)
    f, _ = oracle.generate(row, z, 4000, True)
    assert not u.any() and not st.any()
    assert np.all(f == 0.0)


@pytest.mark.parametrize("pos", [1, 2, 77, 349])
def test_mask_semantics(pos):
    """The low r bits of the oldest word never enter the recurrence; they only
    reach output 0 through the helper word when pos = 1."""
    mexp, n_words = 11213, 351
    r = 32 * n_words - mexp
    rng = np.random.default_rng(pos)
    row, _ = random_row(rng, mexp, pos=pos)
    s = random_state(rng, n_words)
    s_flip = s.copy()
    s_flip[0] ^= np.uint32((1 << r) - 1)
    a, sa = oracle.generate(row, s, 2000)
    b, sb = oracle.generate(row, s_flip, 2000)
    assert np.array_equal(a[1:], b[1:])
    assert np.array_equal(sa, sb)
    if pos >= 2:
        assert a[0] == b[0]


@pytest.mark.parametrize("mexp", [3217, 23209])
def test_continuation(mexp):
    rng = np.random.default_rng(mexp + 1)
    row, _ = random_row(rng, mexp)
    n_words = mexp // 32 + 1
    w = n_words - int(row[1])
    s = oracle.seed(12345, n_words)
    total = 3 * n_words + 100
    full, fs = oracle.generate(row, s, total)
    for l1 in (0, 1, w - 1, w, w + 1, n_words, 2 * n_words + 3):
        a, sa = oracle.generate(row, s, l1)
        b, sb = oracle.generate(row, sa, total - l1)
        assert np.array_equal(np.concatenate([a, b]), full)
        assert np.array_equal(sb, fs)


def test_float_identities():
    rng = np.random.default_rng(11)
    # derived float table ties f32 to u32 exactly
    row, _ = random_row(rng, 11213, independent_float=False)
    s = oracle.seed(3, 351)
    u, _ = oracle.generate(row, s, 20000)
    f, _ = oracle.generate(row, s, 20000, True)
    plus_one = (f + np.float32(1.0)).view(np.uint32)
    assert np.array_equal(plus_one, np.uint32(0x3F800000) | (u >> np.uint32(9)))
    # independent float table: values are k * 2^-23 in [0, 1)
    row2, _ = random_row(rng, 11213, independent_float=True)
    f2, _ = oracle.generate(row2, s, 20000, True)
    assert np.all(f2 >= 0.0) and np.all(f2 < 1.0)
    m = mantissa(f2)
    assert m.max() < (1 << 23)


def test_nonlinear_tables_are_accepted():
    """Any 16-entry table is a well-formed definition; only the invariants
    need linear tables.  Nonlinear tables must break linearity (negative
    control showing the linearity test has teeth)."""
    rng = np.random.default_rng(5)
    row, _ = random_row(rng, 3217)
    row[5:21] = rng.integers(0, 2**32, 16, dtype=np.uint64).astype(np.uint32)
    s1, s2 = random_state(rng, 101), random_state(rng, 101)
    u1, _ = oracle.generate(row, s1, 1000)
    u2, _ = oracle.generate(row, s2, 1000)
    u12, _ = oracle.generate(row, s1 ^ s2, 1000)
    assert not np.array_equal(u12, u1 ^ u2)


def test_param_validation():
    rng = np.random.default_rng(9)
    row, _ = random_row(rng, 11213)
    assert oracle.check_params(row) == 0
    bad = row.copy(); bad[0] = 11200
    assert oracle.check_params(bad) == -1          # mexp multiple of 32
    bad = row.copy(); bad[4] ^= 1 << 31
    assert oracle.check_params(bad) == -2          # mask
    bad = row.copy(); bad[1] = 0
    assert oracle.check_params(bad) == -3
    bad = row.copy(); bad[1] = 350
    assert oracle.check_params(bad) == -3          # pos > N-2
    bad = row.copy(); bad[2] = 32
    assert oracle.check_params(bad) == -4
    bad = row.copy(); bad[3] = 40
    assert oracle.check_params(bad) == -5
    bad = row.copy(); bad[40] = 0x40000000
    assert oracle.check_params(bad) == -6          # float table exponent
    assert oracle.state_words(11213) == 351
    assert oracle.mask(11213) == 0xFFF80000
    assert oracle.mask(23209) == 0xFF800000
    assert oracle.mask(44497) == 0xFFFF8000
    assert oracle.mask(3217) == 0xFFFF8000
