"""The jump-ahead planner's GF(2)[x] arithmetic (host C++ in the library)
against plain Python big-integer polynomial arithmetic, and its
Berlekamp-Massey against the oracle's."""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1501_07701_amd", "csrc")


@pytest.fixture(scope="module")
def shim():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "poly_shim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-mpclmul", "-shared", "-fPIC", "-I", CSRC,
                    os.path.join(ROOT, "tests", "shims", "poly_shim.cpp"),
                    os.path.join(CSRC, "mtgp_poly.cpp"), "-o", so], check=True)
    return ctypes.CDLL(so)


def to_words(x: int):
    n = max(1, (x.bit_length() + 63) // 64)
    return (ctypes.c_ulonglong * n)(*[(x >> (64 * i)) & ((1 << 64) - 1) for i in range(n)]), n


def from_words(buf, n):
    return sum(int(buf[i]) << (64 * i) for i in range(n))


def pmul(a, b):
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def pmod(a, p):
    dp = p.bit_length() - 1
    while a and a.bit_length() - 1 >= dp:
        a ^= p << (a.bit_length() - 1 - dp)
    return a


def ppowx(e, p):
    r, base = 1, pmod(2, p)
    while e:
        if e & 1:
            r = pmod(pmul(r, base), p)
        base = pmod(pmul(base, base), p)
        e >>= 1
    return r


def _call(fn, *args, cap=4096):
    o = (ctypes.c_ulonglong * cap)()
    n = fn(*args, o, cap)
    assert n >= 0
    return from_words(o, n)


@pytest.mark.parametrize("deg", [1, 5, 63, 64, 65, 200, 3217, 11213, 44497])
def test_mulmod_and_powx(shim, deg):
    rng = np.random.default_rng(deg)
    p = (1 << deg) | int(rng.integers(0, 2**62)) | 1
    if deg > 64:
        p |= int.from_bytes(rng.bytes((deg + 7) // 8), "little") & ((1 << deg) - 1)
    a = int.from_bytes(rng.bytes(deg // 4 + 8), "little")
    b = int.from_bytes(rng.bytes(deg // 4 + 8), "little")
    pw, pn = to_words(p)
    aw, an = to_words(a)
    bw, bn = to_words(b)
    got = _call(shim.shim_mulmod, aw, an, bw, bn, pw, pn)
    assert got == pmod(pmul(pmod(a, p), pmod(b, p)), p)
    for e in (0, 1, deg - 1, deg, deg + 1, 2 * deg + 3, 12345, (1 << 24) - 1):
        assert _call(shim.shim_powx, ctypes.c_ulonglong(e), pw, pn) == ppowx(e, p), e


def test_lcm(shim):
    f1, f2, f3 = 0b111, 0b1011, 0b10011          # x^2+x+1, x^3+x+1, x^4+x+1
    a, b = pmul(f1, f2), pmul(f2, f3)
    aw, an = to_words(a)
    bw, bn = to_words(b)
    assert _call(shim.shim_lcm, aw, an, bw, bn) == pmul(pmul(f1, f2), f3)


@pytest.mark.parametrize("n", [10, 300, 5000])
def test_bm_agrees_with_oracle(shim, n):
    rng = np.random.default_rng(n)
    for kind in ("random", "lfsr"):
        if kind == "random":
            s = rng.integers(0, 2, n).astype(np.uint8)
        else:
            a, b = 89, 38
            s = list(rng.integers(0, 2, a))
            while len(s) < n:
                s.append(s[-a] ^ s[-b])
            s = np.array(s[:n], dtype=np.uint8)
        L_ref, conn = oracle.berlekamp_massey(s)
        o = (ctypes.c_ulonglong * (n // 64 + 4))()
        L = ctypes.c_int()
        nw = shim.shim_bm(s.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), n, o,
                          n // 64 + 4, ctypes.byref(L))
        assert L.value == L_ref
        ann = from_words(o, nw)
        # annihilator is the reciprocal of the connection polynomial
        expect = sum(int(conn[L_ref - j]) << j for j in range(L_ref + 1))
        assert ann == expect
        # and it annihilates the sequence
        for t in range(0, n - L_ref):
            acc = 0
            for j in range(L_ref + 1):
                if (ann >> j) & 1:
                    acc ^= int(s[t + j])
            assert acc == 0
            if t > 200:
                break
