"""Plain CPU oracle for MTGP32 bulk generation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it; the two share no code (only the seeded input generators in
``paper_1501_07701_amd.workloads`` feed both sides).

The arithmetic lives in ``mtgp_oracle.c`` (plain C, one word at a time over a
full history, the definition written out); this module only compiles it with
gcc and marshals numpy arrays through ctypes.

Parameter rows are ``uint32[53]``: mexp, pos, sh1, sh2, mask, rec[16],
tmp[16], flt[16] -- a generator's parameterised status (paper Sec. 3.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mtgp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
PARAM_WORDS = 53

_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vector intrinsics)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
         "-o", tmp, _SRC],
        check=True,
    )
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            lib.oracle_state_words.argtypes = [ctypes.c_uint32]
            lib.oracle_state_words.restype = ctypes.c_int
            lib.oracle_mask.argtypes = [ctypes.c_uint32]
            lib.oracle_mask.restype = ctypes.c_uint32
            lib.oracle_check_params.argtypes = [u32p]
            lib.oracle_check_params.restype = ctypes.c_int
            lib.oracle_seed.argtypes = [ctypes.c_uint32, ctypes.c_int, u32p]
            lib.oracle_seed.restype = None
            lib.oracle_generate.argtypes = [u32p, u32p, ctypes.c_uint64,
                                            ctypes.c_int, u32p]
            lib.oracle_generate.restype = ctypes.c_int
            lib.oracle_berlekamp_massey.argtypes = [
                ctypes.POINTER(ctypes.c_uint8), ctypes.c_int,
                ctypes.POINTER(ctypes.c_uint8)]
            lib.oracle_berlekamp_massey.restype = ctypes.c_int
            _lib = lib
    return _lib


def _u32p(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def state_words(mexp: int) -> int:
    """N = floor(mexp/32) + 1, or -1 for an unusable exponent."""
    return _load().oracle_state_words(mexp)


def mask(mexp: int) -> int:
    return int(_load().oracle_mask(mexp))


def check_params(row: np.ndarray) -> int:
    row = np.ascontiguousarray(row, dtype=np.uint32)
    assert row.shape == (PARAM_WORDS,)
    return _load().oracle_check_params(_u32p(row))


def seed(seed_value: int, n_words: int) -> np.ndarray:
    """Seed status -> initial N-word state (Mersenne Twister initialisation)."""
    x = np.zeros(n_words, dtype=np.uint32)
    _load().oracle_seed(seed_value & 0xFFFFFFFF, n_words, _u32p(x))
    return x


def generate(row: np.ndarray, state: np.ndarray, count: int,
             as_float: bool = False):
    """Advance one stream by ``count`` outputs.

    Returns ``(out, new_state)``; ``out`` is uint32, or float32 when
    ``as_float``.  ``state`` is not modified."""
    row = np.ascontiguousarray(row, dtype=np.uint32)
    st = np.array(state, dtype=np.uint32, copy=True)
    out = np.empty(count, dtype=np.uint32)
    rc = _load().oracle_generate(_u32p(row), _u32p(st), count,
                                 1 if as_float else 0, _u32p(out))
    if rc != 0:
        raise ValueError("oracle_generate rejected the parameter set")
    return (out.view(np.float32) if as_float else out), st


def generate_many(params: np.ndarray, states: np.ndarray, counts,
                  as_float=False, threads: int = 1):
    """Run ``generate`` for every stream (row k of params/states), streams
    spread over a thread pool (ctypes releases the GIL during the C call).
    ``counts`` and ``as_float`` may be scalars or per-stream sequences.
    Returns (list of outputs, new states array)."""
    n = params.shape[0]
    counts = [int(counts)] * n if np.isscalar(counts) else [int(c) for c in counts]
    flts = [bool(as_float)] * n if np.isscalar(as_float) else [bool(f) for f in as_float]
    new_states = np.array(states, dtype=np.uint32, copy=True)
    outs = [None] * n

    def one(k):
        o, st = generate(params[k], states[k], counts[k], flts[k])
        outs[k] = o
        new_states[k] = st

    if threads <= 1:
        for k in range(n):
            one(k)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(n)))
    return outs, new_states


def berlekamp_massey(bits: np.ndarray):
    """Linear complexity and connection polynomial of a GF(2) sequence."""
    b = np.ascontiguousarray(bits, dtype=np.uint8) & 1
    n = int(b.shape[0])
    conn = np.zeros(n + 1, dtype=np.uint8)
    L = _load().oracle_berlekamp_massey(
        b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n,
        conn.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if L < 0:
        raise MemoryError("oracle_berlekamp_massey failed")
    return L, conn[: L + 1].copy()
