"""Seeded synthetic inputs for MTGP32 bulk generation.

This module is the only code that feeds both the GPU library and the CPU
oracle.  It draws parameter sets, seeds, request lengths, dtypes and arrival
times from a counter-based splitmix64 (Steele, Lea & Flood, 2014) and holds
none of the generator's arithmetic: the recurrence, tempering and seeding
live separately in the GPU library and in the oracle.

The paper's own parameter sets came from MTGP's Dynamic Creator and were
screened with BigCrush (Sec. 3.1, Sec. 4.1); none are available here, so the
workloads use random parameter sets of the same shape: pos uniform in
[1, N-2], shifts uniform in [0, 31], and the three 16-entry tables built as
GF(2) spans of four random basis words (``tbl[i]`` = XOR of the basis words
selected by the bits of ``i``), which is what MTGP's precomputed "fast"
tables are (Sec. 3.1).  The float table is either derived from the uint32
tempering table (``0x3F800000 | tmp >> 9``) or spans four independent 23-bit
words.  Such streams are correct MTGP-form sequences but carry no period or
statistical-quality guarantee.
"""
from __future__ import annotations

import math

import numpy as np

PARAM_WORDS = 53           # mexp, pos, sh1, sh2, mask, rec[16], tmp[16], flt[16]
GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
SLOTS_PER_STREAM = 16      # splitmix counters reserved per stream

SUPPORTED_MEXP = (3217, 11213, 23209, 44497)


def splitmix64(counters: np.ndarray, master: int) -> np.ndarray:
    """Output ``i`` of splitmix64 seeded with ``master`` is
    mix(master + (i+1)*GOLDEN); evaluated here for an array of counters."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(master & M64) + (c + np.uint64(1)) * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _uniform_int(z: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Integer in [lo, hi] from the top 32 bits of z (multiply-shift; bias
    below (hi-lo+1)/2^32, negligible for these spans)."""
    span = np.uint64(hi - lo + 1)
    return (np.uint64(lo) + (((z >> np.uint64(32)) * span) >> np.uint64(32))).astype(np.uint32)


def _unit_float(z: np.ndarray) -> np.ndarray:
    """Double in [0, 1) from the top 53 bits."""
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def state_words(mexp: int) -> int:
    return mexp // 32 + 1


def _span_table(basis: np.ndarray) -> np.ndarray:
    """(n, 4) basis words -> (n, 16) table, entry i = XOR of basis[b] for
    every set bit b of i."""
    n = basis.shape[0]
    tbl = np.zeros((n, 16), dtype=np.uint32)
    for i in range(16):
        acc = np.zeros(n, dtype=np.uint32)
        for b in range(4):
            if (i >> b) & 1:
                acc ^= basis[:, b]
        tbl[:, i] = acc
    return tbl


def make_params(mexp: int, n_streams: int, master: int,
                float_family: str = "derived", first_stream: int = 0) -> np.ndarray:
    """Random MTGP32 parameter sets, one row of ``uint32[53]`` per stream.

    Draw slots per stream k (counter = 16*k + slot): 0 pos, 1 sh1, 2 sh2,
    3-6 recursion basis, 7-10 tempering basis, 11-14 float basis."""
    if mexp % 32 == 0 or mexp < 65:
        raise ValueError("mexp must be >= 65 and not a multiple of 32")
    n_words = state_words(mexp)
    r = 32 * n_words - mexp
    mask = (0xFFFFFFFF << r) & 0xFFFFFFFF
    k = np.arange(first_stream, first_stream + n_streams, dtype=np.uint64)
    base = k * np.uint64(SLOTS_PER_STREAM)

    def slot(s):
        return splitmix64(base + np.uint64(s), master)

    rows = np.zeros((n_streams, PARAM_WORDS), dtype=np.uint32)
    rows[:, 0] = mexp
    rows[:, 1] = _uniform_int(slot(0), 1, n_words - 2)
    rows[:, 2] = _uniform_int(slot(1), 0, 31)
    rows[:, 3] = _uniform_int(slot(2), 0, 31)
    rows[:, 4] = mask
    rec_basis = np.stack([(slot(3 + b) >> np.uint64(32)).astype(np.uint32) for b in range(4)], 1)
    tmp_basis = np.stack([(slot(7 + b) >> np.uint64(32)).astype(np.uint32) for b in range(4)], 1)
    rows[:, 5:21] = _span_table(rec_basis)
    tmp = _span_table(tmp_basis)
    rows[:, 21:37] = tmp
    if float_family == "derived":
        rows[:, 37:53] = np.uint32(0x3F800000) | (tmp >> np.uint32(9))
    elif float_family == "independent":
        flt_basis = np.stack([(slot(11 + b) >> np.uint64(41)).astype(np.uint32) for b in range(4)], 1)
        rows[:, 37:53] = np.uint32(0x3F800000) | _span_table(flt_basis)
    else:
        raise ValueError(float_family)
    return rows


def make_seeds(n_streams: int, first_stream: int = 0) -> np.ndarray:
    """Seed status of stream k is k+1 (seed 0 is tested separately)."""
    return np.arange(first_stream + 1, first_stream + n_streams + 1, dtype=np.uint32)


def log_uniform_lengths(n: int, lo_log2: float, hi_log2: float, master: int,
                        stream_offset: int = 0) -> np.ndarray:
    """L = floor(2^U), U uniform in [lo_log2, hi_log2]."""
    z = splitmix64(np.arange(stream_offset, stream_offset + n, dtype=np.uint64)
                   * np.uint64(SLOTS_PER_STREAM) + np.uint64(15), master)
    u = lo_log2 + (hi_log2 - lo_log2) * _unit_float(z)
    return np.floor(np.exp2(u)).astype(np.uint64)


def bernoulli_dtypes(n: int, master: int, p_float: float = 0.5,
                     stream_offset: int = 0) -> np.ndarray:
    """0 = uint32, 1 = float32; float with probability p_float."""
    z = splitmix64(np.arange(stream_offset, stream_offset + n, dtype=np.uint64)
                   * np.uint64(SLOTS_PER_STREAM) + np.uint64(14), master ^ 0xD7)
    return (_unit_float(z) < p_float).astype(np.int32)


# Workloads of the benchmark suite.  Master seeds are fixed per workload.
CONFIGS = {
    "C1": dict(name="mtgp11213_4x2^20_u32", mexp=11213, streams=4,
               count=1 << 20, dtypes=("u32",), master=0xC0FFEE01),
    "C2": dict(name="mtgp11213_128x2^24_u32+f32", mexp=11213, streams=128,
               count=1 << 24, dtypes=("u32", "f32"), master=0xC0FFEE02),
    "C3": dict(name="mtgp23209_4096x2^20_u32_batched", mexp=23209,
               streams=4096, count=1 << 20, dtypes=("u32",), master=0xC0FFEE03),
    "C4": dict(name="mtgp44497_1024_loguniform2^10-2^24_mixed", mexp=44497,
               streams=1024, len_log2=(10, 24), p_float=0.5, master=0xC0FFEE04),
    "C5": dict(name="mtgp11213_serve_16384_resident", mexp=11213,
               streams=16384, len_log2=(8, 24), p_float=0.5,
               pool_bytes=64 * 10**9, master=0xC0FFEE05),
    # shapes of the paper's experiments: 10,000 statuses of period 2^3217
    # sharing seed status 0 (Sec. 4.1), and 100 statuses x 100 random seeds
    # (Random Spacing, Sec. 5.1); random parameter sets stand in for the
    # Dynamic Creator's
    "P1": dict(name="mtgp3217_10000_statuses_seed0_2^20", mexp=3217, streams=10000,
               count=1 << 20, dtypes=("u32",), master=0xC0FFEE06),
    "P2": dict(name="mtgp3217_100_statuses_x_100_seeds_2^20", mexp=3217, streams=10000,
               param_sets=100, seeds=100, count=1 << 20, dtypes=("u32",),
               master=0xC0FFEE07),
}


def config_inputs(cfg: str, n_streams: int | None = None):
    """(params, seeds) for a workload, optionally only its first n streams."""
    c = CONFIGS[cfg]
    n = c["streams"] if n_streams is None else n_streams
    if cfg == "P1":      # every status seeded with 0
        return make_params(c["mexp"], n, c["master"]), np.zeros(n, dtype=np.uint32)
    if cfg == "P2":      # stream a*n_seeds + b: parameter set a, seed b
        n_par, n_seed = c["param_sets"], c["seeds"]
        par = np.repeat(make_params(c["mexp"], n_par, c["master"]), n_seed, axis=0)
        seeds = (splitmix64(np.arange(n_seed, dtype=np.uint64), c["master"] ^ 0x5EED)
                 >> np.uint64(32)).astype(np.uint32)
        return par[:n], np.tile(seeds, n_par)[:n]
    return make_params(c["mexp"], n, c["master"]), make_seeds(n)


def uneven_batch(cfg: str = "C4", n_streams: int | None = None):
    """Per-stream (length, dtype) of an uneven batch."""
    c = CONFIGS[cfg]
    n = c["streams"] if n_streams is None else n_streams
    lo, hi = c["len_log2"]
    return (log_uniform_lengths(n, lo, hi, c["master"]),
            bernoulli_dtypes(n, c["master"], c["p_float"]))


def request_trace(n_requests: int, rate_per_s: float, n_streams: int,
                  len_log2=(8, 24), p_float: float = 0.5, master: int = 0xC0FFEE05):
    """Poisson arrivals: returns dict of arrays t_arrival (s), stream, length,
    dtype.  Stream uniform over [0, n_streams), length log-uniform."""
    i = np.arange(n_requests, dtype=np.uint64) * np.uint64(4)
    u_gap = _unit_float(splitmix64(i + np.uint64(0), master ^ 0xA11))
    gaps = -np.log1p(-u_gap) / rate_per_s
    z_stream = splitmix64(i + np.uint64(1), master ^ 0xA11)
    stream = ((z_stream >> np.uint64(32)) * np.uint64(n_streams) >> np.uint64(32)).astype(np.int32)
    lo, hi = len_log2
    u_len = _unit_float(splitmix64(i + np.uint64(2), master ^ 0xA11))
    length = np.floor(np.exp2(lo + (hi - lo) * u_len)).astype(np.uint64)
    dtype = (_unit_float(splitmix64(i + np.uint64(3), master ^ 0xA11)) < p_float).astype(np.int32)
    return dict(t_arrival=np.cumsum(gaps), stream=stream, length=length, dtype=dtype)


def expected_log_uniform_mean(lo_log2: float, hi_log2: float) -> float:
    """E[2^U] for U uniform in [lo, hi] (floor ignored)."""
    return (2.0 ** hi_log2 - 2.0 ** lo_log2) / ((hi_log2 - lo_log2) * math.log(2.0))
