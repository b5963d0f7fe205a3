"""Regression anchor: the oracle still reproduces the committed fixture
written by tests/golden/make_golden.py (which calls only the oracle)."""
import os

import numpy as np

import oracle
from paper_1501_07701_amd import workloads

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _parse(path):
    blocks, cur = {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        if key == "seed":
            cur = blocks.setdefault(int(vals[0]), {})
        else:
            cur[key] = np.array([int(v, 16) for v in vals], dtype=np.uint32)
    return blocks


def test_c1_stream0_fixture():
    blocks = _parse(os.path.join(HERE, "c1_stream0.txt"))
    params, _ = workloads.config_inputs("C1")
    for seed_value, b in blocks.items():
        st = oracle.seed(seed_value, 351)
        u, st1 = oracle.generate(params[0], st, 4096)
        fl, _ = oracle.generate(params[0], st, 4096, as_float=True)
        assert np.array_equal(u[:64], b["u32[0:64]"])
        assert np.array_equal(u[-64:], b["u32[4032:4096]"])
        assert np.array_equal(fl.view(np.uint32)[:64], b["f32bits[0:64]"])
        assert np.array_equal(st1[:16], b["state_after_4096[0:16]"])
