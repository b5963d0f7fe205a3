"""Batch submission (mtgp_submit_many): the same results, in submission
order per stream, as one mtgp_submit per request; all-or-none validation."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1501_07701_amd import mtgp, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    mtgp.lib()
    return t


def test_submit_many_matches_oracle(torch):
    print("case server submit_many", flush=True)
    sys.stdout.flush()
    mexp = 11213
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 16, 0x3C)
    seeds = np.arange(1, 17, dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    srv = mtgp.Server(g, 256 << 20, inflight=4, workspace_bytes_per_batch=8 << 20)
    rng = np.random.default_rng(3)
    st = rng.integers(0, 6, 60).astype(np.int32)
    ct = np.floor(2.0 ** rng.uniform(4, 17, 60)).astype(np.uint64)
    dt = rng.integers(0, 2, 60).astype(np.int32)
    try:
        with pytest.raises(mtgp.MTGPError) as e:
            srv.submit_many([0, 99], [10, 10], [0, 0])         # one bad request: none queued
        assert e.value.code == mtgp.EINVAL
        tk = srv.submit_many(st, ct, dt)
        got = []
        for j in range(60):
            srv.wait(int(tk[j]), 60 * 10**9)
            got.append(srv.result(int(tk[j]), int(ct[j]), int(dt[j])).cpu().numpy().view(np.uint32))
            srv.release(int(tk[j]))
    finally:
        srv.close()
        g.close()
    states = {}
    for j in range(60):
        s = int(st[j])
        if s not in states:
            states[s] = oracle.seed(int(seeds[s]), N)
        o, states[s] = oracle.generate(p[s], states[s], int(ct[j]), bool(dt[j]))
        assert np.array_equal(got[j], np.asarray(o).view(np.uint32)), j


def test_replay_advances_streams_like_the_oracle(torch):
    """A replayed trace completes every request and leaves each stream's
    state exactly where the oracle puts it after that stream's requests."""
    print("case server replay", flush=True)
    mexp = 3217
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 32, 0x4D)
    seeds = np.arange(1, 33, dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    srv = mtgp.Server(g, 256 << 20, inflight=4, workspace_bytes_per_batch=8 << 20)
    rng = np.random.default_rng(5)
    n = 300
    st = rng.integers(0, 32, n).astype(np.int32)
    ct = np.floor(2.0 ** rng.uniform(4, 16, n)).astype(np.uint64)
    dt = rng.integers(0, 2, n).astype(np.int32)
    arr = np.cumsum(rng.exponential(20e3, n)).astype(np.uint64)   # ns
    try:
        lat, stg = srv.replay(arr, st, ct, dt)
    finally:
        srv.close()
    assert (lat > 0).all() and (stg[:, 2] > 0).all()
    states = np.stack([oracle.seed(int(s), N) for s in seeds])
    for k in range(32):
        tot = int(ct[st == k].sum())
        if tot:
            _, states[k] = oracle.generate(p[k], states[k], tot, False)
    assert np.array_equal(g.states_host(), states)
    g.close()
