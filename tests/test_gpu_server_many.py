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


def test_c5_scale_replay_mirrored_streams(torch):
    """Serving at the C5 shape: 16384 resident mexp-11213 streams, a 64 GB
    output pool, requests with log-uniform lengths in [2^8, 2^24] and mixed
    dtype arriving as a Poisson process.  64 mirrored streams (every 256th)
    receive every fourth request; their results are kept and each one is
    compared with the oracle, and the same requests replayed alone (a fresh
    server from the same initial states, no other traffic) give the same
    results.  Every touched stream's final state matches the oracle."""
    print("case server C5 scale, mirrored streams", flush=True)
    sys.stdout.flush()
    cfg = workloads.CONFIGS["C5"]
    params, seeds = workloads.config_inputs("C5")
    n_streams, mexp = params.shape[0], cfg["mexp"]
    N = mexp // 32 + 1
    n_req = 3000
    tr = workloads.request_trace(n_req, 200e3, n_streams, len_log2=cfg["len_log2"],
                                 p_float=cfg["p_float"], master=cfg["master"])
    st = tr["stream"].copy()
    mirrored = np.arange(0, n_streams, 256)
    sel = np.arange(n_req) % 4 == 0
    st[sel] = mirrored[np.arange(int(sel.sum())) % mirrored.size]
    L, dt = tr["length"].astype(np.uint64), tr["dtype"].astype(np.int32)
    arr = (tr["t_arrival"] * 1e9).astype(np.uint64)
    keep_idx = np.flatnonzero(np.isin(st, mirrored))
    offs = np.zeros(n_req, dtype=np.int64)
    offs[keep_idx] = np.concatenate([[0], np.cumsum(L[keep_idx].astype(np.int64))[:-1]])
    total_kept = int(L[keep_idx].sum())
    kept = torch.empty(total_kept, dtype=torch.int32, device="cuda")
    kp = [0] * n_req
    for i in keep_idx:
        kp[int(i)] = kept.data_ptr() + 4 * int(offs[i])

    g = mtgp.Generators(params, seeds)
    srv = mtgp.Server(g, cfg["pool_bytes"], inflight=16, max_batch_items=128,
                      batch_window_ns=50000, workspace_bytes_per_batch=128 << 20)
    try:
        lat, _ = srv.replay(arr, st, L, dt, keep=kp)
        repaired = srv.repaired()
    finally:
        srv.close()
    assert (lat > 0).all()
    assert repaired == 0
    end_states = g.states_host()
    g.close()

    # every kept result against the oracle, per stream in submission order
    host = kept.cpu().numpy().view(np.uint32)
    init = np.stack([oracle.seed(int(seeds[k]), N) for k in range(n_streams)])

    def one_stream(k):
        s = init[k].copy()
        for i in np.flatnonzero(st == k):
            o, s = oracle.generate(params[k], s, int(L[i]), bool(dt[i]))
            got = host[int(offs[i]):int(offs[i]) + int(L[i])]
            assert np.array_equal(got, np.asarray(o).view(np.uint32)), (k, int(i))
        return s

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=16) as ex:
        fins = list(ex.map(one_stream, [int(k) for k in mirrored]))
    for k, s in zip(mirrored, fins):
        assert np.array_equal(end_states[int(k)], s), int(k)

    # every other touched stream's final state
    others = sorted(set(int(k) for k in st) - set(int(k) for k in mirrored))

    def advance(k):
        tot = int(L[st == k].sum())
        _, s = oracle.generate(params[k], init[k], tot, False)
        return s

    with ThreadPoolExecutor(max_workers=16) as ex:
        fins = list(ex.map(advance, others))
    for k, s in zip(others, fins):
        assert np.array_equal(end_states[k], s), k

    # the mirrored streams' requests alone, same initial states
    g2 = mtgp.Generators(params, seeds)
    alone = torch.empty(total_kept, dtype=torch.int32, device="cuda")
    kp2 = [alone.data_ptr() + 4 * int(offs[i]) for i in keep_idx]
    srv2 = mtgp.Server(g2, cfg["pool_bytes"], inflight=16, max_batch_items=128,
                       batch_window_ns=50000, workspace_bytes_per_batch=128 << 20)
    try:
        srv2.replay(arr[keep_idx], st[keep_idx], L[keep_idx], dt[keep_idx], keep=kp2)
    finally:
        srv2.close()
    torch.cuda.synchronize()
    assert torch.equal(alone, kept)
    g2.close()
