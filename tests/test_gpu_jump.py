"""GPU parity of jump-ahead splitting: a request cut into segments whose start
states are jumped must give exactly the outputs and final state of the
unsplit stream (and of the CPU oracle), and every segment's end-state check
must pass."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from orbit_check import annihilates
from paper_1501_07701_amd import mtgp, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    mtgp.lib()
    return t


def _host(t):
    return t.cpu().numpy().view(np.uint32)


class _Tune:
    """Temporarily set the jump target for an exponent."""

    def __init__(self, mexp, target):
        self.mexp, self.target = mexp, target

    def __enter__(self):
        self.t0 = mtgp.get_tuning(self.mexp)
        t = self.t0.as_tuple()
        mtgp.set_tuning(self.mexp, t[0], t[1], t[2], self.target)

    def __exit__(self, *exc):
        mtgp.set_tuning(self.mexp, *self.t0.as_tuple())


def _params(mexp, master):
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 6, master)
    p[0, 1] = N - 2          # W = 2
    p[1, 1] = 1              # W = N - 1
    p[2, 1] = N - 33         # W = 33
    return p


@pytest.mark.parametrize("mexp,count", [(3217, 60000), (11213, 150000), (23209, 200000),
                                        (44497, 300000)])
def test_split_batch_matches_oracle(torch, mexp, count):
    _say("case split mexp=%d count=%d" % (mexp, count))
    p = _params(mexp, 0x5EED + mexp)
    seeds = np.arange(1, 7, dtype=np.uint32)
    N = mexp // 32 + 1
    counts = [count, count // 2 + 7, count, 3 * count // 4 + 1, 1000, count]
    dts = [0, 1, 0, 1, 0, 1]
    with _Tune(mexp, 256):
        g = mtgp.Generators(p, seeds)
        outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in counts]
        items = [(k, dts[k], counts[k], outs[k]) for k in range(6)]
        ws_full = mtgp.batch_workspace_query(g.d_params, items)
        assert ws_full > mtgp.batch_workspace_bytes(6)      # it does split
        ws = g.workspace(items)
        for rep in range(2):                                 # continuation across calls
            g.batch(items, ws)
            got = [_host(o).copy() for o in outs]
            assert mtgp.batch_errors(ws) == 0
            if rep == 0:
                states = np.stack([oracle.seed(int(s), N) for s in seeds])
            for k in range(6):
                o, states[k] = oracle.generate(p[k], states[k], counts[k], bool(dts[k]))
                assert np.array_equal(got[k], np.asarray(o).view(np.uint32)), (rep, k)
        assert np.array_equal(g.states_host(), states)
        g.close()


def test_split_equals_unsplit_and_small_workspace(torch):
    """Same batch three ways: no splitting, full splitting, and splitting
    limited by a workspace that is too small for the full plan."""
    _say("case split vs unsplit")
    mexp, count = 11213, 200000
    p = workloads.make_params(mexp, 16, 0xAB)
    seeds = np.arange(1, 17, dtype=np.uint32)
    results = []
    for target, ws_kind in ((0, "min"), (128, "full"), (128, "half")):
        with _Tune(mexp, target):
            g = mtgp.Generators(p, seeds)
            out = torch.empty(16 * count, dtype=torch.int32, device="cuda")
            items = [(k, k & 1, count, out.data_ptr() + 4 * k * count) for k in range(16)]
            full = mtgp.batch_workspace_query(g.d_params, items)
            nbytes = {"min": mtgp.batch_workspace_bytes(16), "full": full,
                      "half": max(mtgp.batch_workspace_bytes(16), full // 3)}[ws_kind]
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            mtgp.generate_batch(g.d_params, g.d_states, g.stride, items, ws)
            assert mtgp.batch_errors(ws) == 0
            results.append((_host(out).copy(), g.states_host()))
            g.close()
    for r in results[1:]:
        assert np.array_equal(r[0], results[0][0])
        assert np.array_equal(r[1], results[0][1])


def test_split_after_reseed_and_graph_replays(torch):
    """Bench shape: re-seed, split batch replayed from the cached graph."""
    _say("case reseed + replays")
    mexp, count = 3217, 40000
    p = workloads.make_params(mexp, 32, 0xCD)
    seeds = np.arange(1, 33, dtype=np.uint32)
    exp, _ = oracle.generate_many(p, np.stack([oracle.seed(int(s), 101) for s in seeds]),
                                  count, False, threads=8)
    with _Tune(mexp, 32):
        g = mtgp.Generators(p, seeds)
        out = torch.empty(32 * count, dtype=torch.int32, device="cuda")
        items = [(k, 0, count, out.data_ptr() + 4 * k * count) for k in range(32)]
        ws = g.workspace(items)
        for rep in range(3):
            g.reseed()
            mtgp.generate_batch(g.d_params, g.d_states, g.stride, items, ws)
            h = _host(out).reshape(32, count)
            for k in range(32):
                assert np.array_equal(h[k], exp[k]), (rep, k)
        assert mtgp.batch_errors(ws) == 0
        g.close()


def test_phase_timing_stamps(torch):
    """Phase timestamps: present only while enabled, ordered, and the batch
    results do not change with the stamp kernels in the graph."""
    _say("case phase timing")
    mexp, count = 11213, 150000
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 4, 0x7A)
    seeds = np.arange(1, 5, dtype=np.uint32)
    with _Tune(mexp, 256):
        g = mtgp.Generators(p, seeds)
        outs = [torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(4)]
        items = [(k, 0, count, outs[k]) for k in range(4)]
        ws = g.workspace(items)
        g.batch(items, ws)
        with pytest.raises(mtgp.MTGPError):
            mtgp.batch_phase_times(ws)                 # never stamped
        first = [_host(o).copy() for o in outs]
        mtgp.set_phase_timing(True)
        try:
            g.reseed()
            g.batch(items, ws)
            us = mtgp.batch_phase_times(ws)
        finally:
            mtgp.set_phase_timing(False)
        assert all(x >= 0 for x in us) and us[1] > 0 and us[2] > 0, us
        assert mtgp.batch_errors(ws) == 0
        states = np.stack([oracle.seed(int(s), N) for s in seeds])
        for k in range(4):
            o, _ = oracle.generate(p[k], states[k], count, False)
            assert np.array_equal(_host(outs[k]), np.asarray(o).view(np.uint32)), k
            assert np.array_equal(first[k], _host(outs[k])), k
        g.close()


def _foreign_states(p, n_words, rng):
    """States a stream could be restored to: exported from the same
    parameter sets run from other seeds, and uniformly random full states."""
    k = p.shape[0]
    other = np.stack([oracle.seed(1000 + i, n_words) for i in range(k)])
    moved, other = oracle.generate_many(p, other, 5000, False)
    rand = rng.integers(0, 2**32, (k, n_words), dtype=np.uint64).astype(np.uint32)
    return np.where((np.arange(k) % 2 == 0)[:, None], other, rand)


@pytest.mark.parametrize("mexp,count", [(3217, 60000), (11213, 150000)])
def test_load_params_import_then_split(torch, mexp, count):
    """Checkpoint-restore flow: parameters uploaded without seeds, states
    imported from elsewhere (other seeds' streams, random full states);
    split batches from there are exact, with no segment-check repairs (the
    polynomials are built from the imported states)."""
    _say("case load_params + import + split mexp=%d" % mexp)
    N = mexp // 32 + 1
    p = _params(mexp, 0x1A + mexp)
    n = p.shape[0]
    st = _foreign_states(p, N, np.random.default_rng(mexp))
    d_params = torch.empty(n * mtgp.DEVICE_PARAM_BYTES, dtype=torch.uint8, device="cuda")
    d_states = torch.empty(n * N, dtype=torch.int32, device="cuda")
    mtgp.load_params(p, d_params)
    mtgp.state_import(d_params, d_states, N, st)
    counts = [count, count // 2 + 7, count, 3 * count // 4 + 1, 1000, count]
    dts = [0, 1, 0, 1, 0, 1]
    with _Tune(mexp, 256):
        outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in counts]
        items = [(k, dts[k], counts[k], outs[k]) for k in range(n)]
        ws = torch.empty(mtgp.batch_workspace_query(d_params, items), dtype=torch.uint8,
                         device="cuda")
        states = st.copy()
        for rep in range(2):
            mtgp.generate_batch(d_params, d_states, N, items, ws)
            got = [_host(o).copy() for o in outs]
            assert mtgp.batch_errors(ws) == 0, rep
            for k in range(n):
                o, states[k] = oracle.generate(p[k], states[k], counts[k], bool(dts[k]))
                assert np.array_equal(got[k], np.asarray(o).view(np.uint32)), (rep, k)
        assert np.array_equal(mtgp.state_export(d_params, d_states, N, n, N), states)
        # the data is really split: a minimum workspace cannot hold the plan
        assert ws.numel() > mtgp.batch_workspace_bytes(n)
    mtgp.release_params(d_params)


def test_states_written_behind_the_library_are_repaired(torch):
    """States written straight into device memory (no import) can lie
    outside the orbit a stream's polynomial annihilates: the segment checks
    fail, the device regenerates those requests in order, the outputs stay
    exact, the repairs are reported, and the next call rebuilds the
    polynomials from the current states (no repairs)."""
    _say("case repair after states written behind the library")
    mexp, count = 3217, 60000
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 16, 0x4E9A)
    seeds = np.zeros(16, dtype=np.uint32)          # seed status 0 (paper, Sec. 5.1)
    with _Tune(mexp, 256):
        g = mtgp.Generators(p, seeds)
        deg, co = mtgp.stream_polynomials(g.d_params, 16, mexp)
        # random states whose word sequence the stream's polynomial (built
        # from the seed-0 orbit) does not annihilate, checked with the oracle
        rng = np.random.default_rng(7)
        st = g.states_host()
        low = []
        for k in range(16):
            if len(low) == 4 or deg[k] <= 0:
                continue
            for _ in range(4):
                cand = rng.integers(0, 2**32, N, dtype=np.uint64).astype(np.uint32)
                if not annihilates(p[k], co[k], int(deg[k]), cand):
                    st[k] = cand
                    low.append(k)
                    break
        assert len(low) >= 2, deg                  # seed-0 orbits of random sets
        # behind the library's back: a device copy, not mtgp_state_import
        g.d_states.copy_(torch.from_numpy(st.view(np.int32).reshape(-1)).to("cuda"))
        outs = [torch.empty(count, dtype=torch.int32, device="cuda") for _ in low]
        items = [(k, i & 1, count, outs[i]) for i, k in enumerate(low)]
        ws = g.workspace(items)
        states = st.copy()
        repairs = []
        for rep in range(2):
            g.batch(items, ws)
            got = [_host(o).copy() for o in outs]
            repairs.append(mtgp.batch_errors(ws))
            for i, k in enumerate(low):
                o, states[k] = oracle.generate(p[k], states[k], count, bool(i & 1))
                assert np.array_equal(got[i], np.asarray(o).view(np.uint32)), (rep, k)
        assert np.array_equal(g.states_host(), states)
        assert repairs[0] >= 1, repairs            # the checks caught the wrong orbits
        assert repairs[1] == 0, repairs            # rebuilt from the current states
        g.close()


@pytest.mark.parametrize("overlap", ["0", "default"])
def test_whole_requests_beside_the_jumps(torch, overlap):
    """A batch with long (split) and short (whole) requests: by default the
    whole requests run on a second stream beside the prefix and jump launch
    (MTGP_OVERLAP=0 runs the phases one after another).  Both give the
    oracle's outputs and final states, over two calls in a row."""
    import os
    _say("case whole requests beside the jumps, MTGP_OVERLAP=%s" % overlap)
    mexp = 11213
    N = mexp // 32 + 1
    n_long, n_short = 6, 26
    p = workloads.make_params(mexp, n_long + n_short, 0x0E71)
    p[0, 1] = N - 2                                   # a W = 2 stream among the long ones
    seeds = np.arange(1, n_long + n_short + 1, dtype=np.uint32)
    counts = [200000 + 1111 * k for k in range(n_long)] + [3000 + 97 * k for k in range(n_short)]
    dts = [k % 2 for k in range(n_long + n_short)]
    old = os.environ.get("MTGP_OVERLAP")
    if overlap == "0":
        os.environ["MTGP_OVERLAP"] = "0"
    else:
        os.environ.pop("MTGP_OVERLAP", None)
    try:
        with _Tune(mexp, 256):
            g = mtgp.Generators(p, seeds)
            outs = [torch.empty(c, dtype=torch.int32, device="cuda") for c in counts]
            items = [(k, dts[k], counts[k], outs[k]) for k in range(len(counts))]
            assert mtgp.batch_workspace_query(g.d_params, items) > \
                mtgp.batch_workspace_bytes(len(items))    # the long ones split
            ws = g.workspace(items)
            states = [oracle.seed(int(seeds[k]), N) for k in range(len(counts))]
            for rep in range(2):
                g.batch(items, ws)
                got = [_host(o).copy() for o in outs]
                assert mtgp.batch_errors(ws) == 0
                for k in range(len(counts)):
                    o, states[k] = oracle.generate(p[k], states[k], counts[k], bool(dts[k]))
                    assert np.array_equal(got[k], np.asarray(o).view(np.uint32)), (rep, k)
            assert np.array_equal(g.states_host(), np.array(states))
            g.close()
    finally:
        if old is None:
            os.environ.pop("MTGP_OVERLAP", None)
        else:
            os.environ["MTGP_OVERLAP"] = old
