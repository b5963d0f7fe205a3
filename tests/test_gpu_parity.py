"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Small cases span several steps, buffer compactions and ragged tails, for
every supported mexp and every compiled launch tuning; the full-size
workloads (128 x 2^24 through the benchmarked batch path, 4096 x 2^20,
1024 streams of log-uniform length) are checked on every stream.
Tolerance: none.  uint32 outputs, float32 bit patterns and final states must
be identical.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
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
    mtgp.lib()  # fail loudly if the HIP library is missing
    return t


def _host(t):
    return t.cpu().numpy().view(np.uint32)


def _oracle_run(params, seeds, counts, as_float):
    """Run the oracle per stream from its seed over successive calls.
    counts: list of per-call counts; as_float: per-call flags.
    Returns (list of per-call outputs as uint32 views [k][call], final states)."""
    n = params.shape[0]
    N = int(params[0, 0]) // 32 + 1
    outs = [[] for _ in range(n)]
    states = np.stack([oracle.seed(int(s), N) for s in seeds])
    for c, f in zip(counts, as_float):
        res, states = oracle.generate_many(params, states, c, f, threads=8)
        for k in range(n):
            outs[k].append(np.asarray(res[k]).view(np.uint32))
    return outs, states


def _edge_params(mexp, master):
    """Random sets plus the degenerate corners: W = 2, W = N-1, sh1 = 0,
    sh2 = 0, both shifts 31."""
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 8, master)
    p[0, 1] = N - 2          # pos = N-2  -> W = 2
    p[1, 1] = 1              # pos = 1    -> W = N-1
    p[2, 2] = 0              # sh1 = 0
    p[3, 3] = 0              # sh2 = 0
    p[4, 2], p[4, 3] = 31, 31
    p[5, 1] = N - 3          # W = 3
    p[6, 1] = max(1, N - 65)  # W = 65 (one past a wave)
    return p


@pytest.mark.parametrize("mexp", workloads.SUPPORTED_MEXP)
def test_plain_ragged_calls_all_mexp(torch, mexp):
    _say("case plain_ragged mexp=%d" % mexp)
    p = _edge_params(mexp, 0xABC0 + mexp)
    seeds = np.array([0, 1, 2, 3, 5489, 0xFFFFFFFF, 77, 123456], dtype=np.uint32)
    N = mexp // 32 + 1
    calls = [1, 2, 63, 65, 3, N, 1000, 4097, 2 * N + 5]
    flts = [False, True, False, True, False, False, True, False, True]
    g = mtgp.Generators(p, seeds)
    got = [[] for _ in range(p.shape[0])]
    for c, f in zip(calls, flts):
        out = g.generate(c, mtgp.F32 if f else mtgp.U32)
        h = _host(out).reshape(p.shape[0], c)
        for k in range(p.shape[0]):
            got[k].append(h[k])
    torch.cuda.synchronize()
    exp, exp_states = _oracle_run(p, seeds, calls, flts)
    for k in range(p.shape[0]):
        for i in range(len(calls)):
            assert np.array_equal(got[k][i], exp[k][i]), (mexp, k, i)
    assert np.array_equal(g.states_host(), exp_states)
    g.close()


@pytest.mark.parametrize("mexp", [3217, 23209])
def test_nonlinear_recursion_tables(torch, mexp):
    """Tables that are not GF(2) spans take the table-lookup paths (the
    windowed small-step path needs a linear recursion table)."""
    _say("case nonlinear tables mexp=%d" % mexp)
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 6, 0x4E4C + mexp)
    rng = np.random.default_rng(mexp)
    p[:, 5:21] = rng.integers(0, 2**32, (6, 16), dtype=np.uint64).astype(np.uint32)
    p[0, 1], p[1, 1], p[2, 1] = N - 2, N - 40, 1      # W = 2, 40, N-1
    seeds = np.arange(1, 7, dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    a = _host(g.generate(9000, mtgp.U32)).reshape(6, 9000)
    b = _host(g.generate(777, mtgp.F32)).reshape(6, 777)
    exp, exp_states = _oracle_run(p, seeds, [9000, 777], [False, True])
    for k in range(6):
        assert np.array_equal(a[k], exp[k][0]), k
        assert np.array_equal(b[k], exp[k][1]), k
    assert np.array_equal(g.states_host(), exp_states)
    g.close()


@pytest.mark.parametrize("w", [2, 3, 5, 16, 21, 23, 31, 32, 33, 63])
def test_every_short_step_width(torch, w):
    """Each lanes-per-class split (q = 64 // W) of the windowed path, and the
    W-word step path for the same streams (window threshold 0)."""
    for mexp in (11213, 44497):
        t0 = mtgp.get_tuning(mexp)
        N = mexp // 32 + 1
        p = workloads.make_params(mexp, 3, 0x5757 + w)
        p[:, 1] = N - w
        p[1, 3] = 0                                      # sh2 = 0
        p[2, 2], p[2, 3] = 31, 31
        seeds = np.array([0, 7, 0xFFFFFFFF], dtype=np.uint32)
        calls = [1, w - 1 if w > 1 else 1, 5 * N + 3, 2 * N]
        exp, exp_states = _oracle_run(p, seeds, calls, [False] * len(calls))
        try:
            for below in (64, 0):
                _say("case short W=%d mexp=%d window_below=%d" % (w, mexp, below))
                tt = t0.as_tuple()
                mtgp.set_tuning(mexp, tt[0], tt[1], tt[2], tt[3], below)
                g = mtgp.Generators(p, seeds)
                got = [_host(g.generate(c, mtgp.U32)).reshape(3, c) for c in calls]
                for k in range(3):
                    for i in range(len(calls)):
                        assert np.array_equal(got[i][k], exp[k][i]), (mexp, below, k, i)
                assert np.array_equal(g.states_host(), exp_states)
                g.close()
        finally:
            mtgp.set_tuning(mexp, *t0.as_tuple())


@pytest.mark.parametrize("mexp", [11213, 44497])
def test_every_compiled_tuning_gives_identical_output(torch, mexp):
    _say("case tunings mexp=%d" % mexp)
    p = _edge_params(mexp, 0x51 + mexp)
    seeds = np.arange(1, 9, dtype=np.uint32)
    count = 3001
    exp, exp_states = _oracle_run(p, seeds, [count, 517], [False, True])
    t0 = mtgp.get_tuning(mexp)
    try:
        for cand in mtgp.tuning_candidates(mexp):
            _say("  tuning", cand)
            mtgp.set_tuning(mexp, *cand.as_tuple())
            g = mtgp.Generators(p, seeds)
            a = _host(g.generate(count, mtgp.U32)).reshape(8, count)
            b = _host(g.generate(517, mtgp.F32)).reshape(8, 517)
            for k in range(8):
                assert np.array_equal(a[k], exp[k][0]), (cand, k)
                assert np.array_equal(b[k], exp[k][1]), (cand, k)
            assert np.array_equal(g.states_host(), exp_states), cand
            # the batch path with the same tuning
            g2 = mtgp.Generators(p, seeds)
            outs = [torch.empty(count, dtype=torch.int32, device="cuda") for _ in range(8)]
            g2.batch([(k, mtgp.U32, count, outs[k]) for k in range(8)])
            for k in range(8):
                assert np.array_equal(_host(outs[k]), exp[k][0]), ("batch", cand, k)
            g.close()
            g2.close()
    finally:
        mtgp.set_tuning(mexp, *t0.as_tuple())


def test_c1_full(torch):
    """4 streams x 2^20 uint32, seeds 1..4, full comparison; then 2^20 more
    as float32 continuing the streams."""
    _say("case C1 full")
    params, seeds = workloads.config_inputs("C1")
    count = workloads.CONFIGS["C1"]["count"]
    g = mtgp.Generators(params, seeds)
    u = _host(g.generate(count, mtgp.U32)).reshape(4, count)
    f = _host(g.generate(count, mtgp.F32)).reshape(4, count)
    exp, exp_states = _oracle_run(params, seeds, [count, count], [False, True])
    for k in range(4):
        assert np.array_equal(u[k], exp[k][0]), k
        assert np.array_equal(f[k], exp[k][1]), k
    assert np.array_equal(g.states_host(), exp_states)
    g.close()


def test_seed_zero_and_state_roundtrip(torch):
    _say("case seed0 + export/import")
    p = workloads.make_params(3217, 3, 99)
    seeds = np.zeros(3, dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    st0 = g.states_host()
    for k in range(3):
        assert np.array_equal(st0[k], oracle.seed(0, 101))
    a = _host(g.generate(5000)).reshape(3, 5000)
    mid = g.states_host()
    b = _host(g.generate(777)).reshape(3, 777)
    g.load_states(mid)                      # checkpoint restore
    b2 = _host(g.generate(777)).reshape(3, 777)
    assert np.array_equal(b, b2)
    exp, _ = _oracle_run(p, seeds, [5000, 777], [False, False])
    for k in range(3):
        assert np.array_equal(a[k], exp[k][0]) and np.array_equal(b[k], exp[k][1])
    g.close()


def test_batch_uneven_mixed_with_replays(torch):
    """Persistent kernel + hipGraph: uneven lengths, mixed dtypes, a subset
    of streams, three replays of the same graph continuing the streams."""
    _say("case batch uneven")
    mexp = 23209
    p = workloads.make_params(mexp, 40, 0xBA7C)
    seeds = np.arange(1, 41, dtype=np.uint32)
    rng = np.random.default_rng(4)
    sel = rng.choice(40, 25, replace=False)
    lens = rng.integers(1, 20000, 25)
    lens[0], lens[1] = 1, 0     # zero-length items are skipped
    dts = rng.integers(0, 2, 25)
    g = mtgp.Generators(p, seeds)
    ws = g.workspace(25)
    outs = [torch.empty(max(int(L), 1), dtype=torch.int32, device="cuda") for L in lens]
    items = [(int(s), int(d), int(L), o) for s, d, L, o in zip(sel, dts, lens, outs)]
    got = []
    for rep in range(3):
        g.batch(items, ws)
        got.append([_host(o)[:int(L)].copy() for o, L in zip(outs, lens)])
    # oracle: each selected stream advanced three times
    N = mexp // 32 + 1
    states = np.stack([oracle.seed(int(s), N) for s in seeds])
    for rep in range(3):
        for j, (s, d, L) in enumerate(zip(sel, dts, lens)):
            o, states[s] = oracle.generate(p[s], states[s], int(L), bool(d))
            assert np.array_equal(got[rep][j], np.asarray(o).view(np.uint32)), (rep, j)
    assert np.array_equal(g.states_host(), states)
    g.close()


def test_batch_rejects_duplicate_streams(torch):
    p = workloads.make_params(11213, 4, 1)
    g = mtgp.Generators(p, np.arange(4, dtype=np.uint32))
    o = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(mtgp.MTGPError) as e:
        g.batch([(1, 0, 8, o), (1, 0, 8, o)])
    assert "twice" in str(e.value)
    g.close()


def test_fill(torch):
    x = torch.zeros(1 << 20 | 3, dtype=torch.int32, device="cuda")
    mtgp.fill_u32(x, x.numel(), 0xDEADBEEF)
    assert np.all(_host(x) == 0xDEADBEEF)


def test_autotune_keeps_results_identical(torch):
    _say("case autotune")
    mexp = 11213
    p = workloads.make_params(mexp, 32, 0x7777)
    seeds = np.arange(1, 33, dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    before = g.states_host()
    outs = [torch.empty(4096, dtype=torch.int32, device="cuda") for _ in range(32)]
    items = [(k, k & 1, 4096, outs[k]) for k in range(32)]
    scratch = torch.empty(32 * 351 * 4 + 256 + mtgp.batch_workspace_bytes(32),
                          dtype=torch.uint8, device="cuda")
    t0 = mtgp.get_tuning(mexp)
    best, _ = mtgp.autotune(g.d_params, g.d_states, g.stride, items, scratch, reps=1)
    assert np.array_equal(g.states_host(), before)   # caller's states untouched
    assert mtgp.get_tuning(mexp).as_tuple() == best.as_tuple()
    g.batch(items)
    exp, _ = _oracle_run(p, seeds, [4096], [False])
    for k in range(0, 32, 2):
        assert np.array_equal(_host(outs[k]), exp[k][0])
    mtgp.set_tuning(mexp, *t0.as_tuple())
    g.close()


# ------------------------------------------------------- full-size runs ---

def _compare_streams(get_out, params, states0, counts, flts, chunk=16, threads=16):
    """Every stream's outputs against the oracle, `chunk` streams at a time
    (get_out(k) -> host uint32 array of stream k); returns the oracle's
    final states."""
    n = params.shape[0]
    counts = np.broadcast_to(np.asarray(counts, dtype=np.int64), (n,))
    flts = np.broadcast_to(np.asarray(flts, dtype=bool), (n,))
    final = np.array(states0, dtype=np.uint32, copy=True)
    for c0 in range(0, n, chunk):
        ks = list(range(c0, min(n, c0 + chunk)))
        exp, st = oracle.generate_many(params[ks], final[ks], counts[ks], flts[ks],
                                       threads=threads)
        final[ks] = st
        for j, k in enumerate(ks):
            got = get_out(k)
            want = np.asarray(exp[j]).view(np.uint32)
            if not np.array_equal(got, want):
                bad = int(np.flatnonzero(got != want)[0])
                raise AssertionError("stream %d differs first at output %d" % (k, bad))
    return final


def test_c2_full_size_batch_as_benched(torch):
    """128 streams x 2^24 (mexp 11213) exactly as the benchmark runs them:
    re-seed, uint32 pass through mtgp_generate_batch, re-seed, float32 pass,
    three steps (graph replays).  Every output of every stream of both
    passes and every final state against the oracle."""
    _say("case C2 full size, batch path as benched")
    params, seeds = workloads.config_inputs("C2")
    count = workloads.CONFIGS["C2"]["count"]
    n = params.shape[0]
    N = mtgp.state_words(int(params[0, 0]))
    g = mtgp.Generators(params, seeds)
    out_u = torch.empty(n * count, dtype=torch.int32, device="cuda")
    out_f = torch.empty(n * count, dtype=torch.float32, device="cuda")
    list_u = [(k, mtgp.U32, count, out_u.data_ptr() + 4 * k * count) for k in range(n)]
    list_f = [(k, mtgp.F32, count, out_f.data_ptr() + 4 * k * count) for k in range(n)]
    ws_u, ws_f = g.workspace(list_u), g.workspace(list_f)
    assert ws_u.numel() > mtgp.batch_workspace_bytes(n)   # jump-ahead splits the streams
    for step in range(3):
        for items, ws in ((list_u, ws_u), (list_f, ws_f)):
            g.reseed()
            g.batch(items, ws)
    torch.cuda.synchronize()
    assert mtgp.batch_errors(ws_u) == 0 and mtgp.batch_errors(ws_f) == 0
    end = g.states_host()
    init = np.stack([oracle.seed(int(s), N) for s in seeds])
    fin_u = _compare_streams(lambda k: _host(out_u[k * count:(k + 1) * count]),
                             params, init, count, False)
    fin_f = _compare_streams(lambda k: _host(out_f[k * count:(k + 1) * count]),
                             params, init, count, True)
    assert np.array_equal(fin_u, fin_f)
    assert np.array_equal(end, fin_f)
    g.close()


def test_c3_full_size_every_stream(torch):
    """4096 streams x 2^20 uint32 (mexp 23209, 16 GiB) in one persistent
    graph launch: every stream against the oracle."""
    _say("case C3 full size")
    params, seeds = workloads.config_inputs("C3")
    count = workloads.CONFIGS["C3"]["count"]
    n = params.shape[0]
    N = mtgp.state_words(int(params[0, 0]))
    g = mtgp.Generators(params, seeds)
    out = torch.empty(n * count, dtype=torch.int32, device="cuda")
    items = [(k, mtgp.U32, count, out.data_ptr() + 4 * k * count) for k in range(n)]
    ws = g.batch(items)
    torch.cuda.synchronize()
    assert mtgp.batch_errors(ws) == 0
    st = g.states_host()
    init = np.stack([oracle.seed(int(s), N) for s in seeds])
    per = 256   # streams per device-to-host copy (1 GiB)
    cache = {}

    def get(k):
        blk = k // per
        if blk not in cache:
            cache.clear()
            lo, hi = blk * per * count, min(n, (blk + 1) * per) * count
            cache[blk] = _host(out[lo:hi])
        return cache[blk][(k - blk * per) * count:(k - blk * per + 1) * count]

    fin = _compare_streams(get, params, init, count, False, chunk=64)
    assert np.array_equal(st, fin)
    del out
    g.close()


def test_c4_full_size_every_stream(torch):
    """1024 streams of mexp 44497, lengths log-uniform in [2^10, 2^24],
    dtype 50/50, one launch: every stream against the oracle."""
    _say("case C4 full size")
    params, seeds = workloads.config_inputs("C4")
    lens, dts = workloads.uneven_batch("C4")
    n = params.shape[0]
    N = mtgp.state_words(int(params[0, 0]))
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    g = mtgp.Generators(params, seeds)
    out = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    base = out.data_ptr()
    items = [(k, int(dts[k]), int(lens[k]), base + 4 * int(offs[k])) for k in range(n)]
    ws = g.batch(items)
    torch.cuda.synchronize()
    assert mtgp.batch_errors(ws) == 0
    st = g.states_host()
    host = _host(out)
    init = np.stack([oracle.seed(int(s), N) for s in seeds])
    fin = _compare_streams(lambda k: host[int(offs[k]):int(offs[k + 1])], params, init,
                           lens.astype(np.int64), dts.astype(bool), chunk=64)
    assert np.array_equal(st, fin)
    del out
    g.close()


@pytest.mark.parametrize("name", ["P1", "P2"])
def test_paper_shapes_full_size_every_stream(torch, name):
    """The paper's experiment shapes (mexp 3217, 2^20 uint32 per stream):
    P1 10,000 statuses at seed status 0, P2 100 statuses x 100 seeds, in one
    batch call as the benchmark runs them: every stream against the oracle."""
    _say("case %s full size" % name)
    params, seeds = workloads.config_inputs(name)
    count = workloads.CONFIGS[name]["count"]
    n = params.shape[0]
    N = mtgp.state_words(int(params[0, 0]))
    g = mtgp.Generators(params, seeds)
    out = torch.empty(n * count, dtype=torch.int32, device="cuda")
    items = [(k, mtgp.U32, count, out.data_ptr() + 4 * k * count) for k in range(n)]
    ws = g.batch(items)
    torch.cuda.synchronize()
    assert mtgp.batch_errors(ws) == 0
    st = g.states_host()
    init = np.stack([oracle.seed(int(s), N) for s in seeds])
    per = 256   # streams per device-to-host copy (1 GiB)
    cache = {}

    def get(k):
        blk = k // per
        if blk not in cache:
            cache.clear()
            lo, hi = blk * per * count, min(n, (blk + 1) * per) * count
            cache[blk] = _host(out[lo:hi])
        return cache[blk][(k - blk * per) * count:(k - blk * per + 1) * count]

    fin = _compare_streams(get, params, init, count, False, chunk=64)
    assert np.array_equal(st, fin)
    del out
    g.close()


def test_zero_counts_leave_streams_untouched(torch):
    """count = 0 is a valid no-op for the plain, workgroup and batch entry
    points: states do not move and the next call continues from the seed."""
    _say("case zero counts")
    mexp = 11213
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 3, 0x2E0)
    seeds = np.array([5, 6, 7], dtype=np.uint32)
    g = mtgp.Generators(p, seeds)
    before = g.states_host().copy()
    dummy = torch.empty(1, dtype=torch.int32, device="cuda")
    mtgp.generate(g.d_params, g.d_states, g.stride, 3, 0, dummy, mtgp.U32)
    mtgp.generate_workgroup(g.d_params, g.d_states, g.stride, 3, 0, dummy, mtgp.F32, 256)
    ws = g.workspace(3)
    g.batch([(k, 0, 0, dummy) for k in range(3)], ws)
    torch.cuda.synchronize()
    assert np.array_equal(g.states_host(), before)
    out = g.generate(100)
    for k in range(3):
        exp, _ = oracle.generate(p[k], oracle.seed(int(seeds[k]), N), 100, False)
        assert np.array_equal(_host(out).reshape(3, 100)[k], np.asarray(exp).view(np.uint32)), k
    g.close()


def test_single_stream_beyond_2p32_outputs(torch):
    """One stream of 2^32 + 1000 outputs in one batch call (jump-ahead
    splits it): 64-bit output indexing past 2^32 words.  The oracle runs the
    whole stream in chunks and keeps the head, the words around 2^32 and the
    final state."""
    _say("case one stream beyond 2^32")
    mexp = 11213
    N = mexp // 32 + 1
    p = workloads.make_params(mexp, 1, 0x2F32)
    seeds = np.array([11], dtype=np.uint32)
    count = (1 << 32) + 1000
    g = mtgp.Generators(p, seeds)
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    items = [(0, mtgp.U32, count, out)]
    ws = g.workspace(items)
    g.batch(items, ws)
    assert mtgp.batch_errors(ws) == 0
    head = _host(out[:1000])
    tail = _host(out[(1 << 32) - 1000:])
    state = oracle.seed(int(seeds[0]), N)
    exp_head, exp_tail = None, []
    chunk, done = 1 << 25, 0
    while done < count:
        c = min(chunk, count - done)
        o, state = oracle.generate(p[0], state, c, False)
        o = np.asarray(o).view(np.uint32)
        if done == 0:
            exp_head = o[:1000].copy()
        lo = max(done, (1 << 32) - 1000)
        if lo < done + c:
            exp_tail.append(o[lo - done:].copy())
        done += c
    assert np.array_equal(head, exp_head)
    assert np.array_equal(tail, np.concatenate(exp_tail))
    assert np.array_equal(g.states_host()[0], state)
    del out
    g.close()
