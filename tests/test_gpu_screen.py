"""GPU parity of the screening counts (mtgp_screen) against the oracle's
definitions, bit for bit (integer counts), on seeded random words with
planted structure (runs of hits and of equal weights), stream lengths that
leave ragged chunks, and every supported bin count edge."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import screens
from paper_1501_07701_amd import mtgp, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    mtgp.lib()
    return t


def _words(n_streams, count, master):
    z = workloads.splitmix64(np.arange(n_streams * count, dtype=np.uint64), master)
    x = (z >> np.uint64(32)).astype(np.uint32).reshape(n_streams, count)
    x[0, 100:400] = 7                         # a long run of misses (small words)
    x[1, 50:60] = 0x80000000                  # a run of hits
    x[2, :] = 0xFFFFFFFF                      # every word weight 32
    return x


@pytest.mark.parametrize("count,bins,lo,hi", [
    (2, 2, 0, 1 << 31), (1000, 16, 1 << 31, 3 << 30), (65537, 64, 0, 1 << 28),
    (256 * 37 + 5, 8, 0x12345678, 0x9ABCDEF0)])
def test_screen_counts_match_oracle(torch, count, bins, lo, hi):
    print("case screen count=%d bins=%d" % (count, bins), flush=True)
    n = 4
    x = _words(n, count, 0x5C + count)
    d_x = torch.from_numpy(x.view(np.int32).copy()).cuda()
    d_c = torch.zeros(n * (bins + 9), dtype=torch.int64, device="cuda")
    mtgp.screen(d_x, n, count, lo, hi, bins, d_c)
    got = d_c.cpu().numpy().view(np.uint64).reshape(n, bins + 9)
    for k in range(n):
        assert np.array_equal(got[k, :bins], screens.gap_counts(x[k], lo, hi, bins)), k
        assert np.array_equal(got[k, bins:].reshape(3, 3), screens.hwd_counts(x[k])), k


def test_screen_rejects_bad_arguments(torch):
    d_x = torch.zeros(64, dtype=torch.int32, device="cuda")
    d_c = torch.zeros(80, dtype=torch.int64, device="cuda")
    for args in ((1, 1, 0, 10, 8), (1, 64, 10, 10, 8), (1, 64, 0, 10, 1),
                 (1, 64, 0, 10, 65), (0, 64, 0, 10, 8)):
        n, c, lo, hi, b = args
        with pytest.raises(mtgp.MTGPError):
            mtgp.screen(d_x, n, c, lo, hi, b, d_c)
