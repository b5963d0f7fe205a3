"""The C-ABI library loads and exports every function include/mtgp.h declares,
and its host-only entry points (validation, tuning tables, error strings)
behave as documented.  No compute calls: these run without a GPU."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1501_07701_amd import mtgp, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtgp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mtgp_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mtgp.LIB_PATH):
        from paper_1501_07701_amd import build
        build.build()
    return mtgp.lib()


def test_header_declares_the_core_entry_points():
    names = _declared()
    for n in ("mtgp_init_states", "mtgp_generate_u32", "mtgp_generate_f32",
              "mtgp_generate_batch", "mtgp_server_create", "mtgp_submit", "mtgp_poll"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", mtgp.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(lib, n)


def test_binding_covers_every_declared_symbol():
    assert sorted(mtgp._SIGS) == _declared()


def _params(mexp=11213, n=4):
    return workloads.make_params(mexp, n, 0x1234)


def test_state_words(lib):
    assert mtgp.state_words(3217) == 101
    assert mtgp.state_words(11213) == 351
    assert mtgp.state_words(23209) == 726
    assert mtgp.state_words(44497) == 1391
    with pytest.raises(mtgp.MTGPError) as e:
        mtgp.state_words(19937)
    assert e.value.code == mtgp.EINVAL


def test_check_params_accepts_workloads(lib):
    for mexp in workloads.SUPPORTED_MEXP:
        mtgp.check_params(workloads.make_params(mexp, 64, 7))
        mtgp.check_params(workloads.make_params(mexp, 64, 7, float_family="independent"))


@pytest.mark.parametrize("col,val,needle", [
    (0, 19937, "unsupported mexp"),
    (4, 0xFFF00000, "mask"),
    (1, 0, "pos=0"),
    (1, 350, "pos=350"),
    (2, 32, "sh1=32"),
    (3, 99, "sh2=99"),
    (40, 0x40000000, "flt_tbl"),
])
def test_check_params_rejects_bad_fields(lib, col, val, needle):
    p = _params()
    p[2, col] = val
    with pytest.raises(mtgp.MTGPError) as e:
        mtgp.check_params(p)
    assert e.value.code == mtgp.EINVAL
    assert needle in str(e.value)
    assert "stream 2" in str(e.value)


def test_mixed_mexp_rejected(lib):
    p = np.concatenate([_params(11213, 2), _params(3217, 2)])
    with pytest.raises(mtgp.MTGPError) as e:
        mtgp.check_params(p)
    assert "differs" in str(e.value)


def test_unknown_params_buffer_rejected(lib):
    # generation on a buffer the library never initialised fails before
    # touching the device
    with pytest.raises(mtgp.MTGPError) as e:
        mtgp.generate(0x1000, 0x2000, 351, 1, 16, 0x3000, mtgp.U32, stream=0)
    assert e.value.code == mtgp.EINVAL
    assert "not written by" in str(e.value)


def test_tuning_tables(lib):
    for mexp in workloads.SUPPORTED_MEXP:
        cands = mtgp.tuning_candidates(mexp)
        assert len(cands) >= 4
        wgs = {c.workgroup_size for c in cands}
        assert {256, 512, 1024} <= wgs
        t0 = mtgp.get_tuning(mexp)
        assert t0.as_tuple() in {c.as_tuple() for c in cands}
        c = cands[-1]
        mtgp.set_tuning(mexp, *c.as_tuple())
        assert mtgp.get_tuning(mexp).as_tuple() == c.as_tuple()
        mtgp.set_tuning(mexp, *t0.as_tuple())
    with pytest.raises(mtgp.MTGPError):
        mtgp.set_tuning(11213, 64, 3, 256)
    for bad in (-1, 65):
        with pytest.raises(mtgp.MTGPError) as e:
            mtgp.set_tuning(11213, 64, 4, 256, 2048, bad)
        assert "window_below_w" in str(e.value)


def test_default_tunings(lib):
    # the measured defaults: one wave per stream, 4 waves per workgroup, K = 4
    # up to N = 400 and 8 above, jump segments of at least 1024 steps, and the
    # windowed scan below W = 64 (N <= 128), 48 (N = 351) or 56
    expected = {3217: (64, 4, 256, 1024, 64), 11213: (64, 4, 256, 1024, 48),
                23209: (64, 8, 256, 1024, 56), 44497: (64, 8, 256, 1024, 56)}
    for mexp, want in expected.items():
        assert mtgp.get_tuning(mexp).as_tuple() == want, mexp


def test_strerror(lib):
    assert lib.mtgp_strerror(0) == b"ok"
    assert b"pool" in lib.mtgp_strerror(mtgp.ETOOBIG)
    assert lib.mtgp_strerror(-99) == b"unknown error"


def test_batch_workspace_size(lib):
    # header + one 80-byte item per request, 256-aligned
    assert mtgp.batch_workspace_bytes(0) == 256
    assert mtgp.batch_workspace_bytes(10) == 256 + 1024
    assert mtgp.batch_workspace_bytes(1000) == 256 + 80128


def test_library_has_no_oracle_dependency():
    """The product library links nothing from oracle/."""
    out = subprocess.run(["nm", "-D", mtgp.LIB_PATH], check=True, capture_output=True,
                         text=True).stdout
    assert "oracle_" not in out
    for root, _, files in os.walk(os.path.join(ROOT, "paper_1501_07701_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(root, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "mtgp_oracle" not in txt, f


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU and says so when asked for more."""
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([_sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
