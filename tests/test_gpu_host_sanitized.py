"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
on the GPU.

tests/shims/host_sanitize_driver.cpp, built by tests/shims/
build_host_sanitized.py from the host sources compiled with the sanitizers
and the regular kernels object, drives the C ABI end to end: validation,
plain launches, split batches (jump-ahead set-up, workspace sizing, per-call
table uploads), imported states, the allocation-free entry, the serving
runtime and the remaining entry points, comparing the paths bit for bit.
Leak reports from inside the HIP runtime's own libraries are suppressed;
anything else the sanitizers find fails the test.
"""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1501_07701_amd", "_build", "host_sanitized", "driver")

SUPPRESSIONS = "\n".join([
    "leak:libamdhip64",
    "leak:libhsa-runtime64",
    "leak:libamd_comgr",
    "leak:libhsakmt",
    "leak:librocprofiler",
    "leak:libdrm",
]) + "\n"


@pytest.mark.gpu
def test_host_code_under_asan_ubsan(tmp_path):
    if not os.path.exists(EXE):
        pytest.skip("host-sanitized driver not built (tests/shims/build_host_sanitized.py)")
    supp = tmp_path / "lsan.supp"
    supp.write_text(SUPPRESSIONS)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:protect_shadow_gap=0"
    env["LSAN_OPTIONS"] = "suppressions=%s:print_suppressions=0" % supp
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0, (r.stdout[-3000:] + r.stderr[-8000:])
    assert "host sanitize driver: ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-8000:]
