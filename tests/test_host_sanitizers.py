"""Host code under the sanitizers, on the CPU.

* The serving scheduler (csrc/mtgp_sched.cpp: admission in submission order
  under a pool budget, per-stream FIFO, fusion of a stream's consecutive
  requests, at most one item per stream in flight, cancellation, release,
  replay, shutdown with waiters) driven by tests/shims/sched_driver.cpp
  against a fake device, built once with AddressSanitizer +
  UndefinedBehaviorSanitizer and once with ThreadSanitizer.  The fake device
  fills each result with words that encode (stream, position, dtype), so a
  result is right exactly when it continues its stream where the stream's
  previous completed request stopped -- the server's promise that each
  result is the next `count` outputs of its stream.
* The jump-ahead planner's GF(2)[x] routines (csrc/mtgp_poly.cpp) against
  bit-by-bit schoolbook arithmetic (tests/shims/poly_driver.cpp) under
  AddressSanitizer + UndefinedBehaviorSanitizer.

ThreadSanitizer builds use ROCm's clang: the GCC 11 runtime does not
intercept pthread_cond_clockwait (what std::condition_variable::wait_for
calls), loses track of the mutex inside such waits and reports races
between accesses that both hold it.
"""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1501_07701_amd", "csrc")
INC = os.path.join(ROOT, "include")
SHIMS = os.path.join(ROOT, "tests", "shims")
CLANG = "/opt/rocm/llvm/bin/clang++"

ASAN_UBSAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer"]
ENV = {
    "ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:strict_string_checks=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    "TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1",
}


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitized"))


def _build(compiler, flags, sources, exe):
    cmd = [compiler, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-I", CSRC, "-I", INC]
    cmd += flags + sources + ["-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, "build failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-4000:])


def _run(exe, *args):
    env = dict(os.environ)
    env.update(ENV)
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=240, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-6000:]
    return r.stdout


SCENARIOS = ["pool_consistency", "threads_fifo_pool_pressure", "fusion_and_order",
             "fusion_capped_by_pool", "admission_errors", "launch_and_device_failures",
             "shutdown_with_waiters", "replay_keeps_results", "replay_failure_cleanup",
             "shutdown_during_replay", "batch_cap_and_window"]


def _check_scenarios(stdout):
    for sc in SCENARIOS:
        assert "PASS " + sc in stdout, stdout
    assert "FAIL" not in stdout, stdout
    assert "%d scenarios, 0 failed checks" % len(SCENARIOS) in stdout, stdout


def test_scheduler_asan_ubsan(outdir):
    exe = os.path.join(outdir, "sched_asan")
    _build("g++", ASAN_UBSAN, [os.path.join(SHIMS, "sched_driver.cpp"),
                               os.path.join(CSRC, "mtgp_sched.cpp")], exe)
    _check_scenarios(_run(exe))


def test_scheduler_tsan(outdir):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang not found")
    exe = os.path.join(outdir, "sched_tsan")
    _build(CLANG, ["-fsanitize=thread"], [os.path.join(SHIMS, "sched_driver.cpp"),
                                          os.path.join(CSRC, "mtgp_sched.cpp")], exe)
    # twice: thread interleavings differ from run to run
    _check_scenarios(_run(exe))
    _check_scenarios(_run(exe))


def test_scheduler_release_build_is_warning_free(outdir):
    obj = os.path.join(outdir, "mtgp_sched.o")
    cmd = ["g++", "-std=c++17", "-O3", "-Wall", "-Wextra", "-Werror", "-I", CSRC, "-I", INC,
           "-c", os.path.join(CSRC, "mtgp_sched.cpp"), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_poly_asan_ubsan(outdir):
    exe = os.path.join(outdir, "poly_asan")
    _build("g++", ASAN_UBSAN + ["-mpclmul"], [os.path.join(SHIMS, "poly_driver.cpp"),
                                              os.path.join(CSRC, "mtgp_poly.cpp")], exe)
    assert "poly checks: 0 failed" in _run(exe)
