"""Builds tests/shims/host_sanitize_driver.cpp against the library's host
sources compiled with AddressSanitizer + UndefinedBehaviorSanitizer.

The host sources (mtgp_api.cpp, mtgp_batch.cpp, mtgp_server.cpp,
mtgp_sched.cpp, mtgp_poly.cpp) hold no device code, so ROCm's clang builds
them as plain C++ against the HIP runtime headers, with the sanitizers on.
The kernels object is the regular build's (paper_1501_07701_amd/_build/
mtgp_kernels.o, device code unchanged and uninstrumented).  Output:
paper_1501_07701_amd/_build/host_sanitized/driver.  Run on a machine with the
GPU; see tests/test_gpu_host_sanitized.py.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
PKG = os.path.join(ROOT, "paper_1501_07701_amd")
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build", "host_sanitized")
EXE = os.path.join(OUT, "driver")
CLANG = "/opt/rocm/llvm/bin/clang++"
ROCM = "/opt/rocm"

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
CFLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
          "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HOST = ["mtgp_api.cpp", "mtgp_batch.cpp", "mtgp_server.cpp", "mtgp_sched.cpp", "mtgp_poly.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(os.path.splitext(src)[0]) + ".o")
    extra = ["-mpclmul"] if src.endswith("mtgp_poly.cpp") else []
    cmd = [CLANG] + CFLAGS + SAN + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    return obj


def build(verbose: bool = False) -> str:
    kernels = os.path.join(PKG, "_build", "mtgp_kernels.o")
    if not os.path.exists(kernels):
        raise RuntimeError("build the library first (paper_1501_07701_amd/build.py)")
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in HOST]
    srcs.append(os.path.join(ROOT, "tests", "shims", "host_sanitize_driver.cpp"))
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = EXE + ".tmp%d" % os.getpid()
    cmd = [CLANG] + SAN + objs + [kernels, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                                  "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lpthread",
                                  "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    os.replace(tmp, EXE)
    if verbose:
        print("built", EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
