"""Compile libace.so (all HIP sources, gfx950) in-tree.

python -m paper_1601_07159_amd.build   (or call build())

build_host_checks() (also run by build()) compiles the same sources with the
host code under AddressSanitizer and UndefinedBehaviorSanitizer (device code
as usual) and links them with the C-ABI checks of tests/native/host_checks.cpp
into tests/native/ace_host_checks.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libace.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["api.hip", "fft_passes.hip", "dense.hip", "gemm_mfma.hip", "batched.hip",
           "tune.hip", "noalloc.hip", "eigen.hip", "persist.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# host code only: each sanitizer flag goes to the host compilation
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-g", "-fno-gpu-sanitize"]
SAN_DIR = os.path.join(BUILD_DIR, "san")
CLANG = os.environ.get("ACE_CLANG", "/opt/rocm/llvm/bin/clang++")
CHECKS_SRC = os.path.join(ROOT, "tests", "native", "host_checks.cpp")
CHECKS_OUT = os.path.join(ROOT, "tests", "native", "ace_host_checks")


def _compile(src: str, out_dir: str = BUILD_DIR, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed:\n{r.stderr[-4000:]}")


def build_host_checks(verbose: bool = True, jobs: int = 0) -> str:
    """The sanitized host-check program (host code of libace and the checks
    under ASan + UBSan, device code unchanged)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, SAN_DIR, SAN_HOST_FLAGS), SOURCES))
    san = "-fsanitize=address,undefined"   # host-only compile and link lines (clang++, no HIP)
    drv = os.path.join(SAN_DIR, "host_checks.o")
    _run([CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", san,
          "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-c", CHECKS_SRC, "-o", drv], "host checks compile")
    tmp = CHECKS_OUT + ".tmp"
    _run([CLANG, san, "-o", tmp, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib"], "host checks link")
    shutil.move(tmp, CHECKS_OUT)
    if verbose:
        print(f"built {CHECKS_OUT}", file=sys.stderr)
    return CHECKS_OUT


def build(verbose: bool = True, host_checks: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    checks = None
    if host_checks:
        # the sanitized build runs beside the plain one (its longest source
        # sets the time of both)
        pool = cf.ThreadPoolExecutor(1)
        checks = pool.submit(build_host_checks, verbose, jobs)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    shutil.move(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    if checks is not None:
        checks.result()
        pool.shutdown()
    return OUT


if __name__ == "__main__":
    if "--host-checks-only" in sys.argv:
        build_host_checks()
    else:
        build(host_checks="--no-host-checks" not in sys.argv)
