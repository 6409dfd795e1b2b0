"""Build libfloquet.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2102_05054_amd.build  (or build() from Python).
Every .hip / .cpp file under csrc/ is compiled for gfx950 and linked into
paper_2102_05054_amd/libfloquet.so.  Object files go to _build/ at the
repository root.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfloquet.so")

ARCH = os.environ.get("FQ_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # std::complex products and quotients of the host-side dense algebra
    # (Schur form of the projected matrix) inline as plain formulas instead of
    # calls that rescale for infinities and NaNs; its entries are O(1)
    "-fcx-limited-range",
    # host code for x86-64-v3 (AVX2 and FMA, which every EPYC host of an
    # MI355X has): the complex Schur step of the restart (host QR sweeps on
    # the projected matrix) runs ~1.7x faster at 256 x 256 than with the
    # baseline x86-64 instruction set
    "-Xarch_host", "-march=x86-64-v3",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# ---------------------------------------------------------------------------
# Host mock of the device layer (test infrastructure, no GPU): the Krylov-Schur
# driver sources compiled with g++ against hostmock/ (a host stand-in for the
# HIP runtime and the kernels, with a diagonal mock operator), as a shared
# library for the CPU tests and as a self-test executable built with the
# address and undefined-behaviour sanitizers.  Neither is part of libfloquet.so.
# ---------------------------------------------------------------------------
MOCK_DIR = os.path.join(HERE, "hostmock")
MOCK_LIB = os.path.join(MOCK_DIR, "libfloquet_hostmock.so")
MOCK_SELFTEST = os.path.join(BUILD, "hostmock_selftest_asan")
MOCK_DRIVER_SOURCES = ["krylov.cpp", "block.cpp", "dense.cpp"]
MOCK_FLAGS = ["-std=c++17", "-Wall", "-Wno-unused-function", "-fcx-limited-range",
              "-I", MOCK_DIR, "-I", os.path.join(ROOT, "include")]


def _gxx(args):
    r = subprocess.run(["g++", *args], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed: g++ {' '.join(args)}\n{r.stdout}\n{r.stderr}")


def mock_sources():
    return [os.path.join(CSRC, f) for f in MOCK_DRIVER_SOURCES] + [os.path.join(MOCK_DIR, "hostmock.cpp")]


def build_hostmock(verbose: bool = True) -> str:
    """libfloquet_hostmock.so: the driver on the host mock (plain build)."""
    os.makedirs(BUILD, exist_ok=True)
    tmp = MOCK_LIB + ".tmp"
    _gxx([*MOCK_FLAGS, "-O1", "-g", "-fPIC", "-shared", *mock_sources(), "-o", tmp])
    os.replace(tmp, MOCK_LIB)
    if verbose:
        print(f"built {MOCK_LIB}")
    return MOCK_LIB


def build_hostmock_selftest(verbose: bool = True) -> str:
    """The driver on the host mock under AddressSanitizer + UBSan (host code
    only, nothing for the GPU), with the scenario driver hostmock/selftest.cpp."""
    os.makedirs(BUILD, exist_ok=True)
    tmp = MOCK_SELFTEST + ".tmp"
    _gxx([*MOCK_FLAGS, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", *mock_sources(), os.path.join(MOCK_DIR, "selftest.cpp"), "-o", tmp])
    os.replace(tmp, MOCK_SELFTEST)
    if verbose:
        print(f"built {MOCK_SELFTEST}")
    return MOCK_SELFTEST


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    build_hostmock(verbose)
    build_hostmock_selftest(verbose)
    return LIB


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
