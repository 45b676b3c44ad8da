"""Build libhyperpower.so in-tree with hipcc for gfx950.

    python -m paper_1604_07893_amd.build_lib

Each source is compiled to an object of its own (in parallel, under _build/),
then the objects are linked into the shared library.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libhyperpower.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["hp_gemm.hip", "hp_gemm_h16.hip", "hp_tiles.cpp", "hp_kernels.hip", "hp_driver.cpp",
           "hp_batch.cpp", "hp_loop.cpp", "hp_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # let `#pragma unroll` fully unroll the epilogues of the large 16-bit tiles
    # (128 accumulators per lane); past the default size limit the loop stays
    # rolled and the accumulators go to scratch memory. The other kernels
    # compile to the same code either way.
    "-mllvm", "-pragma-unroll-threshold=200000",
]


# roctx ranges around the solve's phases (rocprofv3 --marker-trace)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj,
           os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 8)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
