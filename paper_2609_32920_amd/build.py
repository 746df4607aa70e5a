"""Compile the HIP library liblt.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblt.so")
LIB_COUNTERS = os.path.join(HERE, "liblt_counters.so")
SOURCES = ["lt_kernels.hip", "lt_guide.hip", "lt_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value",
]


def _build_one(out: str, extra, verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs]
    # .cpp files are host+device HIP sources as well
    cmd.insert(1, "-x")
    cmd.insert(2, "hip")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Product library plus the diagnostic counters build."""
    _build_one(LIB_COUNTERS, ["-DLT_COUNTERS"], verbose)
    return _build_one(LIB, [], verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
