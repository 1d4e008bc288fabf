"""Build step for libnecsim_hip.so (gfx950) with hipcc, in-tree.

The library is compiled for gfx950 only, with floating-point contraction off
(the event-time arithmetic must be the exact operation sequence the method
specifies) and packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "necsim_hip.hip")
# radix sort and scan kernels of the event stream (own translation unit)
SORT_SRC = os.path.join(HERE, "csrc", "stream_sort.hip")
HEADER = os.path.join(ROOT, "include", "necsim_hip.h")
LIB = os.path.join(HERE, "libnecsim_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=None) -> str:
    """Compile the HIP library every time it is called; returns the .so path."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, *(extra or []), SRC, SORT_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
