"""Build libace.so (HIP, gfx950) in-tree.

    python -m paper_2202_04140_amd.build

The host graph builder (graph.cpp) is plain C++17 and is compiled with g++;
the kernels and the C ABI (ace.hip, which includes kernels.hip) with hipcc
for gfx950 only.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libace.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def hipcc() -> str:
    p = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; a ROCm toolchain is required to build libace.so")
    return p


def build(verbose: bool = True) -> str:
    """Compile graph.cpp and ace.hip and link libace.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    graph_o = os.path.join(BUILD, "graph.o")
    ace_o = os.path.join(BUILD, "ace.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c",
          os.path.join(CSRC, "graph.cpp"), "-o", graph_o])
    _run([hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, "ace.hip"), "-o", ace_o])
    tmp = LIB + ".tmp"
    _run([hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", ace_o, graph_o, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
