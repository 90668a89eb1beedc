"""Build libp1e.so (host setup + gfx950 kernels) in-tree with hipcc.

Usage: ``python paper_2109_01158_amd/build.py`` (by path: importing the package itself
needs the library). Always recompiles; the result is written next to this file.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libp1e.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["p1e_api.cpp", "p1e_tiles.cpp", "p1e_kernels.hip", "p1e_batch.hip", "p1e_serve.cpp"]

# -packed-fp32-ops keeps the compiler from emitting packed FP32 arithmetic; contraction is
# off because the kernels place their fused multiply-adds explicitly.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libp1e.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
