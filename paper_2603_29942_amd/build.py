"""Build the HIP library ``libbz.so`` for gfx950, in-tree.

    python -m paper_2603_29942_amd.build

One translation unit (``csrc/bz_api.hip``) holds the C ABI of ``include/bz.h``
and instantiates every kernel.  Packed-FP32 instruction selection is switched
off for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "bz_api.hip")
LIB = os.path.join(HERE, "libbz.so")
ARCH = "gfx950"


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(ROOT, "include"), SRC, "-o", LIB + ".tmp", *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
