"""Build the oracle library (test infrastructure) with the host C compiler.

    python -m oracle.build

Produces ``oracle/libbzref.so`` from ``oracle/bzref.c``.  The oracle is plain
C99 with POSIX threads; it is compiled with gcc and never linked into, or
loaded by, the GPU library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bzref.c")
LIB = os.path.join(HERE, "libbzref.so")


def build(verbose: bool = False, src: str = SRC, lib: str = LIB) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-D_POSIX_C_SOURCE=200809L", src, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
