"""Build ``oracle/libeig3_plain.so`` from ``eig3_plain.c`` with the host C
compiler.  Flags: -O2, -ffp-contract=off (the paper's algorithms with one
rounding per operation, no fused multiply-add), OpenMP over matrices."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eig3_plain.c")
LIB = os.path.join(HERE, "libeig3_plain.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall"]


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile ``src`` into the shared library ``out`` (atomically replaced)."""
    cc = os.environ.get("CC", "gcc")
    tmp = out + ".tmp"
    cmd = [cc, *CFLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
