"""Build ``tests/c_abi/c_caller`` (a plain C test program that calls libeig3
through include/eig3.h with hipMalloc'd memory and its own stream) with the
host C compiler against the HIP runtime and the in-tree libeig3.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "c_caller.c")
EXE = os.path.join(HERE, "c_caller")


def build(verbose: bool = False) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    libdir = os.path.join(ROOT, "paper_2511_00292_amd")
    cc = os.environ.get("CC", "gcc")
    tmp = EXE + ".tmp"
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(rocm, "include"), SRC, "-o", tmp,
           "-L", libdir, "-leig3", "-Wl,-rpath,$ORIGIN/../../paper_2511_00292_amd",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
