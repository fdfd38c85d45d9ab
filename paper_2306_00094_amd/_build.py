"""Build the HIP library of the solver for gfx950 (in-tree shared object)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "_dd.so")
SOURCES = [os.path.join(HERE, "csrc", "dd_lib.hip")]
HEADERS = [os.path.join(HERE, "csrc", "dd_kernels.h"), os.path.join(ROOT, "include", "dd.h")]


def hipcc_cmd(out: str) -> list:
    return ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *SOURCES, "-o", out]


def build(verbose: bool = False) -> str:
    """Compile the solver library; always rebuilds."""
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
