"""Builds the HIP library libleyenda.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIB_DIR, "libleyenda.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed fp32 ops (see the project notes on gfx950)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every global atomic on a uniform address here is issued by one lane, so
    # the wave-combining rewrite gains nothing; it also reads the result right
    # after issue, which would stall the local sort's task-id prefetch
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wno-unused-result", "-Wno-unknown-warning-option",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library.  Always recompiles."""
    os.makedirs(LIB_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
