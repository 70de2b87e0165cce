"""Build the gfx950 shared library libmxw.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmxw.so")
SOURCES = ["basis.cpp", "layout.cpp", "fem_kernels.hip", "lu_kernels.hip", "solve_kernels.hip", "multi_solve.hip", "block_krylov.hip", "recycle_kernels.hip", "api.hip"]


def hipcc_cmd(out: str, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 instructions anywhere in device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-result", "-o", out]
    cmd += list(extra)
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    return cmd


def build(verbose: bool = False) -> str:
    """Compile every source into libmxw.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmxw.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
