"""Build libhwisard.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2403_20190_amd.build   (or call build())
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhwisard.so")
SOURCES = ["hw_kernels.hip", "hw_microbench.hip", "hw_noalloc.hip", "hw_pbs.hip", "hw_api.cpp",
           "hw_batch_run.cpp", "hw_engine.cpp"]
HEADERS = ["hw_device.h", "hw_internal.h", "hw_ctx.h"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed fp32 instructions stay off (the path has no fp32 arithmetic anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the host builds the Gaussian table in double: no contraction into FMAs
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_2403_20190_amd/libhwisard.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *FLAGS, "-x", "hip", *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhwisard.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
