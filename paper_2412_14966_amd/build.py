"""Build libpvfind.so (gfx950 kernels + C ABI) in-tree with hipcc.

Usage: ``python -m paper_2412_14966_amd.build``.  The library lands next to
this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpvfind.so")
SOURCES = [os.path.join(CSRC, "pvfind_kernels.hip"), os.path.join(CSRC, "pvfind_api.cpp"),
           os.path.join(CSRC, "pvfind_params.cpp"), os.path.join(CSRC, "pvfind_server.cpp"),
           os.path.join(CSRC, "pvfind_server_hip.cpp"), os.path.join(CSRC, "pvfind_measure.hip"),
           os.path.join(CSRC, "pvfind_compact.hip")]
ARCH = os.environ.get("PV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the projection and histogram stage must round every operation once
    "-ffp-contract=off",
    # packed FP32 instructions stay off (some of their forms misbehave)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-pthread",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
