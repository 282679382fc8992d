"""Build the HIP library libasi.so for gfx950, in-tree.

    python -m paper_2002_11401_amd.build

FP64 model arithmetic must not be contracted into FMAs (-ffp-contract=off):
every kernel that evaluates the same expression must produce the same bits.
Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", "asi_kernels.hip"), os.path.join(PKG, "csrc", "asi_runtime.hip")]
LIB = os.path.join(PKG, "libasi.so")
ARCH = os.environ.get("ASI_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out: str):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
            *SRC, "-L", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"),
            "-lrocprofiler-sdk-roctx", "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
