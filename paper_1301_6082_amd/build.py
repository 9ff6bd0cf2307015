"""Build libpcpd.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1301_6082_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpcpd.so")
SOURCES = ["sweep.hip", "pcpd_api.hip", "mlp.hip"]
ARCH = "gfx950"

# hipcc flags: CDNA4 only; packed FP32 instructions disabled for all device code.
HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-fvisibility=hidden", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpcpd")
    return path


def build_library(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=PKG)
    os.replace(tmp, LIB)
    return LIB


def device_asm(out_path: str, source: str = "sweep.hip") -> str:
    """gfx950 assembly of one source file, for instruction counts."""
    cmd = [hipcc(), *[f for f in HIP_FLAGS if f not in ("-shared", "-fPIC")],
           "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-o", out_path, os.path.join(CSRC, source)]
    subprocess.check_call(cmd, cwd=PKG)
    return out_path


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
