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
# the kernel translation units, longest to compile first (PCPD has the extra
# copy compiled for its default pitch)
SOURCES = ["phase_n2.hip", "persist_n2.hip", "phase_n1.hip", "phase_n3.hip", "phase_n4.hip",
           "persist_n1.hip", "persist_n3.hip", "persist_n4.hip", "mlp.hip", "pcpd_api.hip",
           "sweep.hip"]
BUILD_DIR = os.path.join(PKG, "_build")
ARCH = "gfx950"

# hipcc flags: CDNA4 only; packed FP32 instructions disabled for all device code.
HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-fvisibility=hidden", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpcpd")
    return path


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit (in parallel) and link libpcpd.so."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *HIP_FLAGS, *inc, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=PKG)
        return obj

    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, *HIP_FLAGS, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=PKG)
    os.replace(tmp, LIB)
    return LIB


def device_asm(out_path: str, source: str = "phase_n2.hip") -> str:
    """gfx950 assembly of one source file, for instruction counts."""
    cmd = [hipcc(), *[f for f in HIP_FLAGS if f != "-fPIC"],
           "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"),
           "-o", out_path, os.path.join(CSRC, source)]
    subprocess.check_call(cmd, cwd=PKG)
    return out_path


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
