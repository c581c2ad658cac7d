"""Builds libdpgmi.so (the HIP library behind include/dpg.h) in-tree for gfx950.

    python -m paper_2609_03155_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdpgmi.so")
SOURCES = ["csrc/dpg_kernels.hip", "csrc/dpg_trace_kernels.hip", "csrc/dpg_marking.hip", "csrc/dpg_api.cpp",
           "csrc/dpg_tables.cpp", "csrc/dpg_trace.cpp"]

# Packed FP32 instructions are disabled for every device compilation.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-shared", *DEVICE_FLAGS,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", LIB + ".tmp", *[os.path.join(HERE, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libdpgmi.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
