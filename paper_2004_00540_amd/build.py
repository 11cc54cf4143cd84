"""Builds the gfx950 shared library libomap.so from csrc/ with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (the kernels are integer-only, so nothing is lost).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libomap.so")
SOURCES = ["omap_kernels.hip", "omap_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every source and link libomap.so (always rebuilds)."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def assembly(src: str = "omap_kernels.hip") -> str:
    """gfx950 assembly of one source (for inspecting instruction selection)."""
    out = os.path.join(HERE, "_build", src.replace(".hip", ".s"))
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.check_call([HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, "--cuda-device-only", "-S",
                           os.path.join(CSRC, src), "-o", out])
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
