"""Builds the gfx950 shared library libomap.so from csrc/ with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (the kernels are integer-only, so nothing is lost).
"""
from __future__ import annotations

import concurrent.futures
import os
import re
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libomap.so")
SOURCES = ["omap_kernels.hip", "omap_runtime.hip", "omap_tune.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = os.environ.get("OMAP_LINKER", "/opt/rocm/lib/llvm/bin/clang++")
ROCM_LIB = "/opt/rocm/lib"

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def variants() -> list:
    """(T, C) pairs of the sweep variants, as listed in omap_internal.h."""
    text = open(os.path.join(CSRC, "omap_internal.h")).read()
    body = text[text.index("#define OMAP_SWEEP_VARIANTS(X)"):]
    body = body[:body.index("\n\n")]
    return [(int(t), int(c)) for t, c in re.findall(r"X\((\d+),\s*(\d+)\)", body)]


def bits_variants() -> list:
    """Layers per visit of the bit-sliced variants, as listed in omap_internal.h."""
    text = open(os.path.join(CSRC, "omap_internal.h")).read()
    line = text[text.index("#define OMAP_BITS_VARIANTS(X)"):].split("\n", 1)[0]
    return [int(t) for t in re.findall(r"X\((\d+)\)", line)]


def _compile_jobs(build_dir):
    jobs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        jobs.append(([os.path.join(CSRC, src)], obj))
    for t, c in variants():
        obj = os.path.join(build_dir, f"sweep_T{t}_C{c}.o")
        jobs.append(([f"-DOMAP_T={t}", f"-DOMAP_C={c}", os.path.join(CSRC, "omap_sweep_variant.hip")], obj))
    for t in bits_variants():
        obj = os.path.join(build_dir, f"bits_T{t}.o")
        jobs.append(([f"-DOMAP_BITS_T={t}", os.path.join(CSRC, "omap_bits_variant.hip")], obj))
    return jobs


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (one object per sweep variant, in parallel) and
    link libomap.so (always rebuilds)."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    todo = _compile_jobs(build_dir)
    n = jobs or max(1, min(len(todo), os.cpu_count() or 1, 16))

    def run(job):
        args, obj = job
        cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", *args, "-o", obj]
        t0 = time.time()
        r = subprocess.run(cmd, capture_output=True, text=True)
        if verbose:
            print(f"{time.time() - t0:6.1f} s  {' '.join(cmd)}", flush=True)
        return obj, r.returncode, r.stderr

    with concurrent.futures.ThreadPoolExecutor(max_workers=n) as ex:
        results = list(ex.map(run, todo))
    failed = [(obj, err) for obj, rc, err in results if rc != 0]
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"{o}:\n{e}" for o, e in failed))
    objs = [obj for obj, _, _ in results]
    # Each object already carries its finished gfx950 code object (no
    # relocatable device code), so a plain host link suffices.
    tmp = LIB + ".tmp"
    cmd = [CLANG, "-shared", "-fPIC", "-o", tmp, *objs, "-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lamdhip64"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def assembly(src: str = "omap_kernels.hip", defines=()) -> str:
    """gfx950 assembly of one source (for inspecting instruction selection);
    a sweep variant is omap_sweep_variant.hip with defines ("OMAP_T=16", "OMAP_C=2")."""
    tag = "".join("_" + d.replace("=", "") for d in defines)
    out = os.path.join(HERE, "_build", src.replace(".hip", tag + ".s"))
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.check_call([HIPCC, *FLAGS, *("-D" + d for d in defines), "-I", INCLUDE, "-I", CSRC,
                           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out])
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
