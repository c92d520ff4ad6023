"""Build liblbm.so (the HIP library behind include/lbm.h) in-tree for gfx950.

    python -m paper_2106_01557_amd.build            # build, print the hipcc lines
    python -m paper_2106_01557_amd.build --resources   # also print per-kernel VGPR/SGPR/LDS use

Every HIP translation unit is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  The C++ host files go
through hipcc as well so that one toolchain links the library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm.so")
ARCH = "gfx950"

SOURCES = ["lbm_kernels.hip", "lbm_bounded.hip", "lbm_api.cpp", "lbm_batch.cpp", "thermo.cpp",
           "unet_kernels.hip"]
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def compile_command(src: str, resources: bool = False) -> tuple:
    """(hipcc command, object path) of one source file."""
    path = os.path.join(CSRC, src)
    obj = os.path.join(HERE, "_build", src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c"] + lang + [
        path, "-o", obj, "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"] + NO_PACKED_FP32
    if src in ("lbm_kernels.hip", "lbm_bounded.hip"):
        # contract a*b+c only within one source expression: the fused-multiply-add
        # decisions then do not depend on the surrounding code, and the one- and
        # two-column kernel forms (and the batched kernel) give bitwise equal states
        cmd += ["-ffp-contract=on"]
    if src.endswith(".hip") and resources:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    return cmd, obj


def build(verbose: bool = True, resources: bool = False) -> str:
    """Compiles every source (in parallel, one hipcc per file) and links liblbm.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = [compile_command(src, resources) for src in SOURCES]
    if verbose:
        for cmd, _ in jobs:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as pool:
        results = list(pool.map(lambda j: subprocess.run(j[0], capture_output=True, text=True), jobs))
    for (cmd, _), res in zip(jobs, results):
        if verbose or res.returncode:
            sys.stdout.write(res.stdout)
            sys.stderr.write(res.stderr)
        if res.returncode:
            raise subprocess.CalledProcessError(res.returncode, cmd)
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resources="--resources" in sys.argv)
