"""Build ``libpdinp.so`` (HIP for gfx950 + the C ABI host code) in-tree.

Usage: ``python -m paper_2008_10273_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdinp.so")
SOURCES = [os.path.join(CSRC, n) for n in
           ("pdinp_host.cpp", "pdinp_graph.cpp", "pdinp_server.cpp", "pdinp_kernels.hip",
            "pdinp_wide.hip", "pdinp_diffusion.hip", "pdinp_select.hip", "pdinp_noalloc.hip")]
ARCH = os.environ.get("PDI_OFFLOAD_ARCH", "gfx950")

# Packed FP32 VALU forms are kept out of the generated code.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include")]


# Per-source extra flags: the wave-per-block kernel keeps its rows in
# registers, so its loops over columns must unroll completely.
EXTRA_FLAGS = {"pdinp_wide.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [hipcc()] + HIPCC_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc()] + [f for f in HIPCC_FLAGS if not f.startswith("--offload-arch")] + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
