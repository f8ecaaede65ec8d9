"""Build libtrs.so (the HIP library behind include/trs.h) for gfx950.

Run ``python -m paper_2009_07174_amd.build``; the shared object is written
next to this file and loaded by ``paper_2009_07174_amd.trs``.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrs.so")
SOURCES = ["trs_host.cpp", "trs_kernels.hip", "trs_mlp.hip", "trs_membench.hip"]
ARCH = os.environ.get("TRS_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions are kept out of every HIP code object
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall",
               "-Wno-unused-function"]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + HIP_FLAGS
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
