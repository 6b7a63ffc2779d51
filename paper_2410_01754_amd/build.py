"""Build libmahi.so in-tree with hipcc for gfx950.

Usage: python -m paper_2410_01754_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmahi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed float32 VALU instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                # matrix-core accumulators in architectural VGPRs (no AGPR copies around each MFMA)
                "-mllvm", "-amdgpu-mfma-vgpr-form=true"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src, dev in (("kernels.hip", True), ("m2l_f32.hip", True), ("capi.cpp", True), ("tables.cpp", False)):
        obj = os.path.join(bdir, src + ".o")
        cmd = [HIPCC] + COMMON + (DEVICE_FLAGS if dev else ["-x", "c++"]) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if dev and src.endswith(".cpp"):
            cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
