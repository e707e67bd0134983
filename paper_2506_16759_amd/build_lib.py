"""Builds libh2.so (HIP kernels for gfx950 + host planning + C ABI) in-tree.

    python -m paper_2506_16759_amd.build_lib

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file, where the Python binding loads it from.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libh2.so")

ARCH = "gfx950"
# Packed FP32 VALU forms are switched off for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-std=c++17", "-fPIC", "-O3", "-I", INCLUDE, "-I", CSRC]

SOURCES = [
    # (file, extra flags)
    ("h2_kernels.hip", [f"--offload-arch={ARCH}"] + DEVICE_FLAGS),
    ("h2_api.cpp", [f"--offload-arch={ARCH}", "-x", "hip"] + DEVICE_FLAGS),
    ("h2_batched.cpp", [f"--offload-arch={ARCH}", "-x", "hip"] + DEVICE_FLAGS),
    ("h2_update.cpp", [f"--offload-arch={ARCH}", "-x", "hip"] + DEVICE_FLAGS),
    ("h2_entries.cpp", [f"--offload-arch={ARCH}", "-x", "hip"] + DEVICE_FLAGS),
    # device planning: no contraction either (the admissibility test must
    # round like the host planner's)
    ("h2_plan_device.hip", [f"--offload-arch={ARCH}", "-ffp-contract=off"] + DEVICE_FLAGS),
    # host-only planning: no contraction, so box/admissibility arithmetic is
    # reproducible operation by operation
    ("h2_plan.cpp", ["-ffp-contract=off", "-fno-fast-math"]),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{err}")
    return err


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
