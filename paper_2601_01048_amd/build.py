"""Builds libckc.so in-tree with hipcc for gfx950.

Usage: python -m paper_2601_01048_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libckc.so")
BUILD = os.path.join(HERE, "_build")

ARCH = os.environ.get("CKC_OFFLOAD_ARCH", "gfx950")
# packed fp32 instructions stay disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link libckc.so."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, device in (("kernels.hip", True), ("loader.cpp", False), ("runtime.cpp", False),
                        ("server.cpp", False), ("fuzz.cpp", False)):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        if device:
            cmd += [f"--offload-arch={ARCH}"] + DEVICE_FLAGS
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
