"""Compile libgsdp.so in-tree for gfx950 with hipcc.

Flags that the exactness of the path depends on:
  -ffp-contract=off                          no FMA contraction of a*b+c
  -fhip-fp32-correctly-rounded-divide-sqrt   IEEE division and square root
  -fno-gpu-flush-denormals-to-zero           FP32 denormals preserved
  -Xclang -target-feature -Xclang -packed-fp32-ops   no packed FP32 instructions
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libgsdp.so")
SOURCES = [os.path.join(PKG, "csrc", "gsdp.hip"), os.path.join(PKG, "csrc", "gsdp_lut.cpp")]
HEADERS = [os.path.join(ROOT, "include", "gsdp.h"), os.path.join(PKG, "csrc", "gsdp_internal.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument", "-Wno-pass-failed",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always when force, else only when sources changed)."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
