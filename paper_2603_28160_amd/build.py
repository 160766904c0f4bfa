"""Build libfsm.so (HIP for gfx950) in-tree.

    python -m paper_2603_28160_amd.build

Compiles the host planner with g++, the C ABI and the kernels with hipcc for gfx950, and
links paper_2603_28160_amd/libfsm.so.  Contraction into fused multiply-adds is off everywhere
(the double-precision path reproduces the plain definition bit for bit; the single-precision
kernels write their fused multiply-adds explicitly) and the compiler may not rewrite libm
calls in the planner.  Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfsm.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ... {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libfsm.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    o = os.path.join(BUILD, "fsm_plan.o")
    _run(["g++", *COMMON, "-pthread", "-fno-builtin", "-c", os.path.join(CSRC, "fsm_plan.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "fsm_sched.o")
    _run(["g++", *COMMON, "-c", os.path.join(CSRC, "fsm_sched.cpp"), "-o", o])
    objs.append(o)
    for name in ("fsm_api", "fsm_serve", "fsm_texture_api", "fsm_async"):
        o = os.path.join(BUILD, name + ".o")
        _run([HIPCC, *COMMON, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c",
              os.path.join(CSRC, name + ".cpp"), "-o", o])
        objs.append(o)
    for name in ("fsm_kernels", "fsm_texture", "fsm_noalloc"):
        o = os.path.join(BUILD, name + ".o")
        _run([HIPCC, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, name + ".hip"), "-o", o])
        objs.append(o)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
