"""Build the HIP library libquadswarm.so for gfx950 (in-tree).

Run as ``python -m paper_2306_09537_amd.build``; ``__graft_entry__.build()``
calls :func:`build`.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libquadswarm.so")
SOURCES = [os.path.join(CSRC, "qs_abi.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("qs_device.h", "qs_kernels.h", "qs_adjoint.h",
                                                  "qs_rollout.h", "qs_checks.h")] + [
    os.path.join(INCLUDE, "quadswarm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds fuse only within one source expression, so every kernel
    # specialisation (and the adjoint's recomputation) rounds identically
    "-ffp-contract=on",
    # no packed-FP32 instructions: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # leading kernel arguments arrive in SGPRs instead of through a scalar
    # load of the argument segment (a fallback prologue loads them where the
    # firmware does not preload)
    "-mllvm", "-amdgpu-kernarg-preload-count=16",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
