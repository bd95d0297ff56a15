"""Build liblbe_csf.so (HIP for gfx950) in the package directory.

Usage: python -m paper_1412_6238_amd.build [-v]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbe_csf.so")
SOURCES = [os.path.join(CSRC, "lbe_csf.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("host_layout.h", "lattice.h", "step_kernel.h",
                                           "aux_kernels.h", "adjoint.h")]
HEADERS.append(os.path.join(ROOT, "include", "lbe_csf.h"))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def command(out: str = LIB, extra=()):
    return [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
            # keep the compiler from forming packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), *extra, "-o", out, *SOURCES]


def build(verbose: bool = False) -> str:
    cmd = command()
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[-1 - len(SOURCES)] = tmp
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.exists(f) and os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
