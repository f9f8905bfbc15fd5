"""Build libmadflow_mi355x.so for gfx950 with hipcc (in-tree).

The amplitude code is generated first (csrc/gen_amplitudes.py -> csrc/_gen/),
then the whole library is one hipcc invocation.  Packed-FP32 instructions
are disabled for the whole target.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libmadflow_mi355x.so")
ARCH = os.environ.get("MF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def generate():
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_amplitudes.py"), "--out",
                    os.path.join(CSRC, "_gen")], check=True)


def build(extra_flags=None, out=LIB, verbose=False):
    generate()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = [hipcc(), *HIPCC_FLAGS, *(extra_flags or []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "mf_lib.hip"), "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
