"""Build libqbw.so (HIP kernels for gfx950 + host C++) in-tree.

    python -m paper_2506_00976_amd.build        # or build() from Python

The library lands next to this file; object files go to _build/.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqbw.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# Packed FP32 instructions are kept out of the device code on purpose.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # the R = 32 c-transform tile is one fully unrolled block of ~1.7k
             # instructions; let the unroller go that far where asked to
             "-mllvm", "-pragma-unroll-threshold=200000",
             "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
             "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "is not a recognized feature for this target" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    cxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not os.path.exists(cxx):
        cxx = shutil.which("g++") or "g++"
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, *HIP_FLAGS, "-c", path, "-o", obj]
        elif src.endswith(".cpp"):
            cmd = [cxx, *CXX_FLAGS, "-c", path, "-o", obj]
        else:
            continue
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
