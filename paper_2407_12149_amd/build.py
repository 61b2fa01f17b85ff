"""Build step of the HIP library libmgmc.so (gfx950), in-tree."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmgmc.so")
SOURCES = ["csrc/api.hip", "csrc/kernels.hip", "csrc/kernels_tiled.hip", "csrc/hierarchy.cpp",
           "csrc/api_pnet.hip", "csrc/kernels_pnet.hip", "csrc/kernels_coarse.hip",
           "csrc/kernels_ext.hip"]


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    cmd = [
        hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
        # never let the compiler emit packed FP32 arithmetic
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
        "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
        "-o", LIB + ".tmp",
    ] + [os.path.join(HERE, s) for s in SOURCES] + ["-lpthread", "-Wl,-z,defs"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
