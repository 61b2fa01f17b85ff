"""Build step for the CPU oracle (test infrastructure only).

Compiles ``mgmc_oracle.c`` with gcc into ``liboracle.so`` beside this file.
Floating-point contraction is disabled so that every product and sum is
rounded exactly as written in the C source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "mgmc_oracle.c")
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
        "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
        "-o", LIB + ".tmp", src, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
