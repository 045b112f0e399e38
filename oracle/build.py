"""Build the FP64 CPU oracle (test infrastructure) into oracle/libtwk_ref.so.

Plain gcc, no fused multiply-add contraction, no fast-math: the oracle's
arithmetic must be exactly what its source says.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtwk_ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "twk_ref.c")
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fcx-fortran-rules", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
