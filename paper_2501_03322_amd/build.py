"""Build the HIP library libtwk.so for gfx950 in-tree.

hipcc compiles for the MI355X only (--offload-arch=gfx950).  Packed FP32
instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtwk.so")
SRC = [os.path.join(HERE, "csrc", "twk.hip")]
HEADERS = [os.path.join(HERE, "csrc", f)
           for f in ("twk_device.h", "twk_fs.h", "twk_mlp.h", "twk_gelu.h", "twk_queue.h")] + \
    [os.path.join(ROOT, "include", "twk.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-fno-gpu-rdc", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include")]


# The multi-core CPU backend (plain C++17 and threads; no HIP).
CPU_LIB = os.path.join(HERE, "libtwk_cpu.so")
CPU_SRC = os.path.join(HERE, "cpu", "twk_cpu.cpp")
CPU_FLAGS = ["-O3", "-std=c++17", "-march=x86-64-v2", "-fPIC", "-shared", "-pthread", "-Wall",
             "-Wextra", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, extra=None) -> str:
    cmd = [HIPCC] + FLAGS + (extra or []) + SRC + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_cpu(verbose)
    return LIB


def build_cpu(verbose: bool = False) -> str:
    cmd = ["g++"] + CPU_FLAGS + [CPU_SRC, "-o", CPU_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CPU_LIB + ".tmp", CPU_LIB)
    return CPU_LIB


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build(verbose=True, extra=extra))
