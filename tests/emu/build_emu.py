"""Build the CPU emulation of the device engine (test infrastructure):
the unmodified device code of paper_2501_03322_amd/csrc compiled by g++
against tests/emu/include/hip/hip_runtime.h."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libengine_emu.so")


def build() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    cmd = ["g++", "-std=c++20", "-O2", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
           "-I", os.path.join(HERE, "include"), "-o", LIB + ".tmp",
           os.path.join(HERE, "engine_emu.cpp")]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
