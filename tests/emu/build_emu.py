"""Build the CPU emulation of the device engine (test infrastructure):
the unmodified device code of paper_2501_03322_amd/csrc compiled by g++
against tests/emu/include/hip/hip_runtime.h."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libengine_emu.so")


def build(kgap=None, lcap=None) -> str:
    """kgap: override of the residual detector's gap factor (a blinded
    detector exercises the slope detector); lcap: LDS capacity of the
    emulated engine (default 512)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    name = "libengine_emu" + ("" if kgap is None else f"_kgap{kgap:g}") + \
        ("" if lcap is None else f"_lcap{lcap}") + ".so"
    lib = os.path.join(OUT_DIR, name)
    defs = ([] if kgap is None else [f"-DTWK_KGAP={kgap!r}"]) + \
        ([] if lcap is None else [f"-DEMU_LCAP={int(lcap)}"])
    cmd = ["g++", "-std=c++20", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-I", os.path.join(HERE, "include")] + defs + ["-o", lib + ".tmp",
                                                        os.path.join(HERE, "engine_emu.cpp")]
    tmp = f"{lib}.tmp{os.getpid()}"
    cmd[cmd.index(lib + ".tmp")] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
