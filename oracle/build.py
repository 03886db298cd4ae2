"""Build the CPU FP64 oracle (test infrastructure) as oracle/liboracle.so.

Plain C99, FP64, -O3, no fast-math, no FMA contraction, OpenMP over cells.

The default library is built for the baseline x86-64 instruction set, so a
copy built on one host loads on any other.  `native=True` builds a second
copy, liboracle_native.so, with -march=native for the host it is built on:
the timing copy (same arithmetic: contraction stays off and no reassociation
is allowed, so vector code changes no result).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_tissue.c", "orc_tp06.c", "orc_crn.c", "orc_stewart.c"]
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")
FLAGS = ["-std=c99", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", "-D_DEFAULT_SOURCE"]


def flags(native: bool = False):
    return FLAGS + (["-march=native"] if native else [])


def build(verbose: bool = False, native: bool = False) -> str:
    out = LIB_NATIVE if native else LIB
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc"] + flags(native) + ["-o", tmp]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, native="--native" in sys.argv)
