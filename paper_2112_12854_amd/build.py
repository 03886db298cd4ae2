"""Compile the HIP library libep.so for gfx950 (in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libep.so")
SOURCES = ["ep_api.hip", "instance.hip", "serve.hip", "bidomain.hip", "diffusion.hip", "prep.cpp", "purkinje.cpp",
           "coarse.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-fast-math", "-ffp-contract=fast", "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         "-Wall", "-Wno-unused-function",
         "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC] + FLAGS + list(extra) + [os.path.join(CSRC, s) for s in SOURCES] + \
        ["-lpthread", "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=[a for a in sys.argv[1:] if a != "-v"])
