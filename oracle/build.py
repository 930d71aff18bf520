"""Build the CPU oracle library (test infrastructure; see oracle.cpp's header)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("oracle.cpp", "ssim.cpp", "expand.cpp")]
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = ["-std=c++17", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    cmd = ["g++", *FLAGS, *SRCS, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SRCS):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
