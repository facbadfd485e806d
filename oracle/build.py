"""Build step for the FP64 CPU oracle (test infrastructure only).

Compiles ``spmm_oracle.c`` with gcc into ``liboracle.so`` beside it. The
flags keep the arithmetic plain: no fused multiply-add contraction and no
fast-math, generic x86-64 code so the library runs on any host it is copied to.
``build_native`` makes the CPU baseline's -O3 -march=native build on the host
that times it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_native(path: str, verbose: bool = False) -> str:
    """The CPU baseline's build of the same source: -O3 for the host it runs
    on (-march=native), still without contraction or fast-math, so every sum
    is the same sequence of double additions and results are bitwise those
    of the test build. Built where it runs: the host CPU decides the
    instruction set."""
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", SRC, "-o", path + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


if __name__ == "__main__":
    print(build(verbose=True))
