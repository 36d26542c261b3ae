"""Compile the oracle (plain C, FP64) into oracle/liboracle.so.

Test infrastructure: built by the package build step so that the checker is
available, used only by tests, the smoke check and the CPU baseline.
Flags: -O2 without fast-math and with -ffp-contract=off, so every sum is
evaluated in the order written; OpenMP only splits independent control
volumes across threads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle2d.c", "oracle3d.c", "adjoint2d.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = f"{LIB}.tmp{os.getpid()}"      # one per process: parallel test workers may build at once
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in srcs):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
