"""Build the CPU oracle library (test infrastructure, not product code).

Compiles ljref.c with gcc into libljref.so next to this file.  The flags keep
the arithmetic plain: -ffp-contract=off so that only the explicit fma() calls
fuse, and no fast-math.  build_timing() compiles the same source a second time
with -O3 -march=native into libljref_timing.so, which is only used to time the
oracle on the host (never for a parity check).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ljref.c")
LIB = os.path.join(HERE, "libljref.so")
TIMING_LIB = os.path.join(HERE, "libljref_timing.so")
TIMING_FLAGS = ["-std=gnu99", "-O3", "-march=native", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_timing() -> str:
    cmd = ["gcc", *TIMING_FLAGS, "-o", TIMING_LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(TIMING_LIB + ".tmp", TIMING_LIB)
    return TIMING_LIB


if __name__ == "__main__":
    print(build())
    print(build_timing())
