"""Build the FP64 CPU oracle (test infrastructure only) into oracle/liboracle.so.

Compiled with -O2 -ffp-contract=off and no fast-math so that every
floating-point operation is the one written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["kerr.c", "trace.c", "camera.c", "plasma.c", "transfer.c", "render.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-D_DEFAULT_SOURCE",
           "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-variable",
           "-fPIC", "-shared", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
