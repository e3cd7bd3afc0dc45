"""Build the C oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
SOURCES = [SRC, os.path.join(HERE, "march.c"), os.path.join(HERE, "shade.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    tmp = LIB + ".tmp%d" % os.getpid()
    # no floating-point contraction: the sampled march is defined one IEEE
    # single operation at a time
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared",
           "-pthread", "-Wall", "-Wextra", "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
