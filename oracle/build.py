"""Compile the CPU oracle (test infrastructure) into oracle/libraptor_oracle.so with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "raptor_oracle.c")
LIB = os.path.join(HERE, "libraptor_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
