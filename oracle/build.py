"""Compile the CPU oracle (test infrastructure) into oracle/libraptor_oracle.so with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "raptor_oracle.c")
LIB = os.path.join(HERE, "libraptor_oracle.so")


def build(verbose=False):
    # a temporary name of this process's own, so that concurrent builds (parallel test workers)
    # each replace the library atomically
    tmp = f"{LIB}.tmp{os.getpid()}"
    cmd = ["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
