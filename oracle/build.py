"""Compile the FP64 CPU oracle (oracle/fmo.c) into oracle/libfmo.so.

Test infrastructure only.  Portable flags (no -march=native) so the library
built here also runs on other x86-64 hosts; -ffp-contract=off keeps every
FP64 operation a separately rounded IEEE operation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fmo.c")
LIB = os.path.join(HERE, "libfmo.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
