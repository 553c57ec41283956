"""Compile the FP64 CPU oracle (oracle/fmo.c).

Test infrastructure only.  build(): oracle/libfmo.so for the tests, with
portable flags (no -march=native) so the library built here also runs on
other x86-64 hosts.  build_native(): a copy for the CPU timing of the
benchmark, -O3 -march=native, compiled on the host that runs it.  Both use
-ffp-contract=off, so every FP64 operation is a separately rounded IEEE
operation, and OpenMP, which only spreads loops of independent voxels over
threads (every sum stays sequential in natural order): all builds and thread
counts return the same bits.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fmo.c")
LIB = os.path.join(HERE, "libfmo.so")


def _compile(flags, out, verbose):
    cmd = ["gcc"] + flags + ["-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall",
                             "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def build(verbose=False):
    return _compile(["-O2"], LIB, verbose)


def build_native(out_dir, verbose=False):
    """-O3 -march=native copy in out_dir (for timing on the host it was built on)."""
    os.makedirs(out_dir, exist_ok=True)
    return _compile(["-O3", "-march=native"], os.path.join(out_dir, "libfmo_native.so"), verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
