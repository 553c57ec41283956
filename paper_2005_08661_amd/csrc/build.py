"""Build libfmap.so (the C ABI of include/fmap.h) for gfx950 with hipcc.

Packed FP32 instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libfmap.so")
SOURCES = [os.path.join(HERE, "fm_api.hip")]
ARCH = os.environ.get("FMAP_OFFLOAD_ARCH", "gfx950")


def build(verbose=False, out=None, defines=()):
    lib = out or LIB
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include")] + ["-D" + d for d in defines] + \
          ["-o", lib + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
