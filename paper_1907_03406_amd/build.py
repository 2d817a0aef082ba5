"""Builds libsgf.so (the HIP library behind include/sgf.h) for gfx950.

Run as ``python -m paper_1907_03406_amd.build``.  The shared library is
written next to this file so that it travels with the source tree.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsgf.so")
SOURCES = [os.path.join(HERE, "csrc", "sgf_lib.hip"), os.path.join(HERE, "csrc", "sgf_server.cpp")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("sgf_kernels.hpp", "sgf_plan.hpp", "sgf_tiled.hpp")] + \
    [os.path.join(ROOT, "include", "sgf.h")]


def hipcc_command(out=LIB, arch="gfx950", extra=()):
    return ["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-Wno-unused-result", *extra, "-o", out, *SOURCES]


def build(verbose=True):
    cmd = hipcc_command(out=LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
