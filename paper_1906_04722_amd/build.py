"""Build the HIP library libsc_lbm.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsc_lbm.so")
CLI = os.path.join(PKG, "lbm_drain")
SOURCES = ["sc_kernels.hip", "sg_kernels.hip", "lbm_abi.cpp", "lbm_batch.cpp", "surrogate.cpp",
           "network.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose=False):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-parameter",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp"] + ["-x", "hip"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    build_cli(verbose)
    return LIB


def build_cli(verbose=False):
    """The command-line drain (csrc/lbm_drain_cli.c): plain C against
    include/lbm_abi.h, linked to the library next to it."""
    cmd = [os.environ.get("CC", "gcc"), "-O2", "-std=c99", "-Wall", "-Wextra",
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "lbm_drain_cli.c"),
           "-L", PKG, "-lsc_lbm", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath-link,/opt/rocm/lib",
           "-o", CLI + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(CLI + ".tmp", CLI)
    return CLI


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
