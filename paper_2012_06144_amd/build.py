"""Compile the gfx950 HIP library ``liblbm.so`` (C ABI in include/lbm.h)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liblbm.so")
ARCH = "gfx950"

SOURCES = [os.path.join(CSRC, "lbm_api.hip"), os.path.join(CSRC, "sg_api.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("lbm_kernels.hpp", "lbm_lattice.hpp")] + [
    os.path.join(ROOT, "include", "lbm.h")]


def hipcc_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no contraction of a*b+c: the FP64 sweeps follow the rounding of the
        # formulas as written
        "-ffp-contract=off",
        # keep the compiler from forming packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + hipcc_flags() + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
