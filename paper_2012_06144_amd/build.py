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

SOURCES = [os.path.join(CSRC, "lbm_api.hip"), os.path.join(CSRC, "lbm_sweeps_f32.hip"),
           os.path.join(CSRC, "sg_api.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("lbm_kernels.hpp", "lbm_lattice.hpp")] + [
    os.path.join(ROOT, "include", "lbm.h")]
# Per-source contraction of a*b+c into fused multiply-adds: off where FP64
# kernels follow the rounding of the formulas as written, on (within an
# expression) for the sweeps that compute in FP32.
CONTRACT = {"lbm_sweeps_f32.hip": "on"}


def hipcc_flags(contract: str = "off"):
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        f"-ffp-contract={contract}",
        # keep the compiler from forming packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src in SOURCES:
        obj = os.path.join(LIBDIR, os.path.basename(src) + ".o")
        cmd = ([hipcc] + hipcc_flags(CONTRACT.get(os.path.basename(src), "off")) + list(extra) +
               ["-c", "-o", obj, src])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
