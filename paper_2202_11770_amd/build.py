"""Build libhlb.so (gfx950) in-tree.

The kernels (hlb_kernels.hip) are compiled by hipcc for gfx950 only; the host
runtime (hlb_runtime.cpp, OpenMP) by g++ against the HIP runtime headers; the
two are linked into ``paper_2202_11770_amd/libhlb.so`` next to this file.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhlb.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False, extra_hipcc=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    kobj = os.path.join(BUILD, "hlb_kernels.o")
    cobj = os.path.join(BUILD, "hlb_copy.o")
    robj = os.path.join(BUILD, "hlb_runtime.o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *extra_hipcc, *inc, "-c",
          os.path.join(CSRC, "hlb_kernels.hip"), "-o", kobj], verbose)
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *inc, "-c",
          os.path.join(CSRC, "hlb_copy.hip"), "-o", cobj], verbose)
    aobj = os.path.join(BUILD, "hlb_adjoint.o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *extra_hipcc, *inc, "-c",
          os.path.join(CSRC, "hlb_adjoint.hip"), "-o", aobj], verbose)
    xobj = os.path.join(BUILD, "hlb_aux.o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *inc, "-c",
          os.path.join(CSRC, "hlb_aux.hip"), "-o", xobj], verbose)
    hobj = os.path.join(BUILD, "hlb_halo.o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *inc, "-c",
          os.path.join(CSRC, "hlb_halo.hip"), "-o", hobj], verbose)
    nobj = os.path.join(BUILD, "hlb_noalloc.o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIPCC_FLAGS, *inc, "-c",
          os.path.join(CSRC, "hlb_noalloc.hip"), "-o", nobj], verbose)
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
          *inc, "-c", os.path.join(CSRC, "hlb_runtime.cpp"), "-o", robj], verbose)
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-fopenmp", kobj, cobj, aobj, xobj, hobj, nobj, robj, "-o", tmp, "-L", os.path.join(ROCM, "lib"),
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lamdhip64"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
