"""Builds libfcsdnn.so in-tree: the HIP kernels and C ABI for gfx950 (hipcc)
and the binary128 host precomputation (g++)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfcsdnn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             # no packed FP32 instructions: plain FP32 code only
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # matrix-core products keep their accumulators in ordinary
             # vector registers (no accumulator-register reads in the network)
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-I", os.path.join(ROOT, "include")]


def run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    o1 = os.path.join(BUILD, "fcmat.o")
    o2 = os.path.join(BUILD, "fcsdnn.o")
    run(["g++", "-O2", "-fPIC", "-std=gnu++17", "-c", os.path.join(CSRC, "fcmat.cpp"), "-o", o1])
    run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "fcsdnn.hip"), "-o", o2])
    tmp = LIB + ".tmp"
    run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", o2, o1, "-o", tmp, "-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
