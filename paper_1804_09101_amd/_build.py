"""Compile the HIP library libghmi.so for gfx950 (in-tree, next to this file)."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libghmi.so")
SOURCES = ["csrc/ghmi_capi.hip", "csrc/ghmi_kernels.hip", "csrc/ghmi_setup.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (the path is FP64; this keeps any
    # incidental FP32 code on the scalar forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    """Compile every source into libghmi.so; raises CalledProcessError on failure."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
                             "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_test_harness(verbose=False):
    """Host build of the device pointwise code for the CPU tests (tests/native)."""
    src = os.path.join(ROOT, "tests", "native", "ghpoint_host.cpp")
    out = os.path.join(ROOT, "tests", "native", "libghpoint_host.so")
    if not os.path.exists(src):
        return None
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-shared", "-fPIC",
           "-I", os.path.join(HERE, "csrc"), "-o", out, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_test_harness(verbose=True))
