"""Compile the HIP library libghmi.so for gfx950 (in-tree, next to this file)."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libghmi.so")
SOURCES = ["csrc/ghmi_capi.hip", "csrc/ghmi_gemm.hip", "csrc/ghmi_kernels.hip", "csrc/ghmi_setup.cpp",
           "csrc/ghmi_tensor_filter.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (the path is FP64; this keeps any
    # incidental FP32 code on the scalar forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    """Compile every source (in parallel) and link libghmi.so; raises
    CalledProcessError on failure."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs, objs = [], []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + inc + ["-c", os.path.join(HERE, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, subprocess.Popen(cmd)))
    for cmd, p in jobs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + objs
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
