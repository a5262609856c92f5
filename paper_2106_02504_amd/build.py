"""Build librlx.so (HIP for gfx950) in place next to this file.

    python -m paper_2106_02504_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("rlx.hip", "rlx_batch.hip", "rlx_engine_test.hip", "rlx_rates.hip")]
LIB = os.path.join(HERE, "librlx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of all code built here
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


CPU_SRC = os.path.join(HERE, "cpu", "rlx_cpu.cpp")
CPU_LIB = os.path.join(HERE, "cpu", "librlx_cpu.so")
CXX = os.environ.get("CXX", "g++")


def build_cpu(verbose: bool = False) -> str:
    """Compile the CPU baseline (librlx_cpu.so, host C++) and return its path."""
    tmp = CPU_LIB + ".tmp"
    cmd = [CXX, "-O3", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, CPU_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building librlx_cpu.so failed")
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False, extra=()) -> str:
    """Compile librlx.so (and the CPU baseline) unconditionally and return
    the path of librlx.so."""
    build_cpu(verbose)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building librlx.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
