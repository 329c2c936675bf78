"""Builds libnttmi.so (the C-ABI library with the gfx950 kernels) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnttmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("NTTMI_ARCH", "gfx950")

HIP_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    names = sorted(f for f in os.listdir(CSRC) if f.startswith("launch_") and f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in names] + [os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "server.cpp")]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libnttmi.so (always recompiles)."""
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = []
    for src in sources():
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((subprocess.Popen(cmd), cmd, obj))
    objs = []
    failed = []
    for proc, cmd, obj in jobs:
        if proc.wait() != 0:
            failed.append(" ".join(cmd))
        objs.append(obj)
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


BENCH_SRC = os.path.join(HERE, "bench_csrc", "peak.hip")
BENCH_LIB = os.path.join(HERE, "libnttbench.so")


def build_bench(verbose: bool = False) -> str:
    """Compile the measurement helpers bench.py uses (vector-ALU peak rates)
    into libnttbench.so (not part of the convolution library)."""
    tmp = BENCH_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + HIP_FLAGS + ["-shared", "-x", "hip", BENCH_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, BENCH_LIB)
    return BENCH_LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_bench(verbose="-v" in sys.argv)
    print(LIB)
