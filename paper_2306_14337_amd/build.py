"""Compile the HIP library (gfx950) in-tree, paper_2306_14337_amd/libkktlu.so,
and the hop-latency microbenchmark, paper_2306_14337_amd/hop_latency."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkktlu.so")
SOURCES = ["analyze.cpp", "kernels.hip", "runtime.hip"]
HOP = os.path.join(PKG, "hop_latency")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # bitwise-reproducible host analysis and refactorization: explicit fma only
    "-ffp-contract=off",
    "-Xarch_host", "-mfma",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libkktlu.so")
    os.replace(tmp, LIB)
    # the hop-latency microbenchmark (an executable; bench.py runs it)
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    tmp = HOP + ".tmp"
    cmd = [hipcc, *flags, os.path.join(CSRC, "hop_latency.hip"), "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build hop_latency")
    os.replace(tmp, HOP)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
