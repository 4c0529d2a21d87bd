"""Build libcktlu.so in-tree with hipcc for gfx950 (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcktlu.so")

HOST_SOURCES = ["cktlu.cpp", "analyze.cpp", "factor_host.cpp", "schedule.cpp", "server.cpp"]
DEVICE_SOURCES = ["kernels.hip", "dense.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# device code: gfx950 only; packed FP32 instructions disabled
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: %s" % cmd[-1])


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        _run([HIPCC, "-c", *COMMON, *DEVICE_FLAGS, "-o", obj, os.path.join(CSRC, src)])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        _run([HIPCC, "-c", "-x", "c++", *COMMON, "-pthread", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-o", obj,
              os.path.join(CSRC, src)])
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-pthread", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
