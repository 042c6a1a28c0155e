"""Build libsaq.so in-tree: host C++ (g++, OpenMP) + device HIP (hipcc,
gfx950), linked into one shared library next to this file."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libsaq.so")
ARCH = os.environ.get("SAQ_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions stay disabled in every HIP object.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-ffp-contract=off"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    host_o = os.path.join(BUILD, "host.o")
    dev_o = os.path.join(BUILD, "device.o")
    fit_o = os.path.join(BUILD, "fit.o")
    _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "host.cpp"), "-o", host_o])
    _run([hipcc(), *HIP_FLAGS, "-c", os.path.join(CSRC, "device.hip"), "-o", dev_o])
    _run([hipcc(), *HIP_FLAGS, "-c", os.path.join(CSRC, "fit.hip"), "-o", fit_o])
    tmp = LIB + ".tmp"
    _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", host_o, dev_o, fit_o, "-o", tmp,
          "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
