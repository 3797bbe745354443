"""Compile libkbmi.so in-tree for gfx950 with hipcc.

    python -m paper_1901_02492_amd.build [-v]

The host helpers are built with -ffp-contract=off so the displacement table's
multiply, add and floor stay separately rounded.  All device code is built
with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libkbmi.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", INCLUDE, "-I", CSRC, "-Wall"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", INCLUDE, "-I", CSRC,
              "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)


def build_library(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source and link libkbmi.so (next to this file unless `out`
    is given); `defines` are extra -D options.  Returns the library path."""
    dflags = [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="kbmi_build_") as tmp:
        objs = []
        host_obj = os.path.join(tmp, "kbmi_host.o")
        _run(["g++", *HOST_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_host.cpp"), "-o", host_obj],
             verbose)
        objs.append(host_obj)
        dev_obj = os.path.join(tmp, "kbmi_kernels.o")
        _run([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_kernels.hip"), "-o", dev_obj],
             verbose)
        objs.append(dev_obj)
        tmp_lib = out + ".tmp"
        _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp_lib, *objs], verbose)
        os.replace(tmp_lib, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
