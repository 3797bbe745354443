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
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libkbmi.so")
PEAK_LIB = os.path.join(PKG, "libkbmi_peak.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KM_GROUPS = 8   # list-length groups of the search units (kKmGroups in kbmi_device.h)

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


def build_library(verbose: bool = False, out: str = LIB, defines=(), jobs: int = 0) -> str:
    """Compile every source and link libkbmi.so (next to this file unless `out`
    is given); `defines` are extra -D options.  The search kernels are compiled
    once per plane format and list-length group, all objects in parallel.
    Returns the library path."""
    dflags = [f"-D{d}" for d in defines]
    jobs = jobs or min(16, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="kbmi_build_") as tmp:
        steps = [(["g++", *HOST_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_host.cpp"), "-o",
                   os.path.join(tmp, "kbmi_host.o")], os.path.join(tmp, "kbmi_host.o")),
                 ([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_kernels.hip"),
                   "-o", os.path.join(tmp, "kbmi_kernels.o")], os.path.join(tmp, "kbmi_kernels.o")),
                 ([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_filter.hip"),
                   "-o", os.path.join(tmp, "kbmi_filter.o")], os.path.join(tmp, "kbmi_filter.o")),
                 ([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_threshold.hip"),
                   "-o", os.path.join(tmp, "kbmi_threshold.o")],
                  os.path.join(tmp, "kbmi_threshold.o")),
                 ([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_stamps.hip"),
                   "-o", os.path.join(tmp, "kbmi_stamps.o")], os.path.join(tmp, "kbmi_stamps.o")),
                 ([HIPCC, *DEVICE_FLAGS, *dflags, "-c", os.path.join(CSRC, "kbmi_noalloc.hip"),
                   "-o", os.path.join(tmp, "kbmi_noalloc.o")],
                  os.path.join(tmp, "kbmi_noalloc.o"))]
        # The search kernels: one unit per (plane format, list-length group).
        search = []
        for fmt in (0, 1, 2):
            for grp in range(KM_GROUPS):
                obj = os.path.join(tmp, f"kbmi_search_{fmt}_{grp}.o")
                search.append(([HIPCC, *DEVICE_FLAGS, *dflags, f"-DKBMI_FMT={fmt}",
                                f"-DKBMI_GROUP={grp}", "-c",
                                os.path.join(CSRC, "kbmi_search.hip"), "-o", obj], obj))
        # Longest units first, so the pool ends together.
        steps = search + steps
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            list(pool.map(lambda st: _run(st[0], verbose), steps))
        tmp_lib = out + ".tmp"
        _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp_lib,
              *[o for _, o in steps]], verbose)
        os.replace(tmp_lib, out)
    return out


def build_peak_library(verbose: bool = False, out: str = PEAK_LIB) -> str:
    """Compile the measurement helper libkbmi_peak.so (the gather-pattern peak
    the benchmark sets the search kernel against; not part of libkbmi)."""
    tmp_lib = out + ".tmp"
    _run([HIPCC, *DEVICE_FLAGS, "-shared", "-o", tmp_lib, os.path.join(CSRC, "kbmi_peak.hip")],
         verbose)
    os.replace(tmp_lib, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
    print(build_peak_library(verbose="-v" in sys.argv))
