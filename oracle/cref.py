"""ctypes wrapper of the plain C oracle (oracle/kb_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU-baseline leg use
it; the HIP library never does.  The C code computes what oracle/core.py
computes, in the same order of IEEE double operations, one start pixel and
one trajectory at a time, so its results equal the numpy oracle's bit for
bit (tests/test_oracle_c.py checks that, and the pins of the numpy oracle).
It exists because full-frame comparisons (16.8M start pixels x 600
velocities) are out of reach of the vectorised numpy code in test time.

build() compiles libkb_oracle.so next to the source with gcc
(-ffp-contract=off: products and sums stay separately rounded).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kb_oracle.c")
LIB = os.path.join(HERE, "libkb_oracle.so")
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall"]

_lock = threading.Lock()
_lib = None
_p, _i64 = ctypes.c_void_p, ctypes.c_int64


def build(out: str = LIB, defines=()) -> str:
    """Compile the C oracle into `out` (extra -D `defines` for mutation tests)."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *[f"-D{d}" for d in defines], "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C oracle build failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def _bind(lib):
    lib.orc_planes.restype = None
    lib.orc_planes.argtypes = [_p, _p, _p, _i64, _i64, _i64, _p, _i64, _i64, _i64, _i64, _i64,
                               _i64, _p, _p, _p]
    lib.orc_search_rows.restype = ctypes.c_int
    lib.orc_search_rows.argtypes = [_p, _p, _p, _i64, _i64, _i64, _i64, _i64, _p, _p, _i64,
                                    _i64, _i64, _i64, _p, _p, _p, _p, _p]
    return lib


def load(path: str | None = None):
    """The C oracle library (built here first if it is missing)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def planes(img, var, mask, psf, images=None, rows=None, lib=None):
    """psi, phi (float64) and validity (bool) of images [i0, i1) at frame rows
    [r0, r1): arrays [i1 - i0][r1 - r0][W] (Sec. 2.1.5 Psi and Phi equations)."""
    L = lib or load()
    img = _c(img, np.float32)
    var = _c(var, np.float32)
    n, h, w = img.shape
    m = None if mask is None else _c(mask, np.uint8)
    psf = _c(psf, np.float32)
    i0, i1 = (0, n) if images is None else images
    r0, r1 = (0, h) if rows is None else rows
    psi = np.empty((i1 - i0, r1 - r0, w), dtype=np.float64)
    phi = np.empty_like(psi)
    ok = np.empty(psi.shape, dtype=np.uint8)
    L.orc_planes(img.ctypes.data, var.ctypes.data, None if m is None else m.ctypes.data, n, h, w,
                 psf.ctypes.data, psf.shape[0], psf.shape[1], i0, i1, r0, r1, psi.ctypes.data,
                 phi.ctypes.data, ok.ctypes.data)
    return psi, phi, ok.astype(bool)


def search_rows(psi, phi, ok, h, t, vel, k_out, row_lo, row_hi, plane_row0=0, lib=None):
    """The best k_out trajectories (nu desc, index asc) of start rows
    [row_lo, row_hi) from planes [N][R][W] holding frame rows
    [plane_row0, plane_row0 + R): dict of nu, alpha, Phi (float64), nobs,
    vel (int32), each [row_hi - row_lo][W][k_out]."""
    L = lib or load()
    psi = _c(psi, np.float64)
    phi = _c(phi, np.float64)
    okb = _c(ok, np.uint8)
    n, pr, w = psi.shape
    t = _c(t, np.float64)
    vel = _c(vel, np.float64).reshape(-1, 2)
    nv = vel.shape[0]
    k_out = min(int(k_out), nv)
    shape = (row_hi - row_lo, w, k_out)
    out = dict(nu=np.empty(shape), alpha=np.empty(shape), Phi=np.empty(shape),
               nobs=np.empty(shape, dtype=np.int32), vel=np.empty(shape, dtype=np.int32))
    rc = L.orc_search_rows(psi.ctypes.data, phi.ctypes.data, okb.ctypes.data, n, h, w,
                           plane_row0, pr, t.ctypes.data, vel.ctypes.data, nv, k_out, row_lo,
                           row_hi, out["nu"].ctypes.data, out["alpha"].ctypes.data,
                           out["Phi"].ctypes.data, out["nobs"].ctypes.data,
                           out["vel"].ctypes.data)
    if rc == -2:
        raise MemoryError("C oracle: out of memory")
    if rc != 0:
        raise ValueError("a trajectory leaves the plane rows given")
    return out


def search(img, var, mask, t, psf, vel, k, lib=None):
    """Whole-frame search: ranked best k per start pixel, arrays [H][W][k]."""
    psi, phi, ok = planes(img, var, mask, psf, lib=lib)
    h = psi.shape[1]
    return search_rows(psi, phi, ok, h, t, vel, k, 0, h, lib=lib)
