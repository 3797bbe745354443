"""Whole-frame or row-block runs of the C oracle (oracle/kb_oracle.c) in worker
processes: TEST INFRASTRUCTURE ONLY (the full-frame parity test and the
benchmark's CPU-baseline leg).

The planes of the rows the trajectories visit are computed once, one
(image, row chunk) per task, into memory shared by the workers; then each
task searches one band of start rows against those planes.  Workers are
forked, so a caller's arrays that exist before run_bands() is called (the
stack, results to compare with) are visible to them without copies.
"""
from __future__ import annotations

import math
import mmap
import multiprocessing as mp
import time

import numpy as np

from . import cref
from .core import displacements

_STATE: dict = {}


def shared_array(shape, dtype):
    """A zero-filled array in anonymous memory shared with forked children."""
    nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
    buf = mmap.mmap(-1, max(nbytes, 1))
    return np.frombuffer(buf, dtype=dtype, count=int(np.prod(shape))).reshape(shape)


def _planes_task(arg):
    i, r0, r1 = arg
    st = _STATE
    psi, phi, ok = cref.planes(st["img"], st["var"], st["mask"], st["psf"], images=(i, i + 1),
                               rows=(r0, r1))
    p0 = st["plane_row0"]
    st["psi"][i, r0 - p0:r1 - p0] = psi[0]
    st["phi"][i, r0 - p0:r1 - p0] = phi[0]
    st["ok"][i, r0 - p0:r1 - p0] = ok[0]
    return None


def _band_task(arg):
    r0, r1 = arg
    st = _STATE
    t0 = time.perf_counter()
    res = cref.search_rows(st["psi"], st["phi"], st["ok"], st["h"], st["t"], st["vel"],
                           st["k_out"], r0, r1, plane_row0=st["plane_row0"])
    dt = time.perf_counter() - t0
    if st["on_band"] is not None:
        return st["on_band"](r0, r1, res), dt
    out = st["out"]
    for key in out:
        out[key][r0 - st["row_lo"]:r1 - st["row_lo"]] = res[key]
    return None, dt


def run_bands(img, var, mask, psf, t, vel, k_out, row_lo, row_hi, band_rows=16, workers=15,
              on_band=None):
    """The C oracle's best k_out trajectories of start rows [row_lo, row_hi).

    With on_band=None returns (arrays, timing): arrays nu, alpha, Phi, nobs,
    vel [row_hi - row_lo][W][k_out] in shared memory.  Otherwise each worker
    calls on_band(r0, r1, band_result) for its band and the list of those
    return values comes back instead of the arrays.  timing holds the wall
    seconds of the plane and the search phases."""
    n, h, w = img.shape
    dy = displacements(t, vel)[:, :, 1]
    need_lo = max(0, row_lo + int(dy.min()))
    need_hi = min(h, row_hi + int(dy.max()))
    rows = need_hi - need_lo
    st = _STATE
    st.clear()
    st.update(img=img, var=var, mask=mask, psf=psf, t=np.asarray(t, dtype=np.float64),
              vel=np.asarray(vel, dtype=np.float64).reshape(-1, 2), h=h, k_out=k_out,
              plane_row0=need_lo, row_lo=row_lo, on_band=on_band,
              psi=shared_array((n, rows, w), np.float64),
              phi=shared_array((n, rows, w), np.float64),
              ok=shared_array((n, rows, w), np.uint8))
    kk = min(int(k_out), st["vel"].shape[0])
    if on_band is None:
        shp = (row_hi - row_lo, w, kk)
        st["out"] = dict(nu=shared_array(shp, np.float64), alpha=shared_array(shp, np.float64),
                         Phi=shared_array(shp, np.float64), nobs=shared_array(shp, np.int32),
                         vel=shared_array(shp, np.int32))
    cref.load()                      # loaded once, inherited by the workers
    chunk = max(16, math.ceil(rows / (4 * workers)))
    plane_tasks = [(i, r, min(r + chunk, need_hi)) for i in range(n)
                   for r in range(need_lo, need_hi, chunk)]
    band_tasks = [(r, min(r + band_rows, row_hi)) for r in range(row_lo, row_hi, band_rows)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_planes_task, plane_tasks, chunksize=1)
        t1 = time.perf_counter()
        got = pool.map(_band_task, band_tasks, chunksize=1)
        t2 = time.perf_counter()
    timing = dict(planes_s=t1 - t0, search_s=t2 - t1, plane_rows=rows,
                  band_s=[dt for _, dt in got])
    result = [r for r, _ in got] if on_band is not None else st["out"]
    st.clear()
    return result, timing
