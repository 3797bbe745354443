"""FP64 CPU oracle of coadded postage stamps and the central-moment filter
(test infrastructure only).

Nothing in the product path imports, calls or links this module: only the
tests, the package smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library.

What is computed (Sec. 3.3, second paragraph: coadded postage stamps of the
remaining candidates, whose central moments are compared with those of a
Gaussian centred on the stamp).  The paper gives neither the coadd nor the
comparison, so this is a reading of that passage:

  1. Stamp.  For candidate (x0, y0, j) and each kept image i (valid, and not
     dropped by the light-curve filter when its mask is given), the science
     image is cut out around the trajectory pixel (x_i, y_i) (Sec. 2.2
     displacements) for offsets u, v in [-R, R].  The coadded stamp is the
     mean over the kept images of the pixels that are inside the frame and
     valid (Sec. 2.1.5 validity):
         S(u, v) = (sum_i img_i(x_i + u, y_i + v)) / n(u, v),
     summed in increasing image order in IEEE double; S = 0 where n = 0.
  2. Moments.  One pass over the stamp in row-major order (v outer, u
     inner), with the offsets as weights:
         M00 = sum S,  M10 = sum u S,  M01 = sum v S,
         M20 = sum u*u S,  M02 = sum v*v S,  M11 = sum u*v S,
     then the centroid ub = M10/M00, vb = M01/M00 and the central moments
     per unit flux m20 = M20/M00 - ub*ub, m02 = M02/M00 - vb*vb,
     m11 = M11/M00 - ub*vb (each operation separately rounded).
  3. Filter.  A centred Gaussian has ub = vb = 0, m11 = 0 and m20 = m02 =
     its variance.  A stamp passes when M00 > 0, |ub| <= max_offset,
     |vb| <= max_offset, |m11| <= max_m11, and m2_min <= m20, m02 <= m2_max.
"""
from __future__ import annotations

import numpy as np

from .core import displacements, validity

__all__ = ["coadd_stamps", "moments", "stamp_filter"]


def coadd_stamps(img, var, mask, t, vel, xs, ys, js, R, keep=None):
    """Mean stamps float64 [C][2R+1][2R+1] (step 1).  keep: optional bool
    [C][N] of the images each candidate may use (default: all)."""
    img = np.asarray(img, dtype=np.float32)
    ok = validity(img, var, mask)
    n, h, w = img.shape
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    disp = displacements(t, vel)
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    js = np.asarray(js, dtype=np.int64)
    c = xs.size
    off = np.arange(-R, R + 1)
    acc = np.zeros((c, 2 * R + 1, 2 * R + 1))
    cnt = np.zeros((c, 2 * R + 1, 2 * R + 1), dtype=np.int64)
    for i in range(n):
        use = np.ones(c, dtype=bool) if keep is None else np.asarray(keep)[:, i]
        yy = ys[:, None, None] + disp[js, i, 1][:, None, None] + off[None, :, None]
        xx = xs[:, None, None] + disp[js, i, 0][:, None, None] + off[None, None, :]
        inb = use[:, None, None] & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
        yc, xc = np.clip(yy, 0, h - 1), np.clip(xx, 0, w - 1)
        good = inb & ok[i][yc, xc]
        vals = img[i][yc, xc].astype(np.float64)
        acc = np.where(good, acc + vals, acc)
        cnt = cnt + good
    return np.where(cnt > 0, acc / np.maximum(cnt, 1), 0.0)


def moments(S):
    """(M00, ub, vb, m20, m02, m11) of stamps S [C][2R+1][2R+1] (step 2)."""
    c, side, _ = S.shape
    R = side // 2
    M00 = np.zeros(c)
    M10 = np.zeros(c)
    M01 = np.zeros(c)
    M20 = np.zeros(c)
    M02 = np.zeros(c)
    M11 = np.zeros(c)
    for a in range(side):
        v = float(a - R)
        for b in range(side):
            u = float(b - R)
            s = S[:, a, b]
            M00 = M00 + s
            M10 = M10 + u * s
            M01 = M01 + v * s
            M20 = M20 + (u * u) * s
            M02 = M02 + (v * v) * s
            M11 = M11 + (u * v) * s
    with np.errstate(divide="ignore", invalid="ignore"):
        ub = M10 / M00
        vb = M01 / M00
        m20 = M20 / M00 - ub * ub
        m02 = M02 / M00 - vb * vb
        m11 = M11 / M00 - ub * vb
    return M00, ub, vb, m20, m02, m11


def stamp_filter(mom, max_offset, max_m11, m2_min, m2_max):
    """Step 3: True where the stamp looks like a centred point source."""
    M00, ub, vb, m20, m02, m11 = mom
    with np.errstate(invalid="ignore"):
        return ((M00 > 0) & (np.abs(ub) <= max_offset) & (np.abs(vb) <= max_offset)
                & (np.abs(m11) <= max_m11) & (m20 >= m2_min) & (m20 <= m2_max)
                & (m02 >= m2_min) & (m02 <= m2_max))
