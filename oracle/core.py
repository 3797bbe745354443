"""Plain FP64 CPU oracle of the maximum-likelihood shift-and-stack search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module: only the tests, the package smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library.

What is computed (Whidden et al. 2019, "Fast algorithms for slow moving
asteroids"):

  1. Validity and weights (Sec. 2.1.5, the paragraph on masks: a masked pixel
     gets zero inverse variance).  valid = not masked, finite image, finite
     and positive variance.  w = 1/var and a = img/var where valid, else 0.
  2. Likelihood images for a diagonal covariance (Sec. 2.1.5, the equations
     for Psi and Phi): psi = inverse-variance-weighted cross-correlation of
     the image with the PSF, phi = the same with the squared PSF.  Out-of-frame
     terms are zero.  psi = phi = 0 at invalid pixels.
  3. Linear trajectories (Sec. 2.2): the position in image i of the trajectory
     that starts at pixel (x0, y0) of the earliest image with velocity v is
     x0 + round(vx * tau_i), y0 + round(vy * tau_i), tau_i = t_i - t_0,
     round(u) = floor(u + 0.5) evaluated as an FP64 multiply, then an add,
     then a floor.
  4. Coadd along the trajectory (Sec. 2.1.5, the coadd equations): Psi and Phi
     are the sums of psi_i and phi_i at the trajectory's in-frame valid pixels,
     summed in increasing image order; n_obs counts them.
  5. Scores (Sec. 2.1.5, the maximum-likelihood flux equation and the
     definition of nu): alpha = Psi / Phi and nu = Psi / sqrt(Phi) when
     Phi > 0; otherwise nu = -inf, alpha = 0.
  6. Selection (Sec. 2.2 evaluates nu for every start pixel and velocity; this
     build keeps the K best per start pixel): rank by nu descending, ties by
     ascending velocity index.

Everything runs in float64 on numpy arrays; inputs are promoted from their
stored precision.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "bright_mask", "validity", "weights", "psi_phi", "psi_phi_at", "displacements",
    "trajectory_sums", "trajectory_sums_at", "scores", "rank_topk", "search",
    "search_rows", "search_pixels",
]


def bright_mask(img, mask, threshold) -> np.ndarray:
    """The bright-pixel mask applied before the search (Sec. 5.2): a pixel of
    an image whose value exceeds the count threshold is masked in that image.
    Returns uint8 [N][H][W]: the given mask with bit 0 set where img > threshold
    (a value equal to the threshold, or NaN, does not exceed it)."""
    img = np.asarray(img)
    m = np.zeros(img.shape, dtype=np.uint8) if mask is None else np.array(mask, dtype=np.uint8)
    return np.where(img > threshold, m | np.uint8(1), m).astype(np.uint8)


def validity(img, var, mask) -> np.ndarray:
    """Pixels that carry information (Sec. 2.1.5, masking paragraph).

    A pixel is invalid when its mask byte is nonzero, its image value is not
    finite, or its variance is not a finite positive number.
    """
    img = np.asarray(img, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    ok = np.isfinite(img) & np.isfinite(var) & (var > 0)
    if mask is not None:
        ok &= np.asarray(mask) == 0
    return ok


def weights(img, var, mask):
    """Inverse variance w and inverse-variance-weighted image a (Sec. 2.1.5).

    Masked or otherwise invalid pixels get zero inverse variance, so they add
    nothing to any likelihood sum.
    """
    ok = validity(img, var, mask)
    img = np.asarray(img, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    w = np.zeros(var.shape, dtype=np.float64)
    a = np.zeros(var.shape, dtype=np.float64)
    w[ok] = 1.0 / var[ok]
    a[ok] = img[ok] / var[ok]
    return w, a, ok


def _correlate_zero(plane: np.ndarray, kern: np.ndarray) -> np.ndarray:
    """out[y, x] = sum_{u, v} plane[y + u - cy, x + v - cx] * kern[u, v], zero outside."""
    h, w = plane.shape
    ph, pw = kern.shape
    cy, cx = ph // 2, pw // 2
    out = np.zeros((h, w), dtype=np.float64)
    for u in range(ph):
        dy = u - cy
        for v in range(pw):
            dx = v - cx
            c = kern[u, v]
            # Output rows y with 0 <= y + dy < h, columns x with 0 <= x + dx < w.
            y0, y1 = max(0, -dy), min(h, h - dy)
            x0, x1 = max(0, -dx), min(w, w - dx)
            if y0 >= y1 or x0 >= x1:
                continue
            out[y0:y1, x0:x1] += c * plane[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return out


def psi_phi(img, var, mask, psf):
    """Per-image likelihood planes psi_i and phi_i, float64 [N][H][W] (Sec. 2.1.5).

    psi_i(y) = sum_x a_i(x) T(x - y), phi_i(y) = sum_x w_i(x) T(x - y)^2: the
    cross-correlation of a_i = I_i/var_i and w_i = 1/var_i with the PSF T and
    with T^2.  Zero at invalid pixels.  Also returns the validity planes.
    """
    img = np.asarray(img)
    if img.ndim != 3:
        raise ValueError("img must be [N][H][W]")
    w, a, ok = weights(img, var, mask)
    t = np.asarray(psf, dtype=np.float64)
    t2 = t * t
    psi = np.empty(a.shape, dtype=np.float64)
    phi = np.empty(a.shape, dtype=np.float64)
    for i in range(a.shape[0]):
        psi[i] = _correlate_zero(a[i], t)
        phi[i] = _correlate_zero(w[i], t2)
    psi[~ok] = 0.0
    phi[~ok] = 0.0
    return psi, phi, ok


def psi_phi_at(img_i, var_i, mask_i, psf, ys, xs):
    """psi and phi of one image at the listed pixels only (same definition as psi_phi).

    Used to check sampled outputs of frames too large to correlate whole.
    Returns (psi, phi, valid) as 1-D float64/bool arrays aligned with ys, xs.
    """
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    h, w = np.shape(img_i)
    t = np.asarray(psf, dtype=np.float64)
    ph, pw = t.shape
    cy, cx = ph // 2, pw // 2
    psi = np.zeros(ys.shape, dtype=np.float64)
    phi = np.zeros(ys.shape, dtype=np.float64)
    img_i = np.asarray(img_i)
    var_i = np.asarray(var_i)
    for u in range(ph):
        for v in range(pw):
            yy = ys + (u - cy)
            xx = xs + (v - cx)
            inb = (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
            yc = np.clip(yy, 0, h - 1)
            xc = np.clip(xx, 0, w - 1)
            wv, av, okv = weights(img_i[yc, xc], var_i[yc, xc],
                                  None if mask_i is None else np.asarray(mask_i)[yc, xc])
            okv &= inb
            psi += np.where(okv, av * t[u, v], 0.0)
            phi += np.where(okv, wv * (t[u, v] * t[u, v]), 0.0)
    _, _, ok_here = weights(img_i[ys, xs], var_i[ys, xs],
                            None if mask_i is None else np.asarray(mask_i)[ys, xs])
    psi[~ok_here] = 0.0
    phi[~ok_here] = 0.0
    return psi, phi, ok_here


def displacements(t, vel) -> np.ndarray:
    """Integer pixel offsets of every trajectory in every image, int64 [V][N][2].

    d[j][i] = (floor(vx_j * tau_i + 0.5), floor(vy_j * tau_i + 0.5)) with
    tau_i = t_i - t_0 (Sec. 2.2 linear trajectories y_i = y_0 + v t_i, started
    at the earliest observation as in Sec. 3.2).  The product, the sum and the
    floor are separate IEEE double operations; halves round toward +inf.
    """
    t = np.asarray(t, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    tau = t - t[0]
    d = np.empty((vel.shape[0], t.size, 2), dtype=np.int64)
    for ax in range(2):
        prod = np.multiply(vel[:, ax:ax + 1], tau[None, :])
        d[:, :, ax] = np.floor(np.add(prod, 0.5)).astype(np.int64)
    return d


def trajectory_sums(psi, phi, ok, disp, rows=None, row_offset=0, h_full=None):
    """Psi, Phi (float64) and n_obs (int64) for every velocity and start pixel.

    Output shape [V][R][W] where R are the start rows `rows` (default: all).
    Sum over images in increasing order of the plane values at the in-frame,
    valid trajectory pixels (Sec. 2.1.5 coadd of likelihood images).

    The planes may be a slab of a taller frame: plane row r holds frame row
    r + row_offset, and h_full is the frame height that decides in-frame.
    Every in-frame row a trajectory visits must lie inside the slab.
    """
    n, hs, w = psi.shape
    h = hs if h_full is None else int(h_full)
    rows = np.arange(h) if rows is None else np.asarray(rows, dtype=np.int64)
    nv = disp.shape[0]
    Psi = np.zeros((nv, rows.size, w), dtype=np.float64)
    Phi = np.zeros((nv, rows.size, w), dtype=np.float64)
    cnt = np.zeros((nv, rows.size, w), dtype=np.int64)
    for j in range(nv):
        for i in range(n):
            dx, dy = int(disp[j, i, 0]), int(disp[j, i, 1])
            yy = rows + dy
            rsel = (yy >= 0) & (yy < h)
            if not rsel.any():
                continue
            x0, x1 = max(0, -dx), min(w, w - dx)
            if x0 >= x1:
                continue
            ridx = np.nonzero(rsel)[0]
            src = yy[ridx] - row_offset
            if src.min() < 0 or src.max() >= hs:
                raise ValueError("trajectory leaves the plane slab")
            Psi[j, ridx, x0:x1] += psi[i, src, x0 + dx:x1 + dx]
            Phi[j, ridx, x0:x1] += phi[i, src, x0 + dx:x1 + dx]
            cnt[j, ridx, x0:x1] += ok[i, src, x0 + dx:x1 + dx]
    return Psi, Phi, cnt


def trajectory_sums_at(plane_fn, n, h, w, disp, ys, xs):
    """Psi, Phi, n_obs for start pixels (ys[p], xs[p]) and every velocity: [V][P].

    plane_fn(i, yy, xx) -> (psi, phi, valid) evaluates image i's planes at the
    given in-frame pixels; out-of-frame positions contribute nothing.
    """
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    nv = disp.shape[0]
    Psi = np.zeros((nv, ys.size), dtype=np.float64)
    Phi = np.zeros((nv, ys.size), dtype=np.float64)
    cnt = np.zeros((nv, ys.size), dtype=np.int64)
    for i in range(n):
        yy = ys[None, :] + disp[:, i, 1][:, None]
        xx = xs[None, :] + disp[:, i, 0][:, None]
        inb = (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
        if not inb.any():
            continue
        ps, ph_, ok = plane_fn(i, yy[inb], xx[inb])
        tmp = np.zeros(yy.shape, dtype=np.float64)
        tmp[inb] = ps
        Psi += tmp
        tmp[inb] = ph_
        Phi += tmp
        c = np.zeros(yy.shape, dtype=np.int64)
        c[inb] = ok
        cnt += c
    return Psi, Phi, cnt


def scores(Psi, Phi):
    """nu = Psi/sqrt(Phi) and alpha_ML = Psi/Phi (Sec. 2.1.5); nu = -inf, alpha = 0 if Phi <= 0."""
    Psi = np.asarray(Psi, dtype=np.float64)
    Phi = np.asarray(Phi, dtype=np.float64)
    pos = Phi > 0
    safe = np.where(pos, Phi, 1.0)
    nu = np.where(pos, Psi / np.sqrt(safe), -np.inf)
    alpha = np.where(pos, Psi / safe, 0.0)
    return nu, alpha


def rank_topk(nu, k):
    """Indices along axis 0 of the k best by nu descending, ties by ascending index.

    nu has the velocity on axis 0.  Returns int64 [k][...].
    """
    # A stable sort of -nu keeps equal values in ascending velocity order.
    order = np.argsort(-np.asarray(nu, dtype=np.float64), axis=0, kind="stable")
    return order[:k]


def _gather_top(order, *arrays):
    return [np.take_along_axis(a, order, axis=0) for a in arrays]


def search(img, var, mask, t, psf, vel, k):
    """Full search over every start pixel: per-pixel top-k, arrays [H][W][k].

    Returns dict(nu, alpha, vel, nobs) plus the per-trajectory arrays
    (all_nu, all_alpha, all_nobs: [V][H][W]) the tests use for tolerant
    comparison.
    """
    psi, phi, ok = psi_phi(img, var, mask, psf)
    disp = displacements(t, vel)
    Psi, Phi, cnt = trajectory_sums(psi, phi, ok, disp)
    nu, alpha = scores(Psi, Phi)
    order = rank_topk(nu, k)
    tnu, tal, tcnt = _gather_top(order, nu, alpha, cnt)
    mv = lambda a: np.moveaxis(a, 0, -1)
    return dict(nu=mv(tnu), alpha=mv(tal), vel=mv(order), nobs=mv(tcnt),
                all_nu=nu, all_alpha=alpha, all_nobs=cnt, all_Phi=Phi, psi=psi, phi=phi)


def search_rows(img, var, mask, t, psf, vel, k, row_lo, row_hi):
    """Top-k for start rows [row_lo, row_hi) of a frame, correlating only the
    rows those trajectories can reach (plus the PSF half-height around them).
    Same arrays as search(), with R = row_hi - row_lo rows."""
    n, h, w = np.shape(img)
    disp = displacements(t, vel)
    dy = disp[:, :, 1]
    r = np.shape(psf)[0] // 2
    need_lo = max(0, row_lo + int(dy.min()))
    need_hi = min(h, row_hi - 1 + int(dy.max()) + 1)
    Psi = Phi = cnt = None
    if need_lo < need_hi:
        lo, hi = max(0, need_lo - r), min(h, need_hi + r)
        psi, phi, ok = psi_phi(np.asarray(img)[:, lo:hi], np.asarray(var)[:, lo:hi],
                               None if mask is None else np.asarray(mask)[:, lo:hi], psf)
        # Rows of the slab outside [need_lo, need_hi) may see a cut PSF; no
        # trajectory visits them, so blank them to make any misuse visible.
        psi[:, :need_lo - lo] = np.nan
        psi[:, need_hi - lo:] = np.nan
        Psi, Phi, cnt = trajectory_sums(psi, phi, ok, disp, rows=np.arange(row_lo, row_hi),
                                        row_offset=lo, h_full=h)
    else:
        shape = (disp.shape[0], row_hi - row_lo, w)
        Psi, Phi, cnt = np.zeros(shape), np.zeros(shape), np.zeros(shape, dtype=np.int64)
    nu, alpha = scores(Psi, Phi)
    order = rank_topk(nu, k)
    tnu, tal, tcnt = _gather_top(order, nu, alpha, cnt)
    mv = lambda a: np.moveaxis(a, 0, -1)
    return dict(nu=mv(tnu), alpha=mv(tal), vel=mv(order), nobs=mv(tcnt),
                all_nu=nu, all_alpha=alpha, all_nobs=cnt, all_Phi=Phi)


def search_pixels(img, var, mask, t, psf, vel, k, ys, xs):
    """Top-k for an arbitrary list of start pixels, evaluating the planes only
    at the visited positions.  Arrays are [P][k]; all_* are [V][P]."""
    img = np.asarray(img)
    n, h, w = img.shape
    disp = displacements(t, vel)

    def plane_fn(i, yy, xx):
        return psi_phi_at(img[i], np.asarray(var)[i],
                          None if mask is None else np.asarray(mask)[i], psf, yy, xx)

    Psi, Phi, cnt = trajectory_sums_at(plane_fn, n, h, w, disp, ys, xs)
    nu, alpha = scores(Psi, Phi)
    order = rank_topk(nu, k)
    tnu, tal, tcnt = _gather_top(order, nu, alpha, cnt)
    mv = lambda a: np.moveaxis(a, 0, -1)
    return dict(nu=mv(tnu), alpha=mv(tal), vel=mv(order), nobs=mv(tcnt),
                all_nu=nu, all_alpha=alpha, all_nobs=cnt, all_Phi=Phi)
