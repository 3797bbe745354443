"""Seeded synthetic inputs shaped like the paper's image stacks.

This module draws inputs only: science images, variance planes, masks,
observation times, a PSF kernel and a velocity grid.  It holds none of the
search's arithmetic (no likelihood planes, no displacements, no sums, no
scores), so both the oracle-based tests and the HIP path can consume the same
bytes.

Stand-in for the paper's data: the HiTS DECam warped 4K x 4K patches with
their variance and mask planes (Sec. 3.1) are not available, so every stack
here is synthetic noise plus injected point sources rendered with a Gaussian
PSF (Sec. 2.3 uses a Gaussian PSF approximation; Sec. 4.1 injects sources
with a Gaussian PSF matched to the search PSF).

Conventions used everywhere in this package:
  * img, var: float32 [N][H][W]; mask: uint8 [N][H][W], nonzero = bad pixel;
  * t: float64 [N] in days, ascending; trajectories start at t[0];
  * psf: float32 [ph][pw], odd sizes, centre at (ph//2, pw//2);
  * vel: float64 [V][2] = (vx, vy) in pixels/day; x = column, y = row.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import ndtr

SEED_BASE = 1901_02492


def seed_for(cfg: int, stream: int) -> int:
    """Seed of random stream `stream` (0 noise, 1 masks, 2 injections) of workload `cfg`."""
    return SEED_BASE + 10 * cfg + stream


# ---------------------------------------------------------------------------
# PSF kernels (Sec. 2.1.2: the PSF used for the likelihood images includes the
# pixel transfer function, i.e. a top-hat pixel convolved with the PSF).
# ---------------------------------------------------------------------------

def _pixel_integrated_1d(sigma: float, half: int) -> np.ndarray:
    u = np.arange(-half, half + 1, dtype=np.float64)
    return ndtr((u + 0.5) / sigma) - ndtr((u - 0.5) / sigma)


def psf_gaussian(sigma: float, size: int, integrated: bool = True) -> np.ndarray:
    """Normalised (unit-sum) Gaussian PSF on an odd `size` x `size` window.

    integrated=True integrates the Gaussian over each unit pixel (the pixel
    transfer function of Sec. 2.1.2); False samples it at pixel centres.
    Returned as float32: the float32 values are what both the library and the
    oracle consume.
    """
    if size % 2 != 1:
        raise ValueError("PSF size must be odd")
    half = size // 2
    if integrated:
        g = _pixel_integrated_1d(sigma, half)
    else:
        u = np.arange(-half, half + 1, dtype=np.float64)
        g = np.exp(-0.5 * (u / sigma) ** 2)
    k = np.outer(g, g)
    k /= k.sum()
    return k.astype(np.float32)


# ---------------------------------------------------------------------------
# Velocity grids (Sec. 3.2: a linearly spaced grid of angles x speeds).
# ---------------------------------------------------------------------------

def velocity_grid_xy(vx_values, vy_values) -> np.ndarray:
    """Cartesian grid: index j = a * len(vy_values) + b for (vx_values[a], vy_values[b])."""
    vx = np.asarray(vx_values, dtype=np.float64)
    vy = np.asarray(vy_values, dtype=np.float64)
    out = np.empty((vx.size * vy.size, 2), dtype=np.float64)
    out[:, 0] = np.repeat(vx, vy.size)
    out[:, 1] = np.tile(vy, vx.size)
    return out


def velocity_grid_polar(speeds, angles) -> np.ndarray:
    """Speed x angle grid: j = i_s * n_angles + i_theta, v = s (cos theta, sin theta)."""
    s = np.asarray(speeds, dtype=np.float64)
    th = np.asarray(angles, dtype=np.float64)
    ss = np.repeat(s, th.size)
    tt = np.tile(th, s.size)
    return np.stack([ss * np.cos(tt), ss * np.sin(tt)], axis=1)


# ---------------------------------------------------------------------------
# Source rendering (input synthesis only).
# ---------------------------------------------------------------------------

def render_point_source(img: np.ndarray, cx: float, cy: float, flux: float,
                        sigma: float) -> None:
    """Add a pixel-integrated Gaussian of total `flux` centred at (cx, cy) to img in place."""
    h, w = img.shape
    r = int(math.ceil(5.0 * sigma))
    x0, x1 = int(math.floor(cx)) - r, int(math.floor(cx)) + r + 1
    y0, y1 = int(math.floor(cy)) - r, int(math.floor(cy)) + r + 1
    xa, xb = max(x0, 0), min(x1, w)
    ya, yb = max(y0, 0), min(y1, h)
    if xa >= xb or ya >= yb:
        return
    xs = np.arange(xa, xb, dtype=np.float64)
    ys = np.arange(ya, yb, dtype=np.float64)
    gx = ndtr((xs + 0.5 - cx) / sigma) - ndtr((xs - 0.5 - cx) / sigma)
    gy = ndtr((ys + 0.5 - cy) / sigma) - ndtr((ys - 0.5 - cy) / sigma)
    img[ya:yb, xa:xb] += (flux * np.outer(gy, gx)).astype(img.dtype)


@dataclasses.dataclass
class Stack:
    """One synthetic search problem plus the truth it was drawn from."""
    img: np.ndarray          # float32 [N][H][W]
    var: np.ndarray          # float32 [N][H][W]
    mask: np.ndarray         # uint8  [N][H][W]
    t: np.ndarray            # float64 [N]
    psf: np.ndarray          # float32 [ph][pw]
    vel: np.ndarray          # float64 [V][2]
    k: int                   # results kept per start pixel
    sources: np.ndarray      # float64 [S][5]: x0, y0, vx, vy, flux
    name: str = ""

    @property
    def shape(self):
        return self.img.shape

    @property
    def tie(self) -> int:
        """Trajectory-image evaluations of one full search: N * H * W * V."""
        n, h, w = self.img.shape
        return int(n) * int(h) * int(w) * int(self.vel.shape[0])


# ---------------------------------------------------------------------------
# Workloads.
# ---------------------------------------------------------------------------

def small_stack() -> Stack:
    """5 images of 64x64 at t = 0..0.2 d, unit noise and variance, 7x7 PSF (sigma 1),
    one source of flux 50 from (20, 30) moving (40, 25) px/d, an 11x11 velocity
    grid over [-50, 50] px/d per axis, 5 kept per pixel."""
    n, h, w = 5, 64, 64
    rng = np.random.default_rng(seed_for(0, 0))
    t = np.array([0.0, 0.05, 0.1, 0.15, 0.2], dtype=np.float64)
    img = rng.standard_normal((n, h, w), dtype=np.float32)
    var = np.ones((n, h, w), dtype=np.float32)
    mask = np.zeros((n, h, w), dtype=np.uint8)
    src = np.array([[20.0, 30.0, 40.0, 25.0, 50.0]])
    for i in range(n):
        for x0, y0, vx, vy, f in src:
            render_point_source(img[i], x0 + vx * t[i], y0 + vy * t[i], f, 1.0)
    vals = np.arange(-50.0, 50.0 + 1e-9, 10.0)
    return Stack(img, var, mask, t, psf_gaussian(1.0, 7), velocity_grid_xy(vals, vals),
                 5, src, name="5x64x64, 121 velocities, K=5")


def _smooth_sigma(rng, n, h, w, amp=0.2):
    """Per-image noise sigma field 1 + amp*sin(2pi(x/W+a))*sin(2pi(y/H+b)), in [0.8, 1.2]."""
    ph = rng.random((n, 2))
    xs = np.arange(w, dtype=np.float64) / w
    ys = np.arange(h, dtype=np.float64) / h
    out = np.empty((n, h, w), dtype=np.float32)
    for i in range(n):
        sx = np.sin(2 * np.pi * (xs + ph[i, 0]))
        sy = np.sin(2 * np.pi * (ys + ph[i, 1]))
        out[i] = (1.0 + amp * np.outer(sy, sx)).astype(np.float32)
    return out


def add_flashes(img: np.ndarray, var: np.ndarray, n_flash: int, rng, psf_sigma: float,
                s2: float, snr=(10.0, 100.0)) -> np.ndarray:
    """Point sources that appear in one image only (a fast or bright object
    crossing a trajectory in a single exposure, Sec. 3.3), each at a random
    image, position and single-image signal-to-noise in `snr`.  Returns
    float64 [n_flash][4]: image, x, y, flux."""
    n, h, w = img.shape
    out = np.zeros((n_flash, 4))
    for f in range(n_flash):
        i = int(rng.integers(0, n))
        x, y = rng.uniform(0, w), rng.uniform(0, h)
        flux = rng.uniform(*snr) / math.sqrt(s2 / float(var[i, int(y), int(x)]))
        render_point_source(img[i], x, y, flux, psf_sigma)
        out[f] = (i, x, y, flux)
    return out


def survey_stack(cfg: int = 1, n_nights: int = 3, epochs: int = 5, h: int = 4096,
                 w: int = 4096, n_src: int = 100, snr=(5.0, 20.0), n_speeds: int = 25,
                 n_angles: int = 24, k: int = 50, mask_frac: float = 0.01,
                 psf_sigma: float = 1.5, psf_size: int = 11, n_flash: int = 0) -> Stack:
    """Survey-shaped stack: nights x epochs images 0.06 d apart within a night
    (Sec. 3.1: ~5 visits per night over three nights), smoothly varying noise
    sigma in [0.8, 1.2] with var = sigma^2, random 1% masks per image, an
    11x11 Gaussian PSF (sigma 1.5 px), injected sources at speeds 80-400 px/d
    within +-0.5 rad of the x axis, and a speed x angle velocity grid over the
    same ranges.  Defaults: 15 x 4096^2, 600 velocities, K = 50.  n_flash > 0
    adds that many single-image sources (add_flashes), drawn after the rest."""
    n = n_nights * epochs
    t = np.array([night + 0.06 * e for night in range(n_nights) for e in range(epochs)],
                 dtype=np.float64)
    rng_n = np.random.default_rng(seed_for(cfg, 0))
    rng_m = np.random.default_rng(seed_for(cfg, 1))
    rng_s = np.random.default_rng(seed_for(cfg, 2))
    sigma = _smooth_sigma(rng_n, n, h, w)
    img = np.empty((n, h, w), dtype=np.float32)
    for i in range(n):
        img[i] = rng_n.standard_normal((h, w), dtype=np.float32)
        img[i] *= sigma[i]
    var = sigma
    np.square(var, out=var)
    mask = np.empty((n, h, w), dtype=np.uint8)
    for i in range(n):
        mask[i] = rng_m.random((h, w), dtype=np.float32) < mask_frac
    psf = psf_gaussian(psf_sigma, psf_size)
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    srcs = []
    for _ in range(n_src):
        x0 = rng_s.uniform(0, w)
        y0 = rng_s.uniform(0, h)
        sp = rng_s.uniform(80.0, 400.0)
        an = rng_s.uniform(-0.5, 0.5)
        target = rng_s.uniform(*snr)
        vx, vy = sp * math.cos(an), sp * math.sin(an)
        # Flux giving the requested signal-to-noise over the epochs in frame.
        inv = 0.0
        for i in range(n):
            cx, cy = x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0])
            if 0 <= cx < w and 0 <= cy < h:
                inv += s2 / float(var[i, int(cy), int(cx)])
        flux = target / math.sqrt(inv) if inv > 0 else 0.0
        for i in range(n):
            render_point_source(img[i], x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0]),
                                flux, psf_sigma)
        srcs.append((x0, y0, vx, vy, flux))
    if n_flash:
        add_flashes(img, var, n_flash, np.random.default_rng(seed_for(cfg, 3)), psf_sigma, s2)
    speeds = np.linspace(80.0, 400.0, n_speeds)
    angles = np.linspace(-0.5, 0.5, n_angles)
    return Stack(img, var, mask, t, psf, velocity_grid_polar(speeds, angles), k,
                 np.array(srcs, dtype=np.float64),
                 name=f"{n}x{h}x{w}, {n_speeds * n_angles} velocities, K={k}")


# HiTS geometry (Sec. 3.1, Sec. 3.2): 0.26 arcsec pixels, visits 1.6 h apart.
HITS_ARCSEC_PER_PX = 0.26
HITS_VISIT_GAP_D = 1.6 / 24.0
# Bright-pixel level of the HiTS workload in units of the sky noise sigma.
# Sec. 5.2 masks pixels above 120 counts; with this stack's sigma ~ 1 the
# cut is placed at 5 sigma per pixel, which single-image flashes of SNR
# 10-100 exceed at their peaks and the search's own sources rarely do.
HITS_BRIGHT_SIGMA = 5.0


def hits_velocities(n_speeds: int = 250, n_angles: int = 128) -> np.ndarray:
    """Sec. 3.2 grid: speeds linspace(1, 5.7) arcsec/h (92.3 to 526.2 px/d at
    0.26 arcsec/px) x angles linspace(-12, 12) degrees about the x axis."""
    px_per_day = 24.0 / HITS_ARCSEC_PER_PX
    speeds = np.linspace(1.0, 5.7, n_speeds) * px_per_day
    angles = np.deg2rad(np.linspace(-12.0, 12.0, n_angles))
    return velocity_grid_polar(speeds, angles)


def hits_stack(h: int = 4096, w: int = 4096, visits=(5, 4, 4), n_src: int = 100,
               snr=(5.0, 20.0), k: int = 50, mask_frac: float = 0.01, psf_sigma: float = 1.5,
               psf_size: int = 11, n_flash: int = 20000, n_speeds: int = 250,
               n_angles: int = 128) -> Stack:
    """HiTS-shaped stack (Sec. 3.1, Sec. 3.2): 13 images over three nights
    (5, 4 and 4 visits 1.6 h apart), the survey noise field, masks and PSF,
    n_src sources at SNR U(5, 20) moving within the grid's range, n_flash
    single-image flashes, and the 250 x 128 = 32000-velocity grid."""
    cfg = 5
    t = np.array([night + HITS_VISIT_GAP_D * e for night, nv in enumerate(visits)
                  for e in range(nv)], dtype=np.float64)
    n = t.size
    rng_n = np.random.default_rng(seed_for(cfg, 0))
    rng_m = np.random.default_rng(seed_for(cfg, 1))
    rng_s = np.random.default_rng(seed_for(cfg, 2))
    sigma = _smooth_sigma(rng_n, n, h, w)
    img = np.empty((n, h, w), dtype=np.float32)
    for i in range(n):
        img[i] = rng_n.standard_normal((h, w), dtype=np.float32)
        img[i] *= sigma[i]
    var = sigma
    np.square(var, out=var)
    mask = np.empty((n, h, w), dtype=np.uint8)
    for i in range(n):
        mask[i] = rng_m.random((h, w), dtype=np.float32) < mask_frac
    psf = psf_gaussian(psf_sigma, psf_size)
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    vel = hits_velocities(n_speeds, n_angles)
    sp_lo, sp_hi = np.hypot(vel[:, 0], vel[:, 1]).min(), np.hypot(vel[:, 0], vel[:, 1]).max()
    srcs = []
    for _ in range(n_src):
        x0, y0 = rng_s.uniform(0, w), rng_s.uniform(0, h)
        sp = rng_s.uniform(sp_lo, sp_hi)
        an = rng_s.uniform(-np.deg2rad(12.0), np.deg2rad(12.0))
        target = rng_s.uniform(*snr)
        vx, vy = sp * math.cos(an), sp * math.sin(an)
        inv = 0.0
        for i in range(n):
            cx, cy = x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0])
            if 0 <= cx < w and 0 <= cy < h:
                inv += s2 / float(var[i, int(cy), int(cx)])
        flux = target / math.sqrt(inv) if inv > 0 else 0.0
        for i in range(n):
            render_point_source(img[i], x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0]),
                                flux, psf_sigma)
        srcs.append((x0, y0, vx, vy, flux))
    if n_flash:
        add_flashes(img, var, n_flash, np.random.default_rng(seed_for(cfg, 3)), psf_sigma, s2)
    return Stack(img, var, mask, t, psf, vel, k, np.array(srcs, dtype=np.float64),
                 name=f"{n}x{h}x{w}, {vel.shape[0]} velocities, K={k}, HiTS grid")


def random_stack(seed: int, n: int, h: int, w: int, n_vel: int, k: int,
                 psf_size: int = 5, psf_sigma: float = 1.0, mask_frac: float = 0.05,
                 vmax: float = 40.0, tmax: float = 1.0, n_flash: int = 0) -> Stack:
    """Small randomized stack for parity sweeps: random times, noise, variance
    and masks; velocities drawn uniformly in [-vmax, vmax]^2 so tracks leave
    the frame on every side.  n_flash > 0 adds single-image sources."""
    rng = np.random.default_rng(SEED_BASE + 7919 * seed)
    t = np.sort(rng.uniform(0.0, tmax, size=n))
    t[0] = 0.0
    img = rng.standard_normal((n, h, w), dtype=np.float32)
    var = rng.uniform(0.5, 2.0, size=(n, h, w)).astype(np.float32)
    mask = (rng.random((n, h, w)) < mask_frac).astype(np.uint8)
    vel = rng.uniform(-vmax, vmax, size=(n_vel, 2))
    src = []
    if h > 8 and w > 8:
        x0, y0 = rng.uniform(2, w - 2), rng.uniform(2, h - 2)
        vx, vy = vel[0]
        for i in range(n):
            render_point_source(img[i], x0 + vx * t[i], y0 + vy * t[i], 20.0, psf_sigma)
        src.append((x0, y0, vx, vy, 20.0))
    psf = psf_gaussian(psf_sigma, psf_size)
    if n_flash:
        add_flashes(img, var, n_flash, np.random.default_rng(SEED_BASE + 7919 * seed + 1),
                    psf_sigma, float(np.sum(psf.astype(np.float64) ** 2)))
    return Stack(img, var, mask, t, psf, vel, k,
                 np.array(src, dtype=np.float64).reshape(-1, 5), name=f"random{seed}")


# ---------------------------------------------------------------------------
# Device-side generation (serving workloads): the survey recipe drawn with the
# device's own random generator, so that a request's inputs appear in
# milliseconds.  Same seed, shape and device give the same bytes.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DeviceStack:
    img: "object"            # torch float32 [N][H][W] on the device
    var: "object"            # torch float32 [N][H][W]
    mask: "object"           # torch uint8 [N][H][W]
    t: np.ndarray
    psf: np.ndarray
    vel: np.ndarray
    k: int
    sources: np.ndarray
    name: str = ""

    @property
    def tie(self) -> int:
        n, h, w = self.img.shape
        return int(n) * int(h) * int(w) * int(self.vel.shape[0])


def survey_times(n_img: int, epochs: int = 5) -> np.ndarray:
    """Observation times of a survey-shaped stack: `epochs` visits 0.06 d apart
    per night, consecutive nights, n_img images in total."""
    return np.array([i // epochs + 0.06 * (i % epochs) for i in range(n_img)], dtype=np.float64)


def survey_velocities(n_speeds: int, n_angles: int) -> np.ndarray:
    """Speed x angle grid of the survey workloads: speeds linspace(80, 400) px/d,
    angles linspace(-0.5, 0.5) rad (Sec. 3.1's linearly spaced grid)."""
    return velocity_grid_polar(np.linspace(80.0, 400.0, n_speeds), np.linspace(-0.5, 0.5, n_angles))


def serving_requests(n: int = 200, rate: float = 4.0, seed: int = SEED_BASE + 3000):
    """Request stream of the serving workload: Poisson arrivals at `rate` per
    second (seeded exponential gaps, the first at 0), N uniform in 8..20, frames
    1024^2, 2048^2 or 4096^2, V uniform in [200, 2000] rounded to a multiple of
    20 and laid out as V/20 speeds x 20 angles.  Each entry carries the seed of
    its own stack."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(n):
        n_img = int(rng.integers(8, 21))
        side = int(rng.choice([1024, 2048, 4096]))
        v = int(round(rng.uniform(200.0, 2000.0) / 20.0)) * 20
        out.append(dict(rid=q, arrival=float(arrivals[q]), n_img=n_img, h=side, w=side,
                        n_speeds=v // 20, n_angles=20, seed=seed + 1 + q))
    return out


def device_survey_stack(seed: int, n_img: int, h: int, w: int, n_speeds: int, n_angles: int,
                        device, k: int = 50, src_per_16m: float = 100.0, snr=(5.0, 20.0),
                        mask_frac: float = 0.01, psf_sigma: float = 1.5,
                        psf_size: int = 11) -> DeviceStack:
    """A survey-shaped stack generated on `device`: survey times, noise sigma
    1 + 0.2 sin sin (per-image phases) with var = sigma^2, random masks,
    sources at speeds 80-400 px/d within +-0.5 rad (src_per_16m per 4096^2
    pixels, flux for the drawn signal-to-noise over the epochs in frame) and a
    speed x angle grid over the same ranges."""
    import torch
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    t = survey_times(n_img)
    ph = rng.random((n_img, 2))
    xs = torch.arange(w, device=device, dtype=torch.float64) / w
    ys = torch.arange(h, device=device, dtype=torch.float64) / h
    sig = torch.empty((n_img, h, w), device=device, dtype=torch.float32)
    for i in range(n_img):
        sx = torch.sin(2 * math.pi * (xs + float(ph[i, 0])))
        sy = torch.sin(2 * math.pi * (ys + float(ph[i, 1])))
        sig[i] = (1.0 + 0.2 * torch.outer(sy, sx)).to(torch.float32)
    img = torch.randn((n_img, h, w), generator=gen, device=device, dtype=torch.float32)
    img.mul_(sig)
    var = sig.square_()
    mask = (torch.rand((n_img, h, w), generator=gen, device=device) < mask_frac).to(torch.uint8)
    psf = psf_gaussian(psf_sigma, psf_size)
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    n_src = int(round(src_per_16m * h * w / float(4096 * 4096)))
    srcs = []
    r = int(math.ceil(5.0 * psf_sigma))
    stamps_idx, stamps_val = [], []
    for _ in range(n_src):
        x0, y0 = rng.uniform(0, w), rng.uniform(0, h)
        sp, an = rng.uniform(80.0, 400.0), rng.uniform(-0.5, 0.5)
        target = rng.uniform(*snr)
        vx, vy = sp * math.cos(an), sp * math.sin(an)
        inv = 0.0
        for i in range(n_img):
            cx, cy = x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0])
            if 0 <= cx < w and 0 <= cy < h:
                s = (1.0 + 0.2 * math.sin(2 * math.pi * (int(cx) / w + ph[i, 0])) *
                     math.sin(2 * math.pi * (int(cy) / h + ph[i, 1])))
                inv += s2 / (s * s)
        flux = target / math.sqrt(inv) if inv > 0 else 0.0
        for i in range(n_img):
            cx, cy = x0 + vx * (t[i] - t[0]), y0 + vy * (t[i] - t[0])
            xa, xb = max(int(math.floor(cx)) - r, 0), min(int(math.floor(cx)) + r + 1, w)
            ya, yb = max(int(math.floor(cy)) - r, 0), min(int(math.floor(cy)) + r + 1, h)
            if xa >= xb or ya >= yb:
                continue
            gx = (ndtr((np.arange(xa, xb) + 0.5 - cx) / psf_sigma) -
                  ndtr((np.arange(xa, xb) - 0.5 - cx) / psf_sigma))
            gy = (ndtr((np.arange(ya, yb) + 0.5 - cy) / psf_sigma) -
                  ndtr((np.arange(ya, yb) - 0.5 - cy) / psf_sigma))
            yy, xx = np.meshgrid(np.arange(ya, yb), np.arange(xa, xb), indexing="ij")
            stamps_idx.append(((i * h + yy) * w + xx).ravel())
            stamps_val.append((flux * np.outer(gy, gx)).ravel())
        srcs.append((x0, y0, vx, vy, flux))
    if stamps_idx:
        # Overlapping stamps are summed on the host (fixed order), so that every
        # pixel is written once and the bytes do not depend on atomics.
        uidx, inv = np.unique(np.concatenate(stamps_idx), return_inverse=True)
        uval = np.bincount(inv, weights=np.concatenate(stamps_val)).astype(np.float32)
        idx = torch.from_numpy(uidx).to(device)
        flat = img.view(-1)
        flat[idx] = flat[idx] + torch.from_numpy(uval).to(device)
    vel = survey_velocities(n_speeds, n_angles)
    return DeviceStack(img, var, mask, t, psf, vel, k, np.array(srcs, dtype=np.float64).reshape(-1, 5),
                       name=f"{n_img}x{h}x{w}, {n_speeds * n_angles} velocities, K={k}")
