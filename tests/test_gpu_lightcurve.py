"""Parity of the light-curve filter (kb_lightcurve_filter, Sec. 3.3) with the
FP64 oracle, through the C ABI.

* On the oracle's own planes rounded to float32 (the kernel's input
  precision) both sides make every decision in IEEE double from the same
  values, so masks, counts and the float32 nu', alpha' must be identical.
* On the GPU's planes the inputs differ by float32 rounding; a candidate is
  compared where the oracle's decisions do not change when the cut moves by
  0.1% (its decisions are not near-ties), and nu', alpha' within 1e-5.
* At the survey size (15 x 4096^2, K = 50, the benchmarked configuration) on
  sampled start pixels, matching the GPU's candidate lists to the oracle's by
  velocity index.
Candidate velocity indices always come from the oracle's own search.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import lightcurve as olc
from paper_1901_02492_amd import synth
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1901_02492_amd import lib
    lib.load()
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _f32_planes(psi, phi, ok):
    """Oracle planes as the library stores them: float32 pairs, (+0, +0) at
    invalid pixels, phi = -0 at a valid pixel whose phi rounds to zero."""
    p = np.where(ok, psi, 0.0).astype(np.float32)
    f = np.where(ok, phi, 0.0).astype(np.float32)
    f = np.where(ok & (f == 0), np.float32(-0.0), f)
    return p, f


def _candidates(s, ref_vel, rng, extra=64):
    """(ys, xs, js) [H][W][k]: the oracle's top-k velocity indices, with
    `extra` slots replaced by random indices, some outside the grid."""
    n, h, w = s.img.shape
    js = np.array(ref_vel, dtype=np.int32).copy()
    nv = s.vel.shape[0]
    flat = js.reshape(-1)
    pick = rng.choice(flat.size, size=min(extra, flat.size), replace=False)
    flat[pick] = rng.integers(-3, nv + 3, pick.size)
    return js


def _gpu_filter(torch, planes_np, s, js, cut, q):
    from paper_1901_02492_amd import lib
    dev = torch.device("cuda:0")
    planes = torch.from_numpy(np.ascontiguousarray(planes_np)).to(dev)
    cv = torch.from_numpy(np.ascontiguousarray(js)).to(dev)
    nu, al, no, rej = lib.lightcurve_filter(planes, s.t, s.vel, cv, sigma_cut=cut, q=q,
                                            rejected=True)
    torch.cuda.synchronize()
    return nu.cpu().numpy(), al.cpu().numpy(), no.cpu().numpy(), rej.cpu().numpy()


def _mask_bits(rej):
    """bool [C][N] -> uint64 bit masks as int64."""
    n = rej.shape[1]
    bits = (rej.astype(np.uint64) << np.arange(n, dtype=np.uint64)[None, :]).sum(axis=1,
                                                                              dtype=np.uint64)
    return bits.view(np.int64)


CASES = [
    # (name, stack, cut, q)
    ("small", lambda: synth.small_stack(), 5.0, 0.0),
    ("random15", lambda: synth.random_stack(41, 15, 40, 70, 30, 8, n_flash=40), 5.0, 0.0),
    ("random15_walk", lambda: synth.random_stack(42, 15, 37, 53, 25, 6, n_flash=40), 5.0, 0.8),
    ("random15_cut2", lambda: synth.random_stack(43, 15, 33, 65, 20, 5, n_flash=20), 2.0, 0.3),
    ("random33", lambda: synth.random_stack(44, 33, 24, 40, 12, 4, n_flash=30), 5.0, 0.5),
    ("random64", lambda: synth.random_stack(45, 64, 20, 33, 10, 3, n_flash=30), 3.0, 0.2),
    ("random1", lambda: synth.random_stack(46, 1, 17, 19, 6, 3), 5.0, 0.0),
    ("random2", lambda: synth.random_stack(47, 2, 19, 23, 8, 4, n_flash=10), 1.0, 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_filter_identical_on_oracle_planes(torch_dev, case):
    name, make, cut, q = case
    s = make()
    n, h, w = s.img.shape
    _say(f"case {name}: N={n} HxW={h}x{w} V={s.vel.shape[0]} k={s.k} cut={cut} q={q}")
    psi, phi, ok = oracle.psi_phi(s.img, s.var, s.mask, s.psf)
    p32, f32 = _f32_planes(psi, phi, ok)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k)
    js = _candidates(s, ref["vel"], np.random.default_rng(7))
    planes = np.stack([p32, f32], axis=-1)
    nu, al, no, rej = _gpu_filter(torch_dev, planes, s, js, cut, q)
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    ys = np.repeat(yy.reshape(-1), s.k)
    xs = np.repeat(xx.reshape(-1), s.k)
    o = olc.lightcurve_filter(p32.astype(np.float64), f32.astype(np.float64), ok, s.t, s.vel,
                              ys, xs, js.reshape(-1), cut, q)
    nrej = int(o["rejected"].sum())
    multi = int((o["rejected"].sum(axis=1) > 1).sum())
    _say(f"  {js.size} candidates, {nrej} observations dropped, {multi} candidates with more "
         f"than one drop")
    np.testing.assert_array_equal(rej.reshape(-1), _mask_bits(o["rejected"]))
    np.testing.assert_array_equal(no.reshape(-1), o["nobs"])
    np.testing.assert_array_equal(nu.reshape(-1), o["nu"].astype(np.float32))
    np.testing.assert_array_equal(al.reshape(-1), o["alpha"].astype(np.float32))
    if name not in ("small", "random1"):
        assert nrej > 0


def _robust(lc_psi, lc_phi, obs, t, cut, q, margin=1e-3):
    """Candidates whose oracle decisions are not near-ties: at every round of
    the clip (the oracle's own steps, rerun here to read their margins) the
    largest residual is more than `margin` (relative) from the cut and, where
    it is dropped, from the second largest.  The kernel's float32 planes differ
    from the oracle's by rounding, which may decide either kind of near-tie
    (with q > 0 a lone pair's two residuals are equal only up to rounding)."""
    c2 = cut * cut
    tau = np.asarray(t, dtype=np.float64) - t[0]
    keep = obs.copy()
    rows = np.arange(obs.shape[0])
    active = np.ones(obs.shape[0], dtype=bool)
    m_cut = np.full(obs.shape[0], np.inf)
    m_tie = np.full(obs.shape[0], np.inf)
    while active.any():
        J, H = olc.kalman_loo(lc_psi, lc_phi, keep, tau, q)
        r = olc.residual_ratio(lc_psi, lc_phi, keep, J, H)
        srt = np.sort(r, axis=1)
        r1 = srt[:, -1]
        r2 = srt[:, -2] if r.shape[1] > 1 else np.zeros_like(r1)
        m_cut = np.where(active, np.minimum(m_cut, np.abs(r1 - c2) / c2), m_cut)
        drop = active & (r1 > c2)
        m_tie = np.where(drop, np.minimum(m_tie, (r1 - r2) / np.maximum(r1, 1e-300)), m_tie)
        worst = np.argmax(r, axis=1)
        keep[rows[drop], worst[drop]] = False
        active = drop
    assert np.array_equal(obs & ~keep, olc.filter_curves(lc_psi, lc_phi, obs, t, cut, q)["rejected"])
    return (m_cut > margin) & (m_tie > margin)


def _compare_tolerant(nu, al, no, rej, o, lc_phi, obs, robust):
    """Masks and counts equal on robust candidates; nu', alpha' within the
    float32 tolerance of the search: |dnu| <= 1e-5 max(1, |nu|) and
    |dalpha| <= 1e-5 max(|alpha|, 1/sqrt(Phi'))."""
    np.testing.assert_array_equal(rej[robust], _mask_bits(o["rejected"])[robust])
    np.testing.assert_array_equal(no[robust], o["nobs"][robust])
    phi_kept = (lc_phi * (obs & ~o["rejected"])).sum(axis=1)[robust]
    ref_nu, ref_al = o["nu"][robust], o["alpha"][robust]
    g_nu, g_al = nu[robust].astype(np.float64), al[robust].astype(np.float64)
    fin = np.isfinite(ref_nu)
    assert np.array_equal(np.isfinite(g_nu), fin)
    assert (np.abs(g_nu[fin] - ref_nu[fin]) <= 1e-5 * np.maximum(1.0, np.abs(ref_nu[fin]))).all()
    scale = np.maximum(np.abs(ref_al[fin]), 1.0 / np.sqrt(phi_kept[fin]))
    assert (np.abs(g_al[fin] - ref_al[fin]) <= 1e-5 * scale).all()


@pytest.mark.parametrize("q", [0.0, 0.6])
def test_filter_end_to_end_on_gpu_planes(torch_dev, q):
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.random_stack(48, 15, 48, 80, 24, 8, n_flash=60)
    n, h, w = s.img.shape
    _say(f"case end-to-end random48 q={q}")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes = lib.make_psi_phi(img, var, mask, s.psf)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k)
    js = np.ascontiguousarray(ref["vel"].astype(np.int32))
    cv = torch.from_numpy(js).to(dev)
    nu, al, no, rej = lib.lightcurve_filter(planes, s.t, s.vel, cv, sigma_cut=5.0, q=q,
                                            rejected=True)
    torch.cuda.synchronize()
    nu, al, no, rej = (a.cpu().numpy().reshape(-1) for a in (nu, al, no, rej))
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    ys = np.repeat(yy.reshape(-1), s.k)
    xs = np.repeat(xx.reshape(-1), s.k)
    psi, phi, ok = ref["psi"], ref["phi"], oracle.validity(s.img, s.var, s.mask)
    o = olc.lightcurve_filter(psi, phi, ok, s.t, s.vel, ys, xs, js.reshape(-1), 5.0, q)
    robust = _robust(o["lc_psi"], o["lc_phi"], o["obs"], s.t, 5.0, q)
    _say(f"  {robust.size} candidates, {int((~robust).sum())} near the cut, "
         f"{int(o['rejected'].sum())} observations dropped")
    assert robust.mean() > 0.95
    assert o["rejected"].sum() > 0
    _compare_tolerant(nu, al, no, rej, o, o["lc_phi"], o["obs"], robust)


@pytest.mark.slow
def test_filter_survey_sampled(torch_dev):
    """Survey stack with single-image flashes (15 x 4096^2, 600 velocities,
    K = 50): GPU planes, search and top-k, then the filter over every
    candidate, as the benchmark runs it; compared on sampled start pixels."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.survey_stack(n_flash=20000)
    n, h, w = s.img.shape
    rng = np.random.default_rng(8)
    ys = np.concatenate([rng.integers(0, h, 40), [0, h - 1, h // 2]])
    xs = np.concatenate([rng.integers(0, w, 40), [w - 1, 0, w // 2]])
    ref = oracle.search_pixels(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k, ys, xs)
    _say(f"case survey+flashes: oracle search on {ys.size} pixels done")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes, res = lib.run_search(img, var, mask, s.t, s.psf, s.vel, s.k)
    del img, var, mask
    nu, al, no, rej = lib.lightcurve_filter(planes, s.t, s.vel, res[2], sigma_cut=5.0, q=0.0,
                                            rejected=True)
    torch.cuda.synchronize()
    _say("gpu search and filter done")
    yt, xt = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    g_vel = res[2][yt, xt].cpu().numpy()
    g = [a[yt, xt].cpu().numpy() for a in (nu, al, no, rej)]

    def plane_fn(i, yy, xx):
        ps, ph, ok = oracle.psi_phi_at(s.img[i], s.var[i], s.mask[i], s.psf, yy, xx)
        p32, f32 = _f32_planes(ps, ph, ok)
        return p32.astype(np.float64), f32.astype(np.float64), ok

    # Oracle candidates: its own top-K per sampled pixel; compared where the
    # GPU kept the same velocity for that pixel.
    cy, cx, cj, gi = [], [], [], []
    for p in range(ys.size):
        slot = {int(j): r for r, j in enumerate(g_vel[p])}
        for j in ref["vel"][p]:
            if int(j) in slot:
                cy.append(ys[p])
                cx.append(xs[p])
                cj.append(int(j))
                gi.append((p, slot[int(j)]))
    matched = len(cj)
    assert matched >= 0.99 * ys.size * s.k
    lcp, lcf, obs = olc.light_curves_at(plane_fn, n, h, w, s.t, s.vel, np.array(cy),
                                        np.array(cx), np.array(cj))
    o = olc.filter_curves(lcp, lcf, obs, s.t, 5.0, 0.0)
    robust = _robust(lcp, lcf, obs, s.t, 5.0, 0.0)
    pi = np.array(gi)
    sel = lambda a: a[pi[:, 0], pi[:, 1]]
    _say(f"  matched {matched} candidates, {int((~robust).sum())} near the cut, "
         f"{int(o['rejected'].sum())} observations dropped")
    assert o["rejected"].sum() > 0
    _compare_tolerant(sel(g[0]), sel(g[1]), sel(g[2]), sel(g[3]), o, lcf, obs, robust)
