"""Parity of the HIP path (through the C ABI) with the FP64 oracle on a GPU."""
import math
import sys

import numpy as np
import pytest

import oracle
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


def run_gpu(torch, s, k_cand=None, k=None):
    from paper_1901_02492_amd import lib
    k = s.k if k is None else k
    dev = torch.device("cuda:0")
    img = torch.from_numpy(np.ascontiguousarray(s.img)).to(dev)
    var = torch.from_numpy(np.ascontiguousarray(s.var)).to(dev)
    mask = torch.from_numpy(np.ascontiguousarray(s.mask)).to(dev)
    planes, res = lib.run_search(img, var, mask, s.t, s.psf, s.vel, k, k_cand=k_cand)
    torch.cuda.synchronize()
    return planes.cpu().numpy(), parity.to_numpy(res)


def _full_check(torch, s, k_cand=None, k=None):
    k = s.k if k is None else k
    _say(f"case {s.name}: N={s.img.shape[0]} HxW={s.img.shape[1]}x{s.img.shape[2]} "
         f"V={s.vel.shape[0]} k={k} k_cand={k_cand}")
    planes, res = run_gpu(torch, s, k_cand=k_cand, k=k)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, k)
    parity.check_planes(planes, ref["psi"], ref["phi"], oracle.validity(s.img, s.var, s.mask))
    H, W = s.img.shape[1:]
    gpu = [r.reshape(H * W, k) for r in res]
    return parity.check_topk(gpu, *parity.oracle_full_as_pixels(ref), k), res, ref


def test_small_workload(torch_dev):
    s = synth.small_stack()
    n_tie_px, res, ref = _full_check(torch_dev, s)
    nu, al, vel, nobs = res
    assert tuple(s.vel[vel[30, 20, 0]]) == (40.0, 20.0)
    _say(f"near-tie pixels: {n_tie_px}")


RANDOM_CASES = [
    # seed, n, h, w, n_vel, k, k_cand
    (1, 3, 37, 71, 9, 4, None),        # ragged width (2 tiles, partial second)
    (2, 1, 19, 64, 6, 6, None),        # N = 1, k = V
    (3, 5, 5, 130, 17, 1, None),       # k = 1, three tiles per row
    (4, 17, 23, 29, 12, 5, 12),        # N > 16 (two load batches), k_cand > k
    (5, 33, 9, 33, 8, 3, 8),           # N > 32
    (6, 4, 1, 1, 5, 5, None),          # single pixel
    (7, 6, 64, 64, 64, 64, None),      # k = k_cand = 64 (largest list)
    (8, 2, 40, 100, 50, 41, 50),       # list length 56 with k_cand = 50
]


@pytest.mark.parametrize("case", RANDOM_CASES, ids=[f"seed{c[0]}" for c in RANDOM_CASES])
def test_random_stacks(torch_dev, case):
    seed, n, h, w, nv, k, kc = case
    s = synth.random_stack(seed, n=n, h=h, w=w, n_vel=nv, k=k, psf_size=5,
                           vmax=max(h, w) * 0.8)
    _full_check(torch_dev, s, k_cand=kc, k=k)


def test_fully_masked_image_and_bad_pixels(torch_dev):
    s = synth.random_stack(11, n=4, h=30, w=70, n_vel=10, k=4, psf_size=3)
    s.mask[2] = 1
    s.img[1, 5, 7] = np.nan
    s.var[0, 10, 20] = 0.0
    s.var[3, 11, 21] = -1.0
    s.img[3, 12, 22] = np.inf
    _full_check(torch_dev, s)


def test_everything_masked(torch_dev):
    s = synth.random_stack(12, n=3, h=8, w=70, n_vel=6, k=3, psf_size=3)
    s.mask[:] = 1
    planes, res = run_gpu(torch_dev, s)
    nu, al, vel, nobs = res
    assert np.all(planes == 0)
    assert np.all(np.isneginf(nu)) and np.all(al == 0) and np.all(nobs == 0)
    assert np.array_equal(vel, np.broadcast_to(np.arange(3), vel.shape))


@pytest.mark.parametrize("psf_shape", [(1, 1), (3, 5), (25, 25), (7, 1)])
def test_planes_psf_shapes(torch_dev, psf_shape):
    rng = np.random.default_rng(sum(psf_shape))
    s = synth.random_stack(20 + psf_shape[0], n=2, h=45, w=90, n_vel=3, k=2)
    psf = rng.uniform(0, 1, psf_shape)
    s.psf = (psf / psf.sum()).astype(np.float32)   # asymmetric, unit sum like a real PSF
    _full_check(torch_dev, s)


def test_deterministic_bitwise(torch_dev):
    s = synth.random_stack(30, n=6, h=50, w=200, n_vel=40, k=10)
    p1, r1 = run_gpu(torch_dev, s)
    p2, r2 = run_gpu(torch_dev, s)
    assert p1.tobytes() == p2.tobytes()
    for a, b in zip(r1, r2):
        assert a.tobytes() == b.tobytes()


def test_closed_form_on_gpu(torch_dev):
    # Noise-free integer-step source, constant variance: alpha_ML = flux and
    # nu = flux * sqrt(N * S2) / sigma (Sec. 2.1.5).
    n, h, w, flux, sig = 5, 48, 96, 50.0, 1.0
    psf = synth.psf_gaussian(1.0, 7)
    T = psf.astype(np.float64)
    S2 = float((T * T).sum())
    t = np.arange(n) * 0.25
    img = np.zeros((n, h, w), np.float32)
    for i in range(n):
        yi, xi = 30 + int(-4 * t[i]), 20 + int(8 * t[i])
        img[i, yi - 3:yi + 4, xi - 3:xi + 4] = (flux * T).astype(np.float32)
    s = synth.Stack(img, np.ones_like(img), np.zeros(img.shape, np.uint8), t, psf,
                    np.array([[0.0, 0.0], [8.0, -4.0], [4.0, 4.0]]), 3, np.zeros((0, 5)))
    _, (nu, al, vel, nobs) = run_gpu(torch_dev, s)
    assert vel[30, 20, 0] == 1
    expect = flux * math.sqrt(n * S2) / sig
    assert abs(nu[30, 20, 0] - expect) <= 1e-5 * expect
    assert abs(al[30, 20, 0] - flux) <= 1e-5 * flux
    assert nobs[30, 20, 0] == n


def test_noise_nu_standard_normal_on_gpu(torch_dev):
    from scipy import stats
    n, h, w = 4, 256, 256
    rng = np.random.default_rng(77)
    sig = rng.uniform(0.7, 1.4, (n, h, w))
    img = (sig * rng.standard_normal((n, h, w))).astype(np.float32)
    var = (sig ** 2).astype(np.float32)
    mask = (rng.random((n, h, w)) < 0.02).astype(np.uint8)
    vel = np.array([[0.0, 0.0], [13.0, -7.0], [-21.0, 5.5]])
    s = synth.Stack(img, var, mask, np.array([0.0, 0.3, 0.7, 1.1]), synth.psf_gaussian(1.0, 5),
                    vel, 3, np.zeros((0, 5)))
    _, (nu, al, vi, nobs) = run_gpu(torch_dev, s)
    for j in range(3):
        sel = (vi == j)
        vals = np.where(sel, nu, 0.0).sum(-1)[20:236:8, 20:236:8].ravel()
        vals = vals[np.isfinite(vals)]
        m = vals.size
        assert abs(vals.mean()) < 5 / math.sqrt(m)
        assert abs(vals.std() - 1) < 5 / math.sqrt(2 * m)
        assert stats.kstest(vals, "norm").pvalue > 1e-3


@pytest.mark.slow
def test_survey_workload_sampled(torch_dev):
    """15 images of 4096^2, 600 velocities, K = 50, in the launch configuration the
    benchmark times; checked on sampled start pixels the oracle computes one by one."""
    from paper_1901_02492_amd import lib
    import torch
    s = synth.survey_stack()
    _say(f"case {s.name}: generated")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes, res = lib.run_search(img, var, mask, s.t, s.psf, s.vel, s.k)
    torch.cuda.synchronize()
    _say("gpu search done")
    n, h, w = s.img.shape
    rng = np.random.default_rng(5)
    ys = list(rng.integers(0, h, 48)) + [0, 0, h - 1, h - 1, h // 2, 1, h - 2]
    xs = list(rng.integers(0, w, 48)) + [0, w - 1, 0, w - 1, w // 2, w - 2, 1]
    for x0, y0, *_ in s.sources[:16]:
        ys.append(int(round(y0)))
        xs.append(int(round(x0)))
    ys, xs = np.clip(np.array(ys), 0, h - 1), np.clip(np.array(xs), 0, w - 1)
    yt, xt = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    gpu = [r[yt, xt].cpu().numpy() for r in res]
    ref = oracle.search_pixels(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k, ys, xs)
    ntie = parity.check_topk(gpu, ref["all_nu"], ref["all_alpha"], ref["all_nobs"],
                             ref["all_Phi"], ref["vel"], s.k)
    _say(f"sampled {ys.size} pixels, near-tie pixels {ntie}")
    py = rng.integers(0, h, 300)
    px = rng.integers(0, w, 300)
    pyt, pxt = torch.from_numpy(py).to(dev), torch.from_numpy(px).to(dev)
    for i in range(n):
        ps, ph, ok = oracle.psi_phi_at(s.img[i], s.var[i], s.mask[i], s.psf, py, px)
        pg = planes[i][pyt, pxt].cpu().numpy()
        parity.check_planes(pg[None], ps[None], ph[None], ok[None])
