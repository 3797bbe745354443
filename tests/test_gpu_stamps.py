"""Coadded postage stamps and the moment filter (kb_stamps, Sec. 3.3) against
the FP64 oracle, through the C ABI.  Both sides average and accumulate in
IEEE double in the same order from the same float32 images, so stamps,
moments and decisions must be identical."""
import sys

import numpy as np
import pytest

import oracle
from oracle import cluster as oc
from oracle import stamps as ost
from paper_1901_02492_amd import synth

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


def _records(xs, ys, js):
    from paper_1901_02492_amd import lib
    r = np.zeros(np.size(xs), dtype=lib.HIT_DTYPE)
    r["x"], r["y"], r["vel"] = xs, ys, js
    return r


def _run(torch, s, recs, R, lim, drop=None):
    from paper_1901_02492_amd import lib
    dev = torch.device("cuda:0")
    img = torch.from_numpy(np.ascontiguousarray(s.img)).to(dev)
    var = torch.from_numpy(np.ascontiguousarray(s.var)).to(dev)
    mask = torch.from_numpy(np.ascontiguousarray(s.mask)).to(dev)
    cand = torch.from_numpy(recs.view(np.int32).reshape(-1, 6).copy()).to(dev)
    d = None if drop is None else torch.from_numpy(drop.view(np.int64).copy()).to(dev)
    ok, mom, st = lib.stamps(img, var, mask, s.t, s.vel, cand, recs.size, R, *lim, drop=d)
    torch.cuda.synchronize()
    return ok.cpu().numpy(), mom.cpu().numpy(), st.cpu().numpy()


def _oracle(s, xs, ys, js, R, lim, keep=None):
    S = ost.coadd_stamps(s.img, s.var, s.mask, s.t, s.vel, xs, ys, js, R, keep)
    mom = ost.moments(S)
    return ost.stamp_filter(mom, *lim), np.stack(mom, axis=1), S


def _compare(got, want):
    ok, mom, st = got
    ok_o, mom_o, S_o = want
    np.testing.assert_array_equal(st, S_o.astype(np.float32))
    np.testing.assert_array_equal(mom, mom_o)            # NaN where M00 = 0 on both
    np.testing.assert_array_equal(ok.astype(bool), ok_o)


LIM = (1.0, 1.0, 0.5, 4.0)     # max_offset, max_m11, m2_min, m2_max


@pytest.mark.parametrize("R", [0, 3, 5])
def test_stamps_identical_to_oracle(torch_dev, R):
    s = synth.random_stack(71, 15, 48, 70, 30, 4, n_flash=30, psf_sigma=1.2)
    s.img[2, 10, 10] = np.nan                    # non-finite image pixel
    s.var[4, 20, 30] = 0.0                       # non-positive variance
    n, h, w = s.img.shape
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, 1)
    ys, xs, js = oc.threshold_hits(ref["all_nu"], 3.0)
    rng = np.random.default_rng(R)
    xr, yr = rng.integers(0, w, 200), rng.integers(0, h, 200)
    jr = rng.integers(0, s.vel.shape[0], 200)
    xs, ys, js = np.concatenate([xs, xr, [0, w - 1]]), np.concatenate([ys, yr, [0, h - 1]]), \
        np.concatenate([js, jr, [0, 1]])
    _say(f"case stamps R={R}: {xs.size} candidates")
    got = _run(torch_dev, s, _records(xs, ys, js), R, LIM)
    want = _oracle(s, xs, ys, js, R, LIM)
    _compare(got, want)
    _say(f"  {int(got[0].sum())} pass")
    assert (got[0] == 0).sum() > 0
    if R >= 3:                       # a single pixel has no spread: nothing passes at R = 0
        assert got[0].sum() > 0


def test_stamps_with_drop_masks(torch_dev):
    s = synth.random_stack(72, 12, 40, 56, 20, 4, n_flash=20)
    n, h, w = s.img.shape
    rng = np.random.default_rng(3)
    c = 300
    xs, ys, js = rng.integers(0, w, c), rng.integers(0, h, c), rng.integers(0, 20, c)
    keep = rng.random((c, n)) > 0.3
    keep[:5] = False                                          # nothing kept
    drop = ((~keep).astype(np.uint64) << np.arange(n, dtype=np.uint64)).sum(axis=1,
                                                                           dtype=np.uint64)
    got = _run(torch_dev, s, _records(xs, ys, js), 4, LIM, drop=drop)
    want = _oracle(s, xs, ys, js, 4, LIM, keep)
    _compare(got, want)
    assert np.isnan(got[1][:5, 1]).all() and (got[0][:5] == 0).all()


def test_stamps_out_of_grid_velocity(torch_dev):
    s = synth.small_stack()
    got = _run(torch_dev, s, _records([5, 6], [5, 6], [-1, 121]), 2, LIM)
    assert (got[2] == 0).all() and np.isnan(got[1][:, 1:]).all() and (got[0] == 0).all()


@pytest.mark.slow
def test_stamps_survey_size(torch_dev):
    """1000 seeded candidates on the full survey stack (15 x 4096^2), R = 5."""
    s = synth.survey_stack()
    n, h, w = s.img.shape
    rng = np.random.default_rng(12)
    c = 1000
    xs, ys, js = rng.integers(0, w, c), rng.integers(0, h, c), rng.integers(0, 600, c)
    src = s.sources[:20]
    xs[:20], ys[:20] = np.clip(np.round(src[:, 0]), 0, w - 1), np.clip(np.round(src[:, 1]), 0, h - 1)
    vel_src = np.argmin(((s.vel[None, :, :] - src[:, None, 2:4]) ** 2).sum(axis=2), axis=1)
    js[:20] = vel_src
    got = _run(torch_dev, s, _records(xs, ys, js), 5, (1.0, 1.0, 0.5, 6.0))
    want = _oracle(s, xs, ys, js, 5, (1.0, 1.0, 0.5, 6.0))
    _compare(got, want)
    _say(f"survey stamps: {int(got[0].sum())} of {c} pass; injected sources "
         f"{int(got[0][:20].sum())} of 20")
