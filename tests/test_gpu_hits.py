"""The bright-pixel mask (kb_mask_bright, Sec. 5.2) and the HiTS-shaped
workload (Sec. 3.2: 13 images of 4096^2, 32000 velocities) on the GPU,
against the FP64 oracle through the C ABI."""
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


@pytest.mark.parametrize("shape,offset", [((3, 37, 41), 0), ((2, 64, 64), 0), ((1, 1, 1), 0),
                                          ((4, 33, 17), 1), ((2, 16, 16), 3)])
def test_mask_bright_matches_definition(torch_dev, shape, offset):
    """Ragged sizes and (offset > 0) arrays that are not 16-byte aligned, with
    values at the threshold, NaN and infinities; bitwise against the oracle."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    _say(f"case mask_bright shape={shape} offset={offset}")
    rng = np.random.default_rng(sum(shape) + offset)
    n = int(np.prod(shape))
    img = rng.normal(0.0, 3.0, n).astype(np.float32)
    special = rng.choice(n, size=min(n, 12), replace=False)
    img[special] = np.array([5.0, np.nan, np.inf, -np.inf, 5.0000005, 4.9999995, 5.0, 1e30,
                             -1e30, np.nan, 5.0, 6.0], dtype=np.float32)[:special.size]
    mask = (rng.random(n) < 0.1).astype(np.uint8) * rng.integers(1, 255, n).astype(np.uint8)
    img, mask = img.reshape(shape), mask.reshape(shape)
    want = oracle.bright_mask(img, mask, 5.0)
    dev = torch.device("cuda:0")
    ib = torch.zeros(n + offset, dtype=torch.float32, device=dev)
    mb = torch.zeros(n + offset, dtype=torch.uint8, device=dev)
    ti = ib[offset:].view(shape)
    tm = mb[offset:].view(shape)
    ti.copy_(torch.from_numpy(img))
    tm.copy_(torch.from_numpy(mask))
    lib.mask_bright(ti, tm, 5.0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(tm.cpu().numpy(), want)
    assert mb[:offset].cpu().numpy().sum() == 0        # nothing written before the array


@pytest.mark.slow
def test_hits_workload_sampled(torch_dev):
    """13 x 4096^2 with 20000 flashes, 32000 velocities, K = 50, bright mask at
    5 sigma, in the benchmark's launch configuration; sampled start pixels
    against the oracle (bright mask, then the search one pixel at a time)."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.hits_stack()
    n, h, w = s.img.shape
    _say(f"case {s.name}: generated")
    rng = np.random.default_rng(9)
    ys = list(rng.integers(0, h, 6)) + [0, h - 1]
    xs = list(rng.integers(0, w, 6)) + [w - 1, 0]
    for x0, y0, *_ in s.sources[:4]:
        ys.append(int(round(y0)))
        xs.append(int(round(x0)))
    ys, xs = np.clip(np.array(ys), 0, h - 1), np.clip(np.array(xs), 0, w - 1)
    m = oracle.bright_mask(s.img, s.mask, synth.HITS_BRIGHT_SIGMA)
    ref = oracle.search_pixels(s.img, s.var, m, s.t, s.psf, s.vel, s.k, ys, xs)
    _say(f"oracle on {ys.size} pixels done")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    lib.mask_bright(img, mask, synth.HITS_BRIGHT_SIGMA)
    planes, res = lib.run_search(img, var, mask, s.t, s.psf, s.vel, s.k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(mask.cpu().numpy(), m)
    _say("gpu search done")
    yt, xt = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    gpu = [r[yt, xt].cpu().numpy() for r in res]
    ntie = parity.check_topk(gpu, ref["all_nu"], ref["all_alpha"], ref["all_nobs"],
                             ref["all_Phi"], ref["vel"], s.k)
    _say(f"sampled {ys.size} pixels, near-tie pixels {ntie}")
