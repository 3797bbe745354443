"""kb_search_noalloc (no workspace; the library's fixed device array holds the
tables) against kb_search with a caller workspace, through the C ABI: the
candidate lists must be bitwise equal, on two calls in a row, the second
with a smaller stack, in float32 and 16-bit planes."""
import sys

import numpy as np
import pytest

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


def _planes(torch, s, lp):
    from paper_1901_02492_amd import lib
    dev = torch.device("cuda:0")
    img, var, mask = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                      for a in (s.img, s.var, s.mask))
    if lp is None:
        return lib.make_psi_phi(img, var, mask, s.psf), None
    _, src, sc = lib.make_psi_phi(img, var, mask, s.psf, lp=lp)
    return src, sc


# (seed, n, h, w, n_vel, k_cand): the first stack is larger than the second in
# every dimension, so the second call finds the first one's tables behind it.
PAIRS = [
    ((71, 20, 300, 1100, 700, 50), (72, 5, 37, 71, 9, 4)),      # 2 table batches, ragged
    ((73, 15, 520, 1000, 600, 50), (74, 3, 64, 130, 40, 17)),   # persistent order first
]


@pytest.mark.parametrize("lp", [None, "f16", "bf16"])
@pytest.mark.parametrize("pair", PAIRS, ids=["ragged", "persistent"])
def test_noalloc_equals_workspace_search(torch_dev, pair, lp):
    from paper_1901_02492_amd import lib
    torch = torch_dev
    for (seed, n, h, w, nv, kc) in pair:
        _say(f"kb_search_noalloc seed={seed} N={n} {h}x{w} V={nv} k_cand={kc} lp={lp}")
        s = synth.random_stack(seed, n=n, h=h, w=w, n_vel=nv, k=kc, psf_size=5,
                               vmax=max(h, w) * 0.6)
        src, sc = _planes(torch, s, lp)
        ref = lib.search(src, s.t, s.vel, kc, lp_scale=sc)
        got = lib.search_noalloc(src, s.t, s.vel, kc, lp_scale=sc)
        torch.cuda.synchronize()
        for a, b in zip(parity.to_numpy(got), parity.to_numpy(ref)):
            assert a.tobytes() == b.tobytes()


def test_noalloc_rejects_stack_beyond_scratch(torch_dev):
    """A stack whose tables exceed the fixed array is refused before anything
    is enqueued (the outputs keep their contents)."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    dev = torch.device("cuda:0")
    n, h, w, nv = 40, 8, 64, 20000      # table stride 48: 20000 * 48 * 16 B > 8 MiB
    planes = torch.zeros((n, h, w, 2), dtype=torch.float32, device=dev)
    t = np.arange(n, dtype=np.float64) * 0.01
    vel = np.stack([np.linspace(-5, 5, nv), np.zeros(nv)], axis=1)
    out = [x.fill_(7) for x in lib.alloc_candidates(h, w, 4, dev)]
    with pytest.raises(lib.KbError) as e:
        lib.search_noalloc(planes, t, vel, 4, out=out)
    assert e.value.status == lib.KB_EUNSUPPORTED
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert all(bool((x == 7).all()) for x in out)
