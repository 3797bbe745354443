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


def test_persistent_order_ragged_frame(torch_dev):
    """A frame large enough for the persistent tile order (several generations
    of blocks at K' = 50) with a ragged width and height, so that blocks
    overhang the right and bottom edges: every start pixel is compared with
    the oracle."""
    s = synth.random_stack(21, n=8, h=520, w=1000, n_vel=60, k=50, psf_size=5, vmax=60.0)
    _full_check(torch_dev, s)


def test_concurrent_persistent_searches(torch_dev):
    """Two searches large enough for the persistent order, launched on two
    streams at once, compete for wave slots (so their per-XCD pacing waits can
    time out); each must still return exactly what it returns alone."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    dev = torch.device("cuda:0")
    s = synth.random_stack(21, n=8, h=520, w=1000, n_vel=60, k=50, psf_size=5, vmax=60.0)
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes = lib.make_psi_phi(img, var, mask, s.psf)
    n, h, w = s.img.shape
    alone = parity.to_numpy(lib.search(planes, s.t, s.vel, 50))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=dev) for _ in range(2)]
    outs = []
    for st in streams:
        with torch.cuda.stream(st):
            ws = lib.alloc_workspace(n, h, w, s.vel.shape[0], dev)
            outs.append((lib.search(planes, s.t, s.vel, 50, workspace=ws), ws))
    torch.cuda.synchronize()
    for res, _ in outs:
        for a, b in zip(parity.to_numpy(res), alone):
            assert np.array_equal(a, b)


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
    s, ys, xs, ref = _survey_sampled_reference()
    _say(f"case {s.name}: generated, oracle on {ys.size} pixels done")
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes, res = lib.run_search(img, var, mask, s.t, s.psf, s.vel, s.k)
    torch.cuda.synchronize()
    _say("gpu search done")
    n, h, w = s.img.shape
    rng = np.random.default_rng(6)
    yt, xt = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    gpu = [r[yt, xt].cpu().numpy() for r in res]
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


_SURVEY = {}


def _survey_sampled_reference():
    """The survey stack, its sampled start pixels and their oracle results
    (computed once per test session)."""
    if not _SURVEY:
        s = synth.survey_stack()
        n, h, w = s.img.shape
        rng = np.random.default_rng(5)
        ys = list(rng.integers(0, h, 48)) + [0, 0, h - 1, h - 1, h // 2, 1, h - 2]
        xs = list(rng.integers(0, w, 48)) + [0, w - 1, 0, w - 1, w // 2, w - 2, 1]
        for x0, y0, *_ in s.sources[:16]:
            ys.append(int(round(y0)))
            xs.append(int(round(x0)))
        ys, xs = np.clip(np.array(ys), 0, h - 1), np.clip(np.array(xs), 0, w - 1)
        ref = oracle.search_pixels(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k, ys, xs)
        _SURVEY.update(stack=s, ys=ys, xs=xs, ref=ref)
    return _SURVEY["stack"], _SURVEY["ys"], _SURVEY["xs"], _SURVEY["ref"]


def _errors(nu, al, vel, ref):
    """|nu - nu_o| / max(1, |nu_o|) and |alpha - alpha_o| / max(|alpha_o|, 1/sqrt(Phi_o))
    of every finite entry against the oracle's score of the same trajectory."""
    p = np.arange(vel.shape[0])[:, None]
    nu_o = ref["all_nu"][vel, p]            # oracle scores are [velocity][pixel]
    al_o = ref["all_alpha"][vel, p]
    phi_o = ref["all_Phi"][vel, p]
    fin = np.isfinite(nu_o) & np.isfinite(nu)
    e_nu = np.abs(nu.astype(np.float64) - nu_o)[fin] / np.maximum(1.0, np.abs(nu_o[fin]))
    scale = np.maximum(np.abs(al_o[fin]), 1.0 / np.sqrt(phi_o[fin]))
    e_al = np.abs(al.astype(np.float64) - al_o)[fin] / scale
    return e_nu, e_al


@pytest.mark.slow
@pytest.mark.parametrize("lp", ["f16", "bf16"])
def test_survey_precision_mode_sampled(torch_dev, lp):
    """Precision mode on the survey stack (15 x 4096^2, 600 velocities, K = 50):
    16-bit planes searched with the mode's K' (50 for FP16, 52 for BF16) and
    with 64 candidates, then re-scored in FP32.  On the sampled start pixels: nu/alpha error against the FP64
    oracle before and after the re-score, and recall of the top-K (an entry
    counts when the oracle ranks it in its top K or within the nu tolerance
    of its K-th value).  Recall is statistical (parity unpinned), measured."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s, ys, xs, ref = _survey_sampled_reference()
    n, h, w = s.img.shape
    dev = torch.device("cuda:0")
    img = torch.from_numpy(s.img).to(dev)
    var = torch.from_numpy(s.var).to(dev)
    mask = torch.from_numpy(s.mask).to(dev)
    planes, src, sc = lib.make_psi_phi(img, var, mask, s.psf, lp=lp)
    del img, var, mask
    ws = lib.alloc_workspace(n, h, w, s.vel.shape[0], dev)
    yt, xt = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    kth = ref["nu"][:, s.k - 1].astype(np.float64)
    # bench.py's K': K for FP16, K + 2 for BF16
    for kc in (s.k if lp == "f16" else s.k + 2, 64):
        cand = lib.search(src, s.t, s.vel, kc, workspace=ws, lp_scale=sc)
        res = lib.topk(cand, s.k, n, rescore=(planes, s.t, s.vel, ws))
        torch.cuda.synchronize()
        c = [a[yt, xt].cpu().numpy() for a in cand]
        r = [a[yt, xt].cpu().numpy() for a in res]
        del cand, res
        b_nu, b_al = _errors(c[0], c[1], c[2], ref)
        a_nu, a_al = _errors(r[0], r[1], r[2], ref)
        hits = 0
        for p in range(ys.size):
            top = set(ref["vel"][p].tolist())
            lim = kth[p] - parity.tol_nu(kth[p])
            hits += sum(1 for j in r[2][p] if j in top or ref["all_nu"][j, p] >= lim)
        recall = hits / (ys.size * s.k)
        _say(f"precision {lp} K'={kc}: before re-score nu err max {b_nu.max():.2e} "
             f"p99 {np.quantile(b_nu, 0.99):.2e}, alpha err max {b_al.max():.2e} "
             f"p99 {np.quantile(b_al, 0.99):.2e}; after re-score nu err max "
             f"{a_nu.max():.2e}, alpha err max {a_al.max():.2e}; recall {recall:.5f}")
        assert a_nu.max() <= 1e-5 and a_al.max() <= 1e-5
        assert np.array_equal(r[3], ref["all_nobs"][r[2], np.arange(ys.size)[:, None]])
        assert recall >= 0.999


@pytest.mark.parametrize("kc,k", [(50, 50), (50, 17), (64, 64), (7, 3), (1, 1)])
def test_topk_orders_shuffled_candidates(torch_dev, kc, k):
    """kb_topk must order any candidate set (not only kb_search's ranked lists):
    shuffle each pixel's candidates, plant exact nu ties, and compare with a
    host sort by (nu descending, index ascending)."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    rng = np.random.default_rng(kc * 100 + k)
    h, w = 37, 53
    nu = rng.standard_normal((h, w, kc)).astype(np.float32)
    nu[..., ::3] = np.round(nu[..., ::3])           # many exact ties
    nu[rng.random(nu.shape) < 0.05] = -np.inf
    vel = np.argsort(rng.random((h, w, 4 * kc)), axis=-1)[..., :kc].astype(np.int32)
    al = rng.standard_normal((h, w, kc)).astype(np.float32)
    no = rng.integers(0, 30, (h, w, kc)).astype(np.int16)
    dev = torch.device("cuda:0")
    cand = [torch.from_numpy(a).to(dev) for a in (nu, al, vel, no)]
    out = parity.to_numpy(lib.topk(cand, k, 5))
    torch.cuda.synchronize()
    order = np.lexsort((vel, -nu.astype(np.float64)), axis=-1)[..., :k]
    for got, src in zip(out, (nu, al, vel, no)):
        assert np.array_equal(got, np.take_along_axis(src, order, -1))


@pytest.mark.parametrize("kc,k,in_place", [(50, 50, True), (50, 20, False), (8, 8, False)])
def test_topk_repeated_velocity_keeps_list_order(torch_dev, kc, k, in_place):
    """Entries equal in nu and velocity index (a list that repeats a
    velocity, which kb_search never writes) rank in list order: the result
    equals a stable host sort by (nu descending, index ascending), alpha and
    n_obs moving with their entry."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    rng = np.random.default_rng(kc + k)
    h, w = 19, 23
    nu = np.round(rng.standard_normal((h, w, kc))).astype(np.float32)
    vel = rng.integers(0, 4, (h, w, kc)).astype(np.int32)     # many repeats
    al = rng.standard_normal((h, w, kc)).astype(np.float32)
    no = rng.integers(0, 30, (h, w, kc)).astype(np.int16)
    dev = torch.device("cuda:0")
    cand = [torch.from_numpy(a).to(dev) for a in (nu, al, vel, no)]
    out = parity.to_numpy(lib.topk(cand, k, 5, out=cand if in_place else None))
    torch.cuda.synchronize()
    order = np.lexsort((vel, -nu.astype(np.float64)), axis=-1)[..., :k]
    for got, src in zip(out, (nu, al, vel, no)):
        assert np.array_equal(got, np.take_along_axis(src, order, -1))


@pytest.mark.parametrize("kc", [50, 64, 7, 1])
def test_topk_in_place(torch_dev, kc):
    """kb_topk with the candidate arrays as outputs (k == k_cand): kb_search's
    lists come back unchanged and equal to the out-of-place result, and
    shuffled lists (exact nu ties, -inf entries) are put in rank order in
    place, as a host sort by (nu descending, index ascending) orders them."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    dev = torch.device("cuda:0")
    s = synth.random_stack(90 + kc, n=6, h=41, w=75, n_vel=max(kc, 70), k=kc, psf_size=5,
                           vmax=75.0)
    img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
    planes = lib.make_psi_phi(img, var, mask, s.psf)
    cand = lib.search(planes, s.t, s.vel, kc)
    before = [a.clone() for a in cand]
    copied = lib.topk(cand, kc, 6)
    lib.topk(cand, kc, 6, out=cand)
    torch.cuda.synchronize()
    for a, b, c in zip(parity.to_numpy(cand), parity.to_numpy(before), parity.to_numpy(copied)):
        assert a.tobytes() == b.tobytes() == c.tobytes()
    rng = np.random.default_rng(kc)
    h, w = 37, 53
    nu = rng.standard_normal((h, w, kc)).astype(np.float32)
    nu[..., ::3] = np.round(nu[..., ::3])
    nu[rng.random(nu.shape) < 0.05] = -np.inf
    nu[:5] = np.sort(nu[:5], axis=-1)[..., ::-1]        # some rows already ordered
    vel = np.argsort(rng.random((h, w, 4 * kc)), axis=-1)[..., :kc].astype(np.int32)
    vel[:5] = np.sort(vel[:5], axis=-1)
    al = rng.standard_normal((h, w, kc)).astype(np.float32)
    no = rng.integers(0, 30, (h, w, kc)).astype(np.int16)
    c2 = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (nu, al, vel, no)]
    lib.topk(c2, kc, 5, out=c2)
    torch.cuda.synchronize()
    order = np.lexsort((vel, -nu.astype(np.float64)), axis=-1)
    for got, src in zip(parity.to_numpy(c2), (nu, al, vel, no)):
        assert np.array_equal(got, np.take_along_axis(src, order, -1))


# --- precision mode: scaled 16-bit planes, FP32 re-score ---------------------

def _bf16_rne(x):
    """float32 -> bfloat16 bits, round to nearest even (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("lp", ["f16", "bf16"])
def test_lp_planes_encoding(torch_dev, lp):
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.random_stack(41, n=5, h=33, w=70, n_vel=4, k=2, mask_frac=0.1)
    s.var[2] *= 1e4                      # a much fainter image gets its own scale
    dev = torch.device("cuda:0")
    img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
    planes, lpp, scale = lib.make_psi_phi(img, var, mask, s.psf, lp=lp)
    torch.cuda.synchronize()
    f32 = planes.cpu().numpy()
    bits = lpp.view(torch.int16).cpu().numpy().view(np.uint16)
    sc = scale.cpu().numpy()
    valid = f32[..., 1].view(np.uint32) != 0
    for i in range(5):
        for c in range(2):
            m, e = np.frexp(sc[i, c])
            assert m == 0.5, "scale must be a power of two"
            amax = np.abs(f32[i, ..., c][valid[i]]).max()
            assert 2.0 ** 13 <= amax * sc[i, c] < 2.0 ** 14
            scaled = (f32[i, ..., c] * sc[i, c]).astype(np.float32)
            want = (scaled.astype(np.float16).view(np.uint16) if lp == "f16"
                    else _bf16_rne(scaled))
            if c == 1:
                want = np.where((want & 0x7FFF) == 0, np.uint16(0x8000), want)
            want = np.where(valid[i], want, np.uint16(0))
            assert np.array_equal(bits[i, ..., c], want)
    assert sc[2, 1] > sc[0, 1] * 1e3


RESCORE_CASES = [
    # (seed, n_img, h, w, n_vel, k_cand, k): ragged tiles, odd list lengths,
    # more velocities than counting-sort bins, the longest list, one pixel.
    (81, 7, 37, 101, 50, 33, 20),
    (82, 3, 5, 13, 1500, 64, 64),
    (83, 15, 130, 300, 600, 50, 50),
    (84, 4, 64, 64, 64, 64, 9),
    (85, 2, 1, 1, 1, 1, 1),
]


@pytest.mark.parametrize("case", RESCORE_CASES, ids=lambda c: "x".join(map(str, c[1:])))
def test_rescore_of_plain_candidates_equals_topk(torch_dev, case):
    """kb_topk with re-scoring, given the candidates of a float32 search,
    recomputes exactly the values the search wrote (same planes, same
    arithmetic), so its output equals plain kb_topk's bit for bit.  A
    candidate index outside the grid ranks last with nu = -inf, alpha = 0,
    n_obs = 0 and its index kept."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    seed, n, h, w, nv, kc, k = case
    s = synth.random_stack(seed, n=n, h=h, w=w, n_vel=nv, k=k, psf_size=5, vmax=max(h, w))
    _say(f"case rescore seed={seed} N={n} HxW={h}x{w} V={nv} k_cand={kc} k={k}")
    dev = torch.device("cuda:0")
    img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
    planes = lib.make_psi_phi(img, var, mask, s.psf)
    ws = lib.alloc_workspace(n, h, w, nv, dev)
    cand = lib.search(planes, s.t, s.vel, kc, workspace=ws)
    plain = lib.topk(cand, k, n)
    again = lib.topk(cand, k, n, rescore=(planes, s.t, s.vel, ws))
    full = lib.topk(cand, kc, n, rescore=(planes, s.t, s.vel, ws))
    torch.cuda.synchronize()
    for a, b in zip(parity.to_numpy(plain), parity.to_numpy(again)):
        assert np.ascontiguousarray(a).tobytes() == np.ascontiguousarray(b).tobytes()
    # Corrupt one candidate index per pixel on a stride of pixels.
    full = [np.ascontiguousarray(a).reshape(h * w, kc) for a in parity.to_numpy(full)]
    cv = cand[2].clone().reshape(h * w, kc)
    pix = np.arange(0, h * w, 3)
    slot = (pix * 7) % kc
    bad = np.where(pix % 2 == 0, -1, nv).astype(np.int32)
    pt, st = torch.from_numpy(pix).to(dev), torch.from_numpy(slot).to(dev)
    cv[pt, st] = torch.from_numpy(bad).to(dev)
    cand2 = (cand[0], cand[1], cv.reshape(h, w, kc), cand[3])
    got = lib.topk(cand2, kc, n, rescore=(planes, s.t, s.vel, ws))
    torch.cuda.synchronize()
    got = [np.ascontiguousarray(a).reshape(h * w, kc) for a in parity.to_numpy(got)]
    cv_host = cand[2].reshape(h * w, kc).cpu().numpy()
    for q, p in enumerate(pix):
        lost = cv_host[p, slot[q]]
        keep = full[2][p] != lost
        for fg, ff in zip(got, full):
            assert np.array_equal(fg[p, :kc - 1].view(np.uint8), ff[p, keep].view(np.uint8))
        assert got[0][p, -1] == -np.inf and got[1][p, -1] == 0.0
        assert got[2][p, -1] == bad[q] and got[3][p, -1] == 0
    rest = np.setdiff1d(np.arange(h * w), pix)
    for fg, ff in zip(got, full):
        assert np.array_equal(fg[rest].view(np.uint8), ff[rest].view(np.uint8))


LP_BAND = {"f16": 1e-2, "bf16": 8e-2}   # nu band for near-ties after 16-bit pre-selection


@pytest.mark.parametrize("lp", ["f16", "bf16"])
@pytest.mark.parametrize("which", ["small", "random"])
def test_lp_search_rescored(torch_dev, lp, which):
    """16-bit search + FP32 re-score: every kept value meets the FP32 tolerances
    against the oracle, equals the plain FP32 path bitwise for the same
    trajectory, and the kept set matches the oracle's up to near-ties within
    the 16-bit rounding band."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.small_stack() if which == "small" else synth.random_stack(
        42, n=9, h=40, w=90, n_vel=60, k=8, psf_size=5, vmax=40.0)
    k = s.k
    kc = min(s.vel.shape[0], k + 16)
    dev = torch.device("cuda:0")
    img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
    _, plain = lib.run_search(img, var, mask, s.t, s.psf, s.vel, k)
    _, got = lib.run_search(img, var, mask, s.t, s.psf, s.vel, k, k_cand=kc, lp=lp)
    torch.cuda.synchronize()
    plain = parity.to_numpy(plain)
    got = parity.to_numpy(got)
    H, W = s.img.shape[1:]
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, k)
    all_nu, all_al, all_no, all_phi, top = parity.oracle_full_as_pixels(ref)
    g = [a.reshape(H * W, k) for a in got]
    p = [a.reshape(H * W, k) for a in plain]
    # values of every kept trajectory (FP32 tolerances, exact n_obs)
    nu_g, al_g, j_g, n_g = g
    pidx = np.arange(H * W)[:, None]
    nu_o = all_nu[j_g, pidx]
    fin = np.isfinite(nu_o)
    assert np.all(n_g == all_no[j_g, pidx])
    assert np.all(np.abs(nu_g - nu_o)[fin] <= parity.tol_nu(nu_o)[fin])
    # bitwise equal to the plain FP32 path where both keep the same trajectory
    for a in range(k):
        for b in range(k):
            same = j_g[:, a] == p[2][:, b]
            for fg, fp in zip(g, p):
                assert np.array_equal(fg[same, a].view(np.uint8), fp[same, b].view(np.uint8))
    # ordered, and the set equals the oracle's up to near-ties within the band
    with np.errstate(invalid="ignore"):
        a_, b_ = nu_g[:, :-1], nu_g[:, 1:]
        assert np.all((a_ > b_) | ((a_ == b_) & (j_g[:, :-1] < j_g[:, 1:])))
        nu_k = all_nu[top[:, k - 1], np.arange(H * W)]
        band = np.where(np.isfinite(nu_k), LP_BAND[lp] * np.maximum(1, np.abs(nu_k)), 0.0)
        in_ref = (j_g[:, :, None] == top[:, None, :]).any(-1)
        assert np.all(in_ref | (nu_o >= (nu_k - band)[:, None]))
        in_gpu = (top[:, :, None] == j_g[:, None, :]).any(-1)
        assert np.all(in_gpu | (all_nu[top, pidx] <= (nu_k + band)[:, None]))
        # tie-tolerant recall: a kept entry counts when the oracle ranks it in
        # its top k or within the nu tolerance of its k-th value
        recall = (in_ref | (nu_o >= (nu_k - parity.tol_nu(nu_k))[:, None])).mean()
    _say(f"{lp} {which}: recall {recall:.5f} (exact membership {in_gpu.mean():.5f})")
    assert recall >= 0.999


@pytest.mark.parametrize("lp", [None, "f16", "bf16"])
def test_shorter_list_is_prefix_of_longer(torch_dev, lp):
    """kb_search's rank-ordered list for k_cand = 8 must equal, bit for bit, the
    first 8 entries of the list for k_cand = 40 (different list lengths,
    different merge schedules), including pixels full of exact ties at the
    frame edges."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.random_stack(51, n=6, h=60, w=130, n_vel=96, k=8, psf_size=5, vmax=60.0)
    dev = torch.device("cuda:0")
    img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
    if lp is None:
        src, sc = lib.make_psi_phi(img, var, mask, s.psf), None
    else:
        _, src, sc = lib.make_psi_phi(img, var, mask, s.psf, lp=lp)
    with_census = lib.search(src, s.t, s.vel, 8, lp_scale=sc)
    without = lib.search(src, s.t, s.vel, 40, lp_scale=sc)
    torch.cuda.synchronize()
    for a, b in zip(parity.to_numpy(with_census), parity.to_numpy(without)):
        assert np.ascontiguousarray(a).tobytes() == np.ascontiguousarray(b[..., :8]).tobytes()


@pytest.mark.parametrize("lp", [None, "f16"])
def test_batched_search_equals_solo(torch_dev, lp):
    """kb_search_batch over stacks of uneven size (images, frame, velocities)
    must give every stack exactly (bitwise) what kb_search gives it alone."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    dev = torch.device("cuda:0")
    k = 6
    shapes = [(5, 40, 70, 30), (17, 33, 130, 50), (3, 64, 64, 12), (9, 1, 200, 20),
              (1, 20, 20, 7), (12, 50, 90, 64)]
    jobs, solos = [], []
    for q, (n, h, w, nv) in enumerate(shapes):
        s = synth.random_stack(60 + q, n=n, h=h, w=w, n_vel=nv, k=k, psf_size=5, vmax=max(h, w))
        img, var, mask = (torch.from_numpy(a).to(dev) for a in (s.img, s.var, s.mask))
        if lp is None:
            src, sc = lib.make_psi_phi(img, var, mask, s.psf), None
        else:
            _, src, sc = lib.make_psi_phi(img, var, mask, s.psf, lp=lp)
        solos.append(lib.search(src, s.t, s.vel, k, lp_scale=sc))
        out = lib.alloc_candidates(h, w, k, dev)
        jobs.append(dict(planes=src, t=s.t, vel=s.vel, out=out, lp_scale=sc))
    lib.search_batch(jobs, k)
    torch.cuda.synchronize()
    for jb, solo in zip(jobs, solos):
        for a, b in zip(parity.to_numpy(jb["out"]), parity.to_numpy(solo)):
            assert a.tobytes() == b.tobytes()
