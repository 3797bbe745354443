"""Threshold mode (kb_search_threshold) and duplicate clustering
(kb_cluster_hits) against the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
from oracle import cluster as oc
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


def _gpu_threshold(torch, s, m, cap=1 << 16):
    from paper_1901_02492_amd import lib
    dev = torch.device("cuda:0")
    img = torch.from_numpy(np.ascontiguousarray(s.img)).to(dev)
    var = torch.from_numpy(np.ascontiguousarray(s.var)).to(dev)
    mask = torch.from_numpy(np.ascontiguousarray(s.mask)).to(dev)
    planes = lib.make_psi_phi(img, var, mask, s.psf)
    hits = lib.alloc_hits(cap, dev)
    cnt = lib.search_threshold(planes, s.t, s.vel, m, hits)
    torch.cuda.synchronize()
    n = int(cnt.item())
    return planes, hits, n, lib.hits_to_numpy(hits, min(n, cap))


def _check_hits(h, ref, m):
    """GPU hits against the oracle's scores: every stored hit is a trajectory
    with the oracle's nu >= m up to the float tolerance, with matching
    scores; every oracle hit clear of the threshold is stored."""
    all_nu, all_al, all_no, all_phi = ref["all_nu"], ref["all_alpha"], ref["all_nobs"], ref["all_Phi"]
    keys = set(zip(h["y"].tolist(), h["x"].tolist(), h["vel"].tolist()))
    assert len(keys) == h.size                               # no trajectory twice
    nu_o = all_nu[h["vel"], h["y"], h["x"]]
    tol = parity.tol_nu(m)
    assert (nu_o >= m - tol).all()
    e_nu = np.abs(h["nu"].astype(np.float64) - nu_o) / np.maximum(1.0, np.abs(nu_o))
    assert e_nu.max() <= 1e-5
    al_o = all_al[h["vel"], h["y"], h["x"]]
    scale = np.maximum(np.abs(al_o), 1.0 / np.sqrt(all_phi[h["vel"], h["y"], h["x"]]))
    assert (np.abs(h["alpha"].astype(np.float64) - al_o) / scale).max() <= 1e-5
    np.testing.assert_array_equal(h["nobs"], all_no[h["vel"], h["y"], h["x"]])
    js, ys, xs = np.nonzero(all_nu >= m + tol)
    missing = set(zip(ys.tolist(), xs.tolist(), js.tolist())) - keys
    assert not missing, f"{len(missing)} clear hits missing"
    return len(keys)


CASES = [("small", lambda: synth.small_stack(), 5.0),
         ("random_a", lambda: synth.random_stack(61, 12, 70, 90, 40, 4), 4.0),
         ("random_ragged", lambda: synth.random_stack(62, 20, 33, 130, 30, 4), 3.5),
         ("random_n33", lambda: synth.random_stack(63, 33, 24, 50, 12, 4), 3.0)]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_threshold_hits_match_oracle(torch_dev, case):
    name, make, m = case
    s = make()
    _say(f"case threshold {name}: N={s.img.shape[0]} HxW={s.img.shape[1]}x{s.img.shape[2]} "
         f"V={s.vel.shape[0]} m={m}")
    _, _, n, h = _gpu_threshold(torch_dev, s, m)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, 1)
    assert n == h.size
    got = _check_hits(h, ref, m)
    _say(f"  {got} hits")
    assert got > 0


def test_threshold_scores_equal_topk_scores(torch_dev):
    """The two search modes give the same trajectory bitwise the same nu,
    alpha and n_obs."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.random_stack(64, 15, 40, 72, 48, 4)
    planes, hits, n, h = _gpu_threshold(torch, s, 2.5)
    cand = lib.search(planes, s.t, s.vel, s.vel.shape[0])     # every velocity kept
    torch.cuda.synchronize()
    nu, al, vi, no = (c.cpu().numpy() for c in cand)
    assert n > 100
    for r in h:
        slot = int(np.nonzero(vi[r["y"], r["x"]] == r["vel"])[0][0])
        assert nu[r["y"], r["x"], slot] == r["nu"]
        assert al[r["y"], r["x"], slot] == r["alpha"]
        assert no[r["y"], r["x"], slot] == r["nobs"]


def test_threshold_overflow_counts_everything(torch_dev):
    s = synth.small_stack()
    _, _, n_all, h_all = _gpu_threshold(torch_dev, s, 4.0)
    _, _, n, h = _gpu_threshold(torch_dev, s, 4.0, cap=37)
    assert n == n_all and n > 37 and h.size == 37
    full = set(zip(h_all["y"].tolist(), h_all["x"].tolist(), h_all["vel"].tolist()))
    part = set(zip(h["y"].tolist(), h["x"].tolist(), h["vel"].tolist()))
    assert len(part) == 37 and part <= full


def _upload_hits(torch, recs):
    from paper_1901_02492_amd import lib
    raw = np.ascontiguousarray(recs.astype(lib.HIT_DTYPE)).view(np.int32).reshape(-1, 6)
    return torch.from_numpy(raw.copy()).to(torch.device("cuda:0"))


def _oracle_records(ys, xs, js, nu):
    from paper_1901_02492_amd import lib
    r = np.zeros(ys.size, dtype=lib.HIT_DTYPE)
    r["x"], r["y"], r["vel"] = xs, ys, js
    r["nu"] = nu.astype(np.float32)
    return r


@pytest.mark.parametrize("s_eps", [(0.2, 2.5), (1.0, 4.0), (0.0, 1.5)])
def test_cluster_matches_oracle_in_any_order(torch_dev, s_eps):
    """Hits from the oracle's own threshold search, clustered on the GPU, in
    the oracle's order and shuffled: each hit's representative is the
    oracle's (compared by trajectory, since indices move with the order)."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    scale, eps = s_eps
    s = synth.random_stack(65, 10, 64, 64, 60, 4)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, 1)
    ys, xs, js = oc.threshold_hits(ref["all_nu"], 3.0)
    nu32 = ref["all_nu"][js, ys, xs].astype(np.float32)
    rep_o, lab = oc.cluster(xs, ys, js, nu32, s.vel, scale, eps)
    ident = lambda idx, yy, xx, jj: list(zip(yy[idx].tolist(), xx[idx].tolist(), jj[idx].tolist()))
    want = ident(rep_o, ys, xs, js)
    _say(f"case cluster s={scale} eps={eps}: {ys.size} hits, {len(set(lab.tolist()))} groups")
    assert ys.size > 200 and 1 < len(set(lab.tolist())) < ys.size
    recs = _oracle_records(ys, xs, js, nu32)
    for trial in range(3):
        perm = np.arange(ys.size) if trial == 0 else np.random.default_rng(trial).permutation(ys.size)
        d = _upload_hits(torch, recs[perm])
        rep = lib.cluster_hits(d, ys.size, s.vel, scale, eps)
        torch.cuda.synchronize()
        rep = rep.cpu().numpy().astype(np.int64)
        got = ident(rep, ys[perm], xs[perm], js[perm])
        assert got == [want[p] for p in perm]


def test_cluster_random_points_with_long_chains(torch_dev):
    """5000 random hits with many chains and ties in nu, against the oracle."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    rng = np.random.default_rng(66)
    n = 5000
    vel = rng.uniform(-20.0, 20.0, (300, 2))
    ys, xs, js = rng.integers(0, 200, n), rng.integers(0, 200, n), rng.integers(0, 300, n)
    key = np.unique(np.stack([ys, xs, js], 1), axis=0)           # distinct trajectories
    ys, xs, js = key[:, 0], key[:, 1], key[:, 2]
    nu32 = rng.choice(np.array([5.0, 6.0, 7.5, 9.0], dtype=np.float32), ys.size)
    rep_o, lab = oc.cluster(xs, ys, js, nu32, vel, 0.15, 3.3)
    _say(f"case cluster random: {ys.size} hits, {len(set(lab.tolist()))} groups")
    d = _upload_hits(torch, _oracle_records(ys, xs, js, nu32))
    rep = lib.cluster_hits(d, ys.size, vel, 0.15, 3.3).cpu().numpy()
    np.testing.assert_array_equal(rep, rep_o)     # same order: same indices


@pytest.mark.parametrize("n,eps,s", [(200_000, 4.0, 2.24), (300_000, 2.0, 0.5)])
def test_cluster_many_hits_against_sparse_oracle(torch_dev, n, eps, s):
    """Hundreds of thousands of hits (survey-sized frame and velocity grid,
    clumps of nearby trajectories around random centres, ties in nu, a few
    indices outside the grid) against the oracle's k-d tree clustering: every
    hit's representative index is the oracle's."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    rng = np.random.default_rng(67 + n)
    vel = synth.survey_velocities(25, 24)
    nc = n // 20
    cx, cy = rng.integers(0, 4096, nc), rng.integers(0, 4096, nc)
    cj = rng.integers(0, vel.shape[0], nc)
    pick = rng.integers(0, nc, n)
    xs = np.clip(cx[pick] + rng.integers(-6, 7, n), 0, 4095)
    ys = np.clip(cy[pick] + rng.integers(-6, 7, n), 0, 4095)
    js = np.clip(cj[pick] + rng.integers(-2, 3, n), 0, vel.shape[0] - 1)
    key = np.unique(np.stack([ys, xs, js], 1), axis=0)           # distinct trajectories
    key = key[rng.permutation(key.shape[0])]
    ys, xs, js = key[:, 0], key[:, 1], key[:, 2].copy()
    js[:7] = [-1, vel.shape[0], 70000, -5, vel.shape[0] + 3, -1, 99999]
    nu32 = rng.choice(np.array([10.0, 11.5, 12.0, 20.0], dtype=np.float32), ys.size)
    rep_o, lab = oc.cluster_sparse(xs, ys, js, nu32, vel, s, eps)
    _say(f"case cluster many: {ys.size} hits, {len(set(lab.tolist()))} groups, "
         f"s={s} eps={eps}")
    d = _upload_hits(torch, _oracle_records(ys, xs, js, nu32))
    rep = lib.cluster_hits(d, ys.size, vel, s, eps).cpu().numpy()
    np.testing.assert_array_equal(rep, rep_o)


@pytest.mark.slow
def test_survey_threshold_and_clusters(torch_dev):
    """The survey stack at nu >= 10 (the Sec. 3.2 cut): hits on sampled start
    pixels against the oracle, and the groups against the injected sources."""
    from paper_1901_02492_amd import lib
    torch = torch_dev
    s = synth.survey_stack()
    n_img, h, w = s.img.shape
    planes, hits, n, rec = _gpu_threshold(torch, s, 10.0, cap=1 << 22)
    _say(f"case survey threshold: {n} hits")
    assert 0 < n <= (1 << 22)
    span = float(s.t[-1] - s.t[0])
    rep = lib.cluster_hits(hits, n, s.vel, span, 4.0).cpu().numpy()
    reps = np.unique(rep)
    _say(f"  {reps.size} groups")
    # Sampled start pixels: the hits there are the oracle's.
    rng = np.random.default_rng(10)
    src = s.sources[s.sources[:, 4] > 0]
    ys = np.concatenate([rng.integers(0, h, 6), np.clip(np.round(src[:10, 1]), 0, h - 1)]).astype(int)
    xs = np.concatenate([rng.integers(0, w, 6), np.clip(np.round(src[:10, 0]), 0, w - 1)]).astype(int)
    ref = oracle.search_pixels(s.img, s.var, s.mask, s.t, s.psf, s.vel, 1, ys, xs)
    tol = parity.tol_nu(10.0)
    for p in range(ys.size):
        at = rec[(rec["y"] == ys[p]) & (rec["x"] == xs[p])]
        got = set(at["vel"].tolist())
        clear = set(np.nonzero(ref["all_nu"][:, p] >= 10.0 + tol)[0].tolist())
        maybe = set(np.nonzero(ref["all_nu"][:, p] >= 10.0 - tol)[0].tolist())
        assert clear <= got <= maybe
        for r in at:
            nu_o = ref["all_nu"][r["vel"], p]
            assert abs(float(r["nu"]) - nu_o) <= 1e-5 * max(1.0, abs(nu_o))
    # Every representative is the best hit of its group.
    best = {}
    for i, r in enumerate(rep):
        best.setdefault(int(r), []).append(i)
    for r, members in best.items():
        assert rec["nu"][r] == rec["nu"][members].max()
