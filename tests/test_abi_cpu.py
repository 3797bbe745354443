"""Host-side checks of the C ABI that need no GPU: the library loads and exports
every symbol the header declares, the displacement table equals the oracle's
bit for bit, and invalid arguments are rejected before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1901_02492_amd import lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "kbmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(kb_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert {"kb_make_psi_phi", "kb_search", "kb_topk", "kb_displacements"} <= set(names)
    L = lib.load()
    for n in names:
        assert hasattr(L, n), n


def test_abi_version():
    assert lib.load().kb_abi_version() == 1


@pytest.mark.parametrize("which", ["small", "survey", "random"])
def test_displacements_equal_oracle_bit_for_bit(which):
    if which == "small":
        s = synth.small_stack()
        t, vel = s.t, s.vel
    elif which == "survey":
        t = np.array([n + 0.06 * e for n in range(3) for e in range(5)])
        vel = synth.velocity_grid_polar(np.linspace(80, 400, 25), np.linspace(-0.5, 0.5, 24))
    else:
        rng = np.random.default_rng(4)
        t = np.sort(rng.uniform(0, 3, 40))
        vel = rng.uniform(-500, 500, (3000, 2))
        vel[:100] = np.round(vel[:100]) + 0.5
    got = lib.displacements(t, vel)
    ref = oracle.displacements(t, vel)
    assert got.dtype == np.int32
    assert np.array_equal(got.astype(np.int64), ref)


def test_displacement_half_ties_in_library():
    t = np.array([0.0, 0.05, 0.15])
    vel = np.array([[-50.0, -30.0], [-10.0, 30.0]])
    d = lib.displacements(t, vel)
    assert d[0, 1].tolist() == [-2, -1] and d[0, 2].tolist() == [-7, -4]
    assert d[1, 1].tolist() == [0, 2] and d[1, 2].tolist() == [-1, 5]


@pytest.mark.parametrize("t,vel,msg", [
    ([0.0, 1.0, 0.5], [[1.0, 1.0]], "non-decreasing"),
    ([0.0, np.nan], [[1.0, 1.0]], "not finite"),
    ([0.0, 1.0], [[np.inf, 1.0]], "not finite"),
    ([0.0, 2.0], [[6e8, 0.0]], "2^30"),
])
def test_displacements_reject_bad_inputs(t, vel, msg):
    with pytest.raises(lib.KbError) as e:
        lib.displacements(t, vel)
    assert e.value.status == lib.KB_EINVAL and msg in str(e.value)


def _search_call(**over):
    """Call kb_search with fake device pointers; only argument checks may run."""
    fake = 1 << 20
    a = dict(planes=fake, dtype=0, scale=None, n=3, h=8, w=8, t=np.array([0.0, 1.0, 2.0]),
             vel=np.zeros((4, 2)), nv=4, kc=2, ws=fake, wsb=1 << 20)
    a.update(over)
    t = np.ascontiguousarray(a["t"], dtype=np.float64)
    vel = np.ascontiguousarray(a["vel"], dtype=np.float64)
    L = lib.load()
    st = L.kb_search(a["planes"], a["dtype"], a["scale"], a["n"], a["h"], a["w"], t.ctypes.data,
                     vel.ctypes.data, a["nv"], a["kc"], fake, fake, fake, fake, a["ws"], a["wsb"],
                     None)
    return st, L.kb_last_error().decode()


@pytest.mark.parametrize("over,status", [
    (dict(planes=None), lib.KB_EINVAL),
    (dict(n=0), lib.KB_EINVAL),
    (dict(h=0), lib.KB_EINVAL),
    (dict(kc=0), lib.KB_EINVAL),
    (dict(kc=5), lib.KB_EINVAL),                       # k_cand > n_vel
    (dict(kc=65, nv=100, vel=np.zeros((100, 2))), lib.KB_EUNSUPPORTED),
    (dict(t=np.array([0.0, 2.0, 1.0])), lib.KB_EINVAL),
    (dict(dtype=7), lib.KB_EINVAL),
    (dict(dtype=1), lib.KB_EINVAL),                     # 16-bit planes without scales
    (dict(ws=None), lib.KB_EINVAL),
    (dict(ws=(1 << 20) + 4), lib.KB_EINVAL),            # misaligned workspace
    (dict(wsb=16), lib.KB_ENOMEM),
    (dict(w=(1 << 27) + 1), lib.KB_EINVAL),
])
def test_search_rejects_bad_arguments_before_enqueue(over, status):
    st, msg = _search_call(**over)
    assert st == status and msg


def test_make_psi_phi_lp_needs_buffers():
    L = lib.load()
    psf = np.ones((3, 3), np.float32)
    fake = 1 << 20
    st = L.kb_make_psi_phi(fake, fake, None, 2, 8, 8, psf.ctypes.data, 3, 3, fake, lib.KB_F16,
                           None, None, None)
    assert st == lib.KB_EINVAL and "lp" in L.kb_last_error().decode()
    st = L.kb_make_psi_phi(fake, fake, None, 2, 8, 8, psf.ctypes.data, 3, 3, fake, 9, fake, fake,
                           None)
    assert st == lib.KB_EINVAL


def test_topk_rescore_checks_times():
    L = lib.load()
    fake = 1 << 20
    t = np.array([0.0, 2.0, 1.0])
    v = np.zeros((4, 2))
    out = 5 << 20
    st = L.kb_topk(fake, 3, 8, 8, t.ctypes.data, v.ctypes.data, 4, fake, fake, fake, fake, 4, 4,
                   out, out + 256, out + 512, out + 768, fake, 1 << 20, None)
    assert st == lib.KB_EINVAL and "non-decreasing" in L.kb_last_error().decode()


def test_topk_in_place_argument_checks():
    """kb_topk's outputs are either all four candidate arrays (k == k_cand, no
    re-scoring) or separate from them; anything else fails before enqueue."""
    L = lib.load()
    a, b, c, d = (1 << 20), (2 << 20), (3 << 20), (4 << 20)
    o = 5 << 20
    t = np.array([0.0, 1.0, 2.0])
    v = np.zeros((4, 2))
    # one output is a candidate array, the others are not
    st = L.kb_topk(None, 3, 8, 8, None, None, 0, a, b, c, d, 4, 4, a, o, o + 1, o + 2,
                   None, 0, None)
    assert st == lib.KB_EINVAL and "candidate arrays" in L.kb_last_error().decode()
    st = L.kb_topk(None, 3, 8, 8, None, None, 0, a, b, c, d, 4, 4, o, o + 1, o + 2, a,
                   None, 0, None)
    assert st == lib.KB_EINVAL
    # in place with k < k_cand, or with re-scoring
    st = L.kb_topk(None, 3, 8, 8, None, None, 0, a, b, c, d, 4, 3, a, b, c, d, None, 0, None)
    assert st == lib.KB_EINVAL and "in place" in L.kb_last_error().decode()
    st = L.kb_topk(o, 3, 8, 8, t.ctypes.data, v.ctypes.data, 4, a, b, c, d, 4, 4, a, b, c, d,
                   o, 1 << 20, None)
    assert st == lib.KB_EINVAL and "in place" in L.kb_last_error().decode()


def test_make_psi_phi_rejects_bad_psf():
    L = lib.load()
    psf = np.ones((4, 5), np.float32)
    fake = 1 << 20
    st = L.kb_make_psi_phi(fake, fake, None, 2, 8, 8, psf.ctypes.data, 4, 5, fake, 0, None,
                           None, None)
    assert st == lib.KB_EINVAL and "odd" in L.kb_last_error().decode()
    big = np.ones((27, 27), np.float32)
    st = L.kb_make_psi_phi(fake, fake, None, 2, 8, 8, big.ctypes.data, 27, 27, fake, 0, None,
                           None, None)
    assert st == lib.KB_EUNSUPPORTED


def test_topk_rejects_k_above_k_cand():
    L = lib.load()
    fake = 1 << 20
    st = L.kb_topk(None, 3, 8, 8, None, None, 0, fake, fake, fake, fake, 4, 5, fake, fake, fake,
                   fake, None, 0, None)
    assert st == lib.KB_EINVAL


def test_workspace_size():
    nb = lib.search_workspace_bytes(15, 4096, 4096, 600)
    assert nb >= 15 * 600 * 8
    assert nb % 256 == 0
    assert lib.search_workspace_bytes(0, 8, 8, 600) == 0
    assert lib.search_workspace_bytes(3, 0, 8, 600) == 0


def test_batch_rejects_bad_jobs_before_enqueue():
    L = lib.load()
    fake = 1 << 20
    t = np.array([0.0, 1.0, 2.0])
    v = np.zeros((4, 2))
    good = lib.KbJob(fake, None, 3, 8, 8, t.ctypes.data, v.ctypes.data, 4, fake, fake, fake, fake)
    bad_t = np.array([0.0, 2.0, 1.0])
    bad = lib.KbJob(fake, None, 3, 8, 8, bad_t.ctypes.data, v.ctypes.data, 4, fake, fake, fake,
                    fake)
    arr = (lib.KbJob * 2)(good, bad)
    st = L.kb_search_batch(ctypes.addressof(arr), 2, 0, 2, fake, 1 << 20, None)
    assert st == lib.KB_EINVAL and "job 1" in L.kb_last_error().decode()
    arr = (lib.KbJob * 1)(good)
    assert L.kb_search_batch(ctypes.addressof(arr), 1, 0, 5, fake, 1 << 20, None) == lib.KB_EINVAL
    assert L.kb_search_batch(ctypes.addressof(arr), 0, 0, 2, fake, 1 << 20, None) == lib.KB_EINVAL
    assert L.kb_search_batch(ctypes.addressof(arr), 1, 1, 2, fake, 1 << 20, None) == lib.KB_EINVAL
    assert L.kb_search_batch(ctypes.addressof(arr), 1, 0, 2, fake, 16, None) == lib.KB_ENOMEM
    assert L.kb_search_batch_workspace_bytes(ctypes.addressof(arr), 1) > 0


def _lc_call(n=3, h=8, w=8, t=None, nv=4, k=2, cut=5.0, q=0.0, ws_bytes=1 << 20, ws=1 << 20,
             cand=1 << 20):
    L = lib.load()
    fake = 1 << 20
    t = np.arange(n, dtype=np.float64) if t is None else t
    v = np.zeros((nv, 2))
    st = L.kb_lightcurve_filter(fake, n, h, w, t.ctypes.data, v.ctypes.data, nv, cand, k, cut, q,
                                fake, fake, fake, None, ws, ws_bytes, None)
    return st, L.kb_last_error().decode()


def test_lightcurve_filter_argument_checks():
    st, msg = _lc_call(n=65, t=np.arange(65, dtype=np.float64))
    assert st == lib.KB_EUNSUPPORTED and "64" in msg
    assert _lc_call(cut=0.0)[0] == lib.KB_EINVAL
    assert _lc_call(cut=float("nan"))[0] == lib.KB_EINVAL
    assert _lc_call(cut=1e200)[0] == lib.KB_EINVAL            # cut^2 overflows
    assert _lc_call(q=-1.0)[0] == lib.KB_EINVAL
    assert _lc_call(q=float("inf"))[0] == lib.KB_EINVAL
    assert _lc_call(k=0)[0] == lib.KB_EINVAL
    assert _lc_call(nv=0)[0] == lib.KB_EINVAL
    assert _lc_call(cand=None)[0] == lib.KB_EINVAL
    assert _lc_call(ws=None)[0] == lib.KB_EINVAL
    assert _lc_call(ws=(1 << 20) + 8)[0] == lib.KB_EINVAL   # misaligned
    st, msg = _lc_call(ws_bytes=16)
    assert st == lib.KB_ENOMEM and "workspace" in msg
    st, msg = _lc_call(t=np.array([0.0, 2.0, 1.0]))
    assert st == lib.KB_EINVAL and "non-decreasing" in msg


def test_threshold_and_cluster_argument_checks():
    L = lib.load()
    fake = 1 << 20
    t = np.arange(3, dtype=np.float64)
    v = np.zeros((4, 2))
    call = lambda **kw: L.kb_search_threshold(
        fake, 3, kw.get("h", 8), kw.get("w", 8), t.ctypes.data, v.ctypes.data, kw.get("nv", 4),
        kw.get("m", 10.0), kw.get("hits", fake), kw.get("cap", 16), kw.get("cnt", fake),
        kw.get("ws", fake), kw.get("wsb", 1 << 20), None)
    assert call(m=float("nan")) == lib.KB_EINVAL
    assert call(m=float("inf")) == lib.KB_EINVAL
    assert call(cnt=None) == lib.KB_EINVAL
    assert call(cap=-1) == lib.KB_EINVAL
    assert call(hits=None) == lib.KB_EINVAL
    assert call(w=1 << 24) == lib.KB_EUNSUPPORTED
    assert call(wsb=64) == lib.KB_ENOMEM
    assert call(nv=0) == lib.KB_EINVAL
    vv = np.zeros((4, 2))
    cl = lambda **kw: L.kb_cluster_hits(kw.get("hits", fake), kw.get("n", 10), vv.ctypes.data,
                                        4, kw.get("s", 1.0), kw.get("eps", 2.0),
                                        kw.get("rep", fake), kw.get("ws", fake),
                                        kw.get("wsb", 1 << 20), None)
    assert cl(n=0, hits=None) == lib.KB_OK          # nothing to do
    assert cl(n=-1) == lib.KB_EINVAL
    assert cl(eps=-1.0) == lib.KB_EINVAL
    assert cl(s=float("nan")) == lib.KB_EINVAL
    assert cl(rep=None) == lib.KB_EINVAL
    assert cl(wsb=16) == lib.KB_ENOMEM
    assert cl(n=(1 << 30) + 1) == lib.KB_EUNSUPPORTED
    assert L.kb_cluster_workspace_bytes(1000, 4) >= 1000 * 20
    assert lib.HIT_DTYPE.itemsize == 24


def test_stamps_argument_checks():
    L = lib.load()
    fake = 1 << 20
    t = np.arange(3, dtype=np.float64)
    v = np.zeros((4, 2))
    call = lambda **kw: L.kb_stamps(
        fake, fake, None, kw.get("n", 3), 8, 8, t.ctypes.data if kw.get("n", 3) == 3 else
        np.arange(kw["n"], dtype=np.float64).ctypes.data, v.ctypes.data, 4, fake, None,
        kw.get("nc", 5), kw.get("R", 2), kw.get("off", 1.0), 1.0, 0.5, 4.0, None, None,
        kw.get("ok", fake), fake, kw.get("wsb", 1 << 20), None)
    assert call(R=-1) == lib.KB_EINVAL
    assert call(R=16) == lib.KB_EINVAL
    assert call(off=float("nan")) == lib.KB_EINVAL
    assert call(ok=None) == lib.KB_EINVAL
    assert call(nc=-1) == lib.KB_EINVAL
    assert call(wsb=32) == lib.KB_ENOMEM
    tt = np.arange(65, dtype=np.float64)
    st = L.kb_stamps(fake, fake, None, 65, 8, 8, tt.ctypes.data, v.ctypes.data, 4, fake, None, 5,
                     2, 1.0, 1.0, 0.5, 4.0, None, None, fake, fake, 1 << 20, None)
    assert st == lib.KB_EUNSUPPORTED


@pytest.mark.parametrize("n_img,n_vel", [(16, 29955), (32, 15649)])
def test_noalloc_limit_is_the_documented_one(n_img, n_vel):
    """kb_search_noalloc refuses, before touching a device, the first stack
    past the limits its header states (16 images with 29954 velocities, 32
    with 15648 fit the fixed array)."""
    L = lib.load()
    fake = 1 << 20
    t = np.arange(n_img, dtype=np.float64)
    vel = np.zeros((n_vel, 2))
    st = L.kb_search_noalloc(fake, lib.KB_F32, None, n_img, 8, 70, t.ctypes.data,
                             vel.ctypes.data, n_vel, 4, fake, fake, fake, fake, None)
    assert st == lib.KB_EUNSUPPORTED
    a = lambda x: (x + 255) // 256 * 256   # noqa: E731
    def need(nv):
        base = a(lib.search_workspace_bytes(n_img, 8, 70, nv))
        return a(a(a(base + 8 * n_img) + 16 * nv) + 4 * nv)
    assert need(n_vel) > (8 << 20) >= need(n_vel - 1)   # KB_NOALLOC_SCRATCH_BYTES
