"""The C oracle (oracle/kb_oracle.c), CPU only: bit-for-bit equal to the numpy
oracle (itself pinned by tests/test_oracle_pins.py) on random stacks with
masks, non-finite and zero-variance pixels, exact ties and trajectories that
leave the frame; pinned directly by the closed form, the static coadd and
literal-loop brute force; planted mistakes fail; and the row-band runner and
the band checker used by the full-frame parity test."""
import math

import numpy as np
import pytest

import oracle
from oracle import bands, cref
from paper_1901_02492_amd import synth
from tests import brute_ref, parity


def _same(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.shape == b.shape and a.tobytes() == b.tobytes()


CASES = [  # seed, n, h, w, n_vel, k
    (401, 5, 30, 50, 20, 6), (402, 7, 12, 40, 30, 30), (403, 3, 1, 64, 9, 4),
    (404, 17, 20, 70, 12, 5), (405, 1, 9, 9, 7, 3), (406, 2, 16, 33, 40, 10),
]


def _stack(seed, n, h, w, nv, k):
    s = synth.random_stack(seed, n=n, h=h, w=w, n_vel=nv, k=k, psf_size=5, vmax=12.0, tmax=2.0)
    s.img[0, h // 2, w // 3] = np.nan
    s.var[-1, h - 1, w - 1] = 0.0
    s.vel[min(3, nv - 1)] = s.vel[min(1, nv - 1)]      # a duplicate velocity: exact ties
    return s


@pytest.mark.parametrize("case", CASES, ids=[str(c[0]) for c in CASES])
def test_c_oracle_equals_numpy_oracle_bitwise(case):
    s = _stack(*case)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k)
    psi, phi, ok = cref.planes(s.img, s.var, s.mask, s.psf)
    assert _same(psi, ref["psi"]) and _same(phi, ref["phi"])
    assert np.array_equal(ok, oracle.validity(s.img, s.var, s.mask))
    got = cref.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k)
    for key in ("nu", "alpha"):
        assert _same(got[key], ref[key]), key
    assert np.array_equal(got["vel"], ref["vel"])
    assert np.array_equal(got["nobs"], ref["nobs"])


def test_c_oracle_closed_form():
    """Noise-free source flux * T centred on integer pixels along a grid
    velocity, unit variance, kernel inside the frame: Psi = N flux S2,
    Phi = N S2 with S2 = sum T^2, so alpha = flux and nu = flux sqrt(N S2)
    (= 30.31733 for N = 5, flux 50 and the pixel-integrated 7x7 PSF with
    sigma = 1).  The stamp is stored in float32, hence the 1e-6 tolerance."""
    psf = synth.psf_gaussian(1.0, 7)
    T = psf.astype(np.float64)
    S2 = float((T * T).sum())
    t = np.array([0.0, 0.05, 0.1, 0.15, 0.2])
    n, h, w, c = 5, 64, 64, 3
    img = np.zeros((n, h, w), np.float32)
    for i in range(n):
        xi = 20 + int(math.floor(40.0 * t[i] + 0.5))
        yi = 30 + int(math.floor(20.0 * t[i] + 0.5))
        img[i, yi - c:yi + c + 1, xi - c:xi + c + 1] = (50.0 * T).astype(np.float32)
    vel = np.array([[0.0, 0.0], [40.0, 20.0], [10.0, -10.0]])
    got = cref.search(img, np.ones_like(img), None, t, psf, vel, 3)
    assert got["vel"][30, 20, 0] == 1
    assert got["nobs"][30, 20, 0] == 5
    assert got["Phi"][30, 20, 0] == pytest.approx(n * S2, rel=1e-12)
    assert got["alpha"][30, 20, 0] == pytest.approx(50.0, rel=1e-6)
    assert got["nu"][30, 20, 0] == pytest.approx(50.0 * math.sqrt(n * S2), rel=1e-6)
    assert got["nu"][30, 20, 0] == pytest.approx(30.31733045, rel=1e-6)


def test_c_oracle_static_coadd_and_brute_force():
    s = synth.random_stack(411, n=3, h=7, w=9, n_vel=5, k=5, psf_size=3, vmax=3.0, tmax=1.0)
    vel = np.vstack([[0.0, 0.0], s.vel])
    psi, phi, ok = cref.planes(s.img, s.var, s.mask, s.psf)
    r = cref.search_rows(psi, phi, ok, 7, s.t, vel, 6, 0, 7)
    j0 = np.argmax(r["vel"] == 0, axis=-1)
    Psi = np.zeros((7, 9))
    Phi = np.zeros((7, 9))
    for i in range(3):
        Psi += psi[i]
        Phi += phi[i]
    pick = lambda a: np.take_along_axis(a, j0[..., None], -1)[..., 0]
    fin = Phi > 0
    assert np.allclose(pick(r["nu"])[fin], (Psi / np.sqrt(np.where(fin, Phi, 1)))[fin],
                       rtol=1e-13)
    bpsi, bphi, bok = brute_ref.planes(s.img.tolist(), s.var.tolist(), s.mask.tolist(),
                                       s.psf.tolist())
    assert np.allclose(psi, np.array(bpsi), rtol=1e-12, atol=1e-14)
    assert np.allclose(phi, np.array(bphi), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mutation", ["ORC_MUTATION_CONVOLVE", "ORC_MUTATION_RINT",
                                      "ORC_MUTATION_NO_SQRT"])
def test_c_oracle_planted_mistakes_fail(tmp_path, mutation):
    lib = cref.load(cref.build(str(tmp_path / "libmut.so"), defines=[mutation]))
    s = synth.small_stack()
    s3 = synth.random_stack(412, n=4, h=14, w=20, n_vel=12, k=4, psf_size=5, vmax=10.0,
                            tmax=1.0)
    s3.psf[0, 1] *= 3.0        # asymmetric PSF: correlation and convolution differ
    differs = False
    for st in (s, s3):
        ref = oracle.search(st.img, st.var, st.mask, st.t, st.psf, st.vel, st.k)
        got = cref.search(st.img, st.var, st.mask, st.t, st.psf, st.vel, st.k, lib=lib)
        differs |= not (_same(got["nu"], ref["nu"]) and np.array_equal(got["vel"], ref["vel"]))
    assert differs


def test_run_bands_and_band_checker():
    s = synth.random_stack(413, n=6, h=40, w=70, n_vel=24, k=6, psf_size=5, vmax=8.0, tmax=1.0)
    full = cref.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k + 4)
    got, timing = bands.run_bands(s.img, s.var, s.mask, s.psf, s.t, s.vel, s.k + 4, 5, 33,
                                  band_rows=7, workers=2)
    for key in ("nu", "alpha", "Phi", "nobs", "vel"):
        assert _same(got[key], full[key][5:33]), key
    assert timing["planes_s"] >= 0 and len(timing["band_s"]) == math.ceil(28 / 7)
    # the oracle's own top k, in float32, passes the band checker
    k = s.k
    gpu = [full["nu"][..., :k].astype(np.float32), full["alpha"][..., :k].astype(np.float32),
           full["vel"][..., :k].astype(np.int32), full["nobs"][..., :k].astype(np.int16)]
    stats = parity.check_band(gpu, full, k)
    assert stats["recalled"] == stats["entries"]
    bad = [g.copy() for g in gpu]
    bad[3][3, 4, 1] += 1
    with pytest.raises(AssertionError):
        parity.check_band(bad, full, k)
    bad = [g.copy() for g in gpu]
    bad[2][7, 8, 0] = full["vel"][7, 8, k + 3]        # a trajectory far down the list
    with pytest.raises(AssertionError):
        parity.check_band(bad, full, k)
