"""Pins of the stamp/moment oracle against facts that do not come from it.

* A noise-free point source on the trajectory gives a symmetric stamp whose
  centroid is 0, m11 is 0 and m20 = m02 equal the variance of the
  pixel-integrated Gaussian over the stamp, computed in one dimension.
* A source 2 px beside the trajectory moves the centroid by 2 px.
* The coadd is the mean over valid pixels: a masked pixel is left out of its
  own image's term, a constant stack gives a constant stamp.
* An elongated source has m20 >> m02 and fails the filter.
* Excluding the image that carries a flash restores the point source.
"""
import math

import numpy as np
import pytest

from oracle import stamps as os_
from paper_1901_02492_amd import synth


def _stack(n=5, h=48, w=48, sigma=1.0):
    t = np.array([0.0, 0.05, 0.1, 0.15, 0.2])[:n]
    img = np.zeros((n, h, w), dtype=np.float32)
    var = np.ones((n, h, w), dtype=np.float32)
    mask = np.zeros((n, h, w), dtype=np.uint8)
    return t, img, var, mask


def _profile_1d(sigma, R):
    from scipy.special import ndtr
    u = np.arange(-R, R + 1, dtype=np.float64)
    return ndtr((u + 0.5) / sigma) - ndtr((u - 0.5) / sigma), u


@pytest.mark.parametrize("sigma,R", [(1.0, 6), (1.5, 5)])
def test_point_source_moments_are_the_psf_variance(sigma, R):
    t, img, var, mask = _stack(sigma=sigma)
    vel = np.array([[40.0, 20.0]])          # integer pixel steps at these times
    x0, y0 = 20, 22
    for i in range(t.size):
        synth.render_point_source(img[i], x0 + 40.0 * t[i], y0 + 20.0 * t[i], 30.0, sigma)
    S = os_.coadd_stamps(img, var, mask, t, vel, [x0], [y0], [0], R)
    M00, ub, vb, m20, m02, m11 = os_.moments(S)
    g, u = _profile_1d(sigma, R)
    var1 = float((u * u * g).sum() / g.sum())
    assert abs(ub[0]) < 1e-9 and abs(vb[0]) < 1e-9 and abs(m11[0]) < 1e-9
    assert m20[0] == pytest.approx(var1, rel=1e-5) and m02[0] == pytest.approx(var1, rel=1e-5)
    assert M00[0] == pytest.approx(30.0 * g.sum() ** 2, rel=1e-5)
    assert os_.stamp_filter((M00, ub, vb, m20, m02, m11), 0.5, 0.1, 0.5 * var1, 2 * var1)[0]


def test_source_beside_the_trajectory_moves_the_centroid():
    t, img, var, mask = _stack()
    vel = np.array([[40.0, 20.0]])
    for i in range(t.size):
        synth.render_point_source(img[i], 22 + 40.0 * t[i], 22 + 20.0 * t[i], 30.0, 1.0)
    S = os_.coadd_stamps(img, var, mask, t, vel, [20], [22], [0], 8)
    mom = os_.moments(S)
    assert mom[1][0] == pytest.approx(2.0, abs=1e-4) and abs(mom[2][0]) < 1e-9
    # Central moments are taken about the centroid: the spread is the PSF's
    # (pixel-integrated sigma = 1: variance 1 + 1/12), not 4 px^2 more.
    assert mom[3][0] == pytest.approx(1.0 + 1.0 / 12.0, abs=1e-3)
    assert mom[4][0] == pytest.approx(1.0 + 1.0 / 12.0, abs=1e-3)
    assert not os_.stamp_filter(mom, 1.0, 0.5, 0.5, 2.0)[0]


def test_mean_over_valid_pixels():
    t, img, var, mask = _stack(n=3, h=12, w=12)
    img[:] = np.array([1.0, 2.0, 6.0], dtype=np.float32)[:, None, None]
    mask[2, 5, 5] = 1                      # only image 2's pixel (5, 5) is invalid
    var[1, 5, 6] = 0.0                     # image 1's pixel (6, 5) too (variance)
    S = os_.coadd_stamps(img, var, mask, t, np.zeros((1, 2)), [5], [5], [0], 1)[0]
    assert S[1, 1] == pytest.approx(1.5)   # (1 + 2) / 2
    assert S[1, 2] == pytest.approx(3.5)   # (1 + 6) / 2
    assert S[0, 0] == pytest.approx(3.0)
    # Off the frame nothing contributes.
    S2 = os_.coadd_stamps(img, var, mask, t, np.zeros((1, 2)), [0], [0], [0], 2)[0]
    assert (S2[:2, :] == 0).all() and (S2[:, :2] == 0).all() and S2[2, 2] == pytest.approx(3.0)


def test_elongated_source_fails():
    t, img, var, mask = _stack()
    for i in range(t.size):
        for dx in np.linspace(-4, 4, 9):
            synth.render_point_source(img[i], 24 + dx, 24, 5.0, 1.0)
    S = os_.coadd_stamps(img, var, mask, t, np.zeros((1, 2)), [24], [24], [0], 8)
    mom = os_.moments(S)
    assert mom[3][0] > 4 * mom[4][0]
    assert not os_.stamp_filter(mom, 1.0, 0.5, 0.5, 3.0)[0]


def test_excluding_the_flash_image_restores_the_point_source():
    t, img, var, mask = _stack()
    vel = np.array([[40.0, 20.0]])
    for i in range(t.size):
        synth.render_point_source(img[i], 20 + 40.0 * t[i], 22 + 20.0 * t[i], 30.0, 1.0)
    synth.render_point_source(img[3], 20 + 40.0 * t[3] + 4, 22 + 20.0 * t[3] - 3, 400.0, 1.0)
    keep = np.ones((1, t.size), dtype=bool)
    bad = os_.moments(os_.coadd_stamps(img, var, mask, t, vel, [20], [22], [0], 6))
    keep[0, 3] = False
    good = os_.moments(os_.coadd_stamps(img, var, mask, t, vel, [20], [22], [0], 6, keep))
    assert abs(bad[1][0]) > 1.0
    assert abs(good[1][0]) < 1e-9 and abs(good[2][0]) < 1e-9
