"""Pins of the light-curve filter oracle against facts that do not come from it.

* With q > 0 the filter's leave-one-out estimate is the posterior of a
  Gaussian process with the random-walk covariance, computed by dense linear
  algebra (a different method from the recursion).
* With q = 0 it is the inverse-variance mean of the other observations.
* Residuals of noise-only light curves are standard normal, so the share of
  squared residuals above c^2 is the two-sided normal tail, for q = 0 and for
  light curves drawn from the random walk itself.
* A planted outlier in a noise-free constant light curve is the only
  observation rejected (a single pass would also drop good observations whose
  estimate it pulled), and the refit matches the closed form.
"""
import math

import numpy as np
import pytest

from oracle import core
from oracle import lightcurve as lc

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tau(n, rng):
    """Survey-like times: 5 visits per night, gaps drawn at random."""
    return np.sort(np.concatenate([[0.0], rng.uniform(0.0, 2.5, n - 1)]))


def _gp_posterior(tau, y, var, obs, k, q):
    """Predictive mean and variance of f(tau_k) from the observations other
    than k, by universal kriging: f = mu + g with a flat prior on the level mu
    and g a random walk with variance q per day, g = 0 at the first
    observation; y_i = f(tau_i) + noise of variance var_i."""
    idx = [i for i in range(len(tau)) if obs[i] and i != k]
    t1 = min(tau[i] for i in range(len(tau)) if obs[i])
    g = lambda a, b: q * (min(a, b) - t1)
    C = np.array([[g(tau[a], tau[b]) for b in idx] for a in idx]) + np.diag([var[i] for i in idx])
    c = np.array([g(tau[k], tau[b]) for b in idx])
    one = np.ones(len(idx))
    yy = np.array([y[i] for i in idx])
    Ci1, Ciy, Cic = np.linalg.solve(C, one), np.linalg.solve(C, yy), np.linalg.solve(C, c)
    s = one @ Ci1
    mu = (one @ Ciy) / s
    m = mu + c @ np.linalg.solve(C, yy - mu * one)
    v = g(tau[k], tau[k]) - c @ Cic + (1.0 - one @ Cic) ** 2 / s
    return m, v


@pytest.mark.parametrize("q", [0.5, 20.0])
def test_loo_estimate_is_the_random_walk_posterior(q):
    rng = np.random.default_rng(11)
    n, c = 12, 6
    tau = _tau(n, rng)
    phi = rng.uniform(0.3, 3.0, (c, n))
    psi = phi * rng.normal(5.0, 2.0, (c, n))
    obs = rng.random((c, n)) < 0.8
    obs[:, 0] = True
    obs[:, 5] = True
    psi[~obs] = 0.0
    phi[~obs] = 0.0
    J, H = lc.kalman_loo(psi, phi, obs, tau, q)
    for a in range(c):
        y = psi[a] / np.where(obs[a], phi[a], 1.0)
        var = 1.0 / np.where(obs[a], phi[a], 1.0)
        for k in np.nonzero(obs[a])[0]:
            m, s2 = _gp_posterior(tau, y, var, obs[a], k, q)
            assert J[a, k] == pytest.approx(1.0 / s2, rel=1e-10)
            assert H[a, k] / J[a, k] == pytest.approx(m, rel=1e-10, abs=1e-10)


def test_without_process_noise_the_estimate_is_the_mean_of_the_others():
    rng = np.random.default_rng(12)
    c, n = 50, 15
    phi = rng.uniform(0.1, 4.0, (c, n))
    psi = rng.normal(0.0, 3.0, (c, n))
    obs = rng.random((c, n)) < 0.7
    psi[~obs] = 0.0
    phi[~obs] = 0.0
    J, H = lc.kalman_loo(psi, phi, obs, _tau(n, rng), 0.0)
    Jw = (phi.sum(axis=1, keepdims=True) - phi) * obs
    Hw = (psi.sum(axis=1, keepdims=True) - psi) * obs
    np.testing.assert_allclose(J, Jw, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(H, Hw, rtol=1e-12, atol=1e-12)


def _null_curves(rng, c, n, q, tau):
    """Noise-only light curves with the stated variances: the flux is constant
    (q = 0) or a random walk with variance q per day."""
    phi = rng.uniform(0.2, 5.0, (c, n))
    f = np.full((c, 1), 3.0) + np.cumsum(
        np.concatenate([np.zeros((c, 1)),
                        rng.normal(0.0, 1.0, (c, n - 1)) * np.sqrt(q * np.diff(tau))[None, :]],
                       axis=1), axis=1)
    y = f + rng.normal(0.0, 1.0, (c, n)) / np.sqrt(phi)
    return y * phi, phi


@pytest.mark.parametrize("q", [0.0, 4.0])
@pytest.mark.parametrize("cut", [1.0, 2.0])
def test_null_exceedance_rate_is_the_normal_tail(q, cut):
    rng = np.random.default_rng(13 + int(q))
    c, n = 20000, 10
    tau = _tau(n, rng)
    psi, phi = _null_curves(rng, c, n, q, tau)
    obs = np.ones((c, n), dtype=bool)
    J, H = lc.kalman_loo(psi, phi, obs, tau, q)
    rej = lc.residual_ratio(psi, phi, obs, J, H) > cut * cut
    p = math.erfc(cut / math.sqrt(2.0))
    m = c * n
    assert abs(rej.sum() - p * m) < 6.0 * math.sqrt(m * p * (1 - p))


@pytest.mark.parametrize("q", [0.0, 1.0])
def test_null_residuals_are_standard_normal(q):
    rng = np.random.default_rng(17)
    c, n = 20000, 15
    tau = _tau(n, rng)
    psi, phi = _null_curves(rng, c, n, q, tau)
    obs = np.ones((c, n), dtype=bool)
    J, H = lc.kalman_loo(psi, phi, obs, tau, q)
    z = (psi / phi - H / J) / np.sqrt(1.0 / phi + 1.0 / J)
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    np.testing.assert_allclose(lc.residual_ratio(psi, phi, obs, J, H), z * z, rtol=1e-9)


def test_planted_outlier_is_the_only_rejection():
    rng = np.random.default_rng(19)
    n, alpha = 15, 20.0
    tau = _tau(n, rng)
    phi = rng.uniform(0.5, 2.0, (1, n))
    psi = alpha * phi
    k = 6
    psi[0, k] = (alpha + 100.0 / math.sqrt(phi[0, k])) * phi[0, k]
    obs = np.ones((1, n), dtype=bool)
    for q in (0.0, 2.0):
        rej = lc.clip(psi, phi, obs, tau, q, 5.0)
        assert np.nonzero(rej[0])[0].tolist() == [k]
        nu, al, cnt = lc.refit(psi, phi, obs & ~rej)
        phi_kept = phi[0].sum() - phi[0, k]
        assert nu[0] == pytest.approx(alpha * math.sqrt(phi_kept), rel=1e-13)
        assert al[0] == pytest.approx(alpha, rel=1e-13)
        assert cnt[0] == n - 1


def test_clean_light_curve_keeps_every_observation():
    rng = np.random.default_rng(23)
    n, alpha = 15, 7.5
    phi = rng.uniform(0.5, 2.0, (3, n))
    psi = alpha * phi
    obs = np.ones((3, n), dtype=bool)
    assert not lc.clip(psi, phi, obs, _tau(n, rng), 0.0, 5.0).any()
    nu, al, cnt = lc.refit(psi, phi, obs)
    np.testing.assert_allclose(nu, alpha * np.sqrt(phi.sum(axis=1)), rtol=1e-13)
    assert (cnt == n).all()


def test_lone_observation_is_kept_and_a_pair_is_judged_together():
    psi = np.array([[4.0, 0.0, 0.0], [1.0, 0.0, 90.0], [1.0, 0.0, 1.5]])
    phi = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 1.0], [1.0, 0.0, 1.0]])
    obs = phi > 0
    rej = lc.clip(psi, phi, obs, np.array([0.0, 0.5, 1.0]), 0.3, 5.0)
    # The pair's residuals are equal: the first is dropped, the second is then alone.
    assert rej.tolist() == [[False, False, False], [True, False, False], [False, False, False]]


def test_filter_on_a_stack_gathers_the_trajectory_pixels():
    """lightcurve_filter reads the plane values the search sums (Sec. 2.2)."""
    rng = np.random.default_rng(29)
    n, h, w = 6, 20, 24
    t = np.array([0.0, 0.05, 0.1, 1.0, 1.05, 1.1])
    psi = rng.normal(0.0, 1.0, (n, h, w))
    phi = rng.uniform(0.5, 1.5, (n, h, w))
    ok = rng.random((n, h, w)) > 0.1
    psi[~ok] = 0.0
    phi[~ok] = 0.0
    vel = np.array([[3.0, -2.0], [-7.5, 4.0], [0.0, 0.0]])
    ys = np.array([3, 10, 19, 0])
    xs = np.array([5, 23, 0, 12])
    js = np.array([0, 1, 2, 5])                      # the last index is off the grid
    out = lc.lightcurve_filter(psi, phi, ok, t, vel, ys, xs, js, 5.0, 0.0)
    disp = core.displacements(t, vel)
    for c in range(3):
        for i in range(n):
            y, x = ys[c] + disp[js[c], i, 1], xs[c] + disp[js[c], i, 0]
            inside = 0 <= y < h and 0 <= x < w
            assert out["obs"][c, i] == (inside and ok[i, y, x])
            if out["obs"][c, i]:
                assert out["lc_psi"][c, i] == psi[i, y, x]
                assert out["lc_phi"][c, i] == phi[i, y, x]
    assert not out["obs"][3].any()
    assert out["nu"][3] == -np.inf and out["alpha"][3] == 0.0 and out["nobs"][3] == 0
    # With nothing rejected the refit is the search's own score.
    keep = out["obs"] & ~out["rejected"]
    P = (out["lc_psi"] * keep).sum(axis=1)
    F = (out["lc_phi"] * keep).sum(axis=1)
    nu, al = core.scores(P, F)
    np.testing.assert_allclose(out["nu"][:3], nu[:3], rtol=1e-12)


def test_sampled_light_curves_equal_the_full_gather():
    rng = np.random.default_rng(31)
    n, h, w = 5, 16, 18
    t = np.array([0.0, 0.1, 0.2, 1.0, 1.1])
    psi = rng.normal(0.0, 1.0, (n, h, w))
    phi = rng.uniform(0.5, 1.5, (n, h, w))
    ok = rng.random((n, h, w)) > 0.2
    vel = rng.uniform(-20.0, 20.0, (7, 2))
    ys, xs = rng.integers(0, h, 40), rng.integers(0, w, 40)
    js = rng.integers(-1, 8, 40)
    full = lc.light_curves(psi, phi, ok, t, vel, ys, xs, js)
    at = lc.light_curves_at(lambda i, yy, xx: (psi[i, yy, xx], phi[i, yy, xx], ok[i, yy, xx]),
                            n, h, w, t, vel, ys, xs, js)
    for a, b in zip(full, at):
        np.testing.assert_array_equal(a, b)
