"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case swaps one oracle step for a plausible wrong version and re-runs a
pin from test_oracle_pins.py, which must then fail.
"""
import numpy as np
import pytest

import oracle
import oracle.core as core
from tests import test_oracle_pins as pins


def _patch(monkeypatch, name, fn):
    """Replace an oracle step both where the pins call it and where the oracle does."""
    monkeypatch.setattr(core, name, fn)
    monkeypatch.setattr(oracle, name, fn, raising=False)


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_convolution_instead_of_correlation_is_caught(monkeypatch):
    orig = core._correlate_zero
    _patch(monkeypatch, "_correlate_zero", lambda p, k: orig(p, k[::-1, ::-1]))
    assert _fails(pins.test_planes_equal_scipy_correlate_asymmetric_psf)


def test_round_half_even_is_caught(monkeypatch):
    def disp_rint(t, vel):
        t = np.asarray(t, np.float64)
        vel = np.asarray(vel, np.float64).reshape(-1, 2)
        return np.rint(vel[:, None, :] * (t - t[0])[None, :, None]).astype(np.int64)
    _patch(monkeypatch, "displacements", disp_rint)
    assert _fails(pins.test_displacement_half_ties, -30, 0.05, -1)
    assert _fails(pins.test_displacements_equal_exact_rationals_on_small_grid)


def test_swapped_axes_are_caught(monkeypatch):
    orig = core.displacements
    _patch(monkeypatch, "displacements", lambda t, v: orig(t, v)[:, :, ::-1])
    assert _fails(pins.test_search_equals_brute_force, 0, 3, 7, 9, 6, 3)


def test_invalid_centre_not_zeroed_is_caught(monkeypatch):
    orig = core.psi_phi

    def leaky(img, var, mask, psf):
        psi, phi, ok = orig(img, var, None, psf)     # mask ignored
        return psi, phi, ok
    _patch(monkeypatch, "psi_phi", leaky)
    assert _fails(pins.test_masking_an_image_equals_dropping_it)


def test_dropped_sqrt_is_caught(monkeypatch):
    def bad_scores(Psi, Phi):
        pos = Phi > 0
        safe = np.where(pos, Phi, 1.0)
        return np.where(pos, Psi / safe, -np.inf), np.where(pos, Psi / safe, 0.0)
    _patch(monkeypatch, "scores", bad_scores)
    assert _fails(pins.test_closed_form_point_source, 1.0, 7, 5, 50.0, 1.0)
    assert _fails(pins.test_noise_only_nu_is_standard_normal)


def test_unweighted_phi_is_caught(monkeypatch):
    # phi built with T instead of T^2.
    orig = core._correlate_zero
    calls = {"n": 0}

    def corr(p, k):
        calls["n"] += 1
        return orig(p, np.sqrt(k) if calls["n"] % 2 == 0 else k)
    _patch(monkeypatch, "_correlate_zero", corr)
    assert _fails(pins.test_closed_form_point_source, 1.5, 11, 15, 12.5, 0.8)


def test_tie_break_by_descending_index_is_caught(monkeypatch):
    _patch(monkeypatch, "rank_topk", lambda nu, k: (nu.shape[0] - 1 - np.argsort(-nu[::-1], axis=0, kind="stable"))[:k])
    assert _fails(pins.test_rank_topk_equals_sorted_with_ties)


# Light-curve filter: each planted mistake must fail a pin of
# test_oracle_lightcurve.py.

from oracle import lightcurve as lcf  # noqa: E402
from tests import test_oracle_lightcurve as lcpins  # noqa: E402


def test_estimate_that_uses_the_observation_itself_is_caught(monkeypatch):
    orig = lcf.kalman_loo

    def with_self(lc_psi, lc_phi, obs, tau, q):
        J, H = orig(lc_psi, lc_phi, obs, tau, q)
        return J + lc_phi * obs, H + lc_psi * obs
    monkeypatch.setattr(lcf, "kalman_loo", with_self)
    assert _fails(lcpins.test_loo_estimate_is_the_random_walk_posterior, 0.5)
    assert _fails(lcpins.test_null_residuals_are_standard_normal, 0.0)


def test_ignored_process_noise_is_caught(monkeypatch):
    orig = lcf._one_direction
    monkeypatch.setattr(lcf, "_one_direction",
                        lambda lp, lf, o, tau, q, order: orig(lp, lf, o, tau, 0.0, order))
    assert _fails(lcpins.test_loo_estimate_is_the_random_walk_posterior, 20.0)
    assert _fails(lcpins.test_null_residuals_are_standard_normal, 1.0)


def test_forward_only_filter_is_caught(monkeypatch):
    def forward(lc_psi, lc_phi, obs, tau, q):
        return lcf._one_direction(lc_psi, lc_phi, obs, np.asarray(tau, np.float64), q,
                                  range(lc_psi.shape[1]))
    monkeypatch.setattr(lcf, "kalman_loo", forward)
    assert _fails(lcpins.test_loo_estimate_is_the_random_walk_posterior, 0.5)


def test_residual_variance_without_the_estimate_term_is_caught(monkeypatch):
    def narrow(lc_psi, lc_phi, obs, J, H):
        a = lc_psi * J - lc_phi * H
        d = (lc_phi * J) * J
        pos = obs & (d > 0)
        return np.where(pos, (a * a) / np.where(pos, d, 1.0), 0.0)
    monkeypatch.setattr(lcf, "residual_ratio", narrow)
    assert _fails(lcpins.test_null_exceedance_rate_is_the_normal_tail, 2.0, 0.0)
    assert _fails(lcpins.test_null_residuals_are_standard_normal, 0.0)


def test_single_pass_clip_is_caught(monkeypatch):
    def one_pass(lc_psi, lc_phi, obs, tau, q, sigma_cut):
        J, H = lcf.kalman_loo(lc_psi, lc_phi, obs, tau, q)
        return obs & (lcf.residual_ratio(lc_psi, lc_phi, obs, J, H) > sigma_cut ** 2)
    monkeypatch.setattr(lcf, "clip", one_pass)
    assert _fails(lcpins.test_planted_outlier_is_the_only_rejection)


# Threshold mode and clustering.

from oracle import cluster as ocl  # noqa: E402
from tests import test_oracle_cluster as clpins  # noqa: E402


def test_unscaled_velocity_distance_is_caught(monkeypatch):
    orig = ocl.features
    monkeypatch.setattr(ocl, "features", lambda xs, ys, js, vel, s: orig(xs, ys, js, vel, 1.0))
    assert _fails(clpins.test_groups_equal_sklearn_dbscan_min_samples_1, 0) or \
        _fails(clpins.test_chains_join_and_gaps_split)


def test_groups_without_transitivity_are_caught(monkeypatch):
    # Label each hit by its smallest direct neighbour only (no chaining).
    def direct(adj):
        return np.array([int(np.nonzero(adj[i])[0].min()) for i in range(adj.shape[0])])
    monkeypatch.setattr(ocl, "components", direct)
    assert _fails(clpins.test_chains_join_and_gaps_split)


def test_ties_to_the_largest_index_are_caught(monkeypatch):
    def rev(labels, nu32, xs, ys, js):
        best = {}
        for i in range(labels.size):
            key = (-float(nu32[i]), -int(ys[i]), -int(xs[i]), -int(js[i]))
            lab = int(labels[i])
            if lab not in best or key < best[lab][0]:
                best[lab] = (key, i)
        return np.array([best[int(labels[i])][1] for i in range(labels.size)])
    monkeypatch.setattr(ocl, "representatives", rev)
    assert _fails(clpins.test_representative_is_best_nu_with_ordered_ties)


# Stamps and moments.

from oracle import stamps as ost  # noqa: E402
from tests import test_oracle_stamps as stpins  # noqa: E402


def test_sum_instead_of_mean_is_caught(monkeypatch):
    orig = ost.coadd_stamps

    def summed(img, var, mask, t, vel, xs, ys, js, R, keep=None):
        S = orig(img, var, mask, t, vel, xs, ys, js, R, keep)
        return S * np.asarray(img).shape[0]
    monkeypatch.setattr(ost, "coadd_stamps", summed)
    assert _fails(stpins.test_mean_over_valid_pixels)


def test_moments_about_the_centre_not_the_centroid_are_caught(monkeypatch):
    orig = ost.moments

    def raw(S):
        M00, ub, vb, m20, m02, m11 = orig(S)
        return M00, ub, vb, m20 + ub * ub, m02 + vb * vb, m11 + ub * vb
    monkeypatch.setattr(ost, "moments", raw)
    assert _fails(stpins.test_elongated_source_fails) or \
        _fails(stpins.test_source_beside_the_trajectory_moves_the_centroid) or \
        _fails(stpins.test_point_source_moments_are_the_psf_variance, 1.0, 6)


def test_ignored_keep_mask_is_caught(monkeypatch):
    orig = ost.coadd_stamps
    monkeypatch.setattr(ost, "coadd_stamps",
                        lambda img, var, mask, t, vel, xs, ys, js, R, keep=None:
                        orig(img, var, mask, t, vel, xs, ys, js, R, None))
    assert _fails(stpins.test_excluding_the_flash_image_restores_the_point_source)
