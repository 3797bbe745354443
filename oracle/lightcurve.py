"""FP64 CPU oracle of the light-curve outlier filter (test infrastructure only).

Nothing in the product path imports, calls or links this module: only the
tests, the package smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library.

What is computed (Sec. 3.3, filtering of candidate trajectories): after the
search, each candidate's light curve (its per-image likelihood values along
the trajectory) is run through a Kalman-type filter; observations more than
five standard deviations from the filter's flux estimate at that observation
are dropped, and the likelihood is recomputed from the remaining ones.  The
paper names the filter only as a Kalman-filter variant, so the
variant below is a reading of that passage:

  1. Observations.  Image i observes candidate (x0, y0, j) when the trajectory
     pixel (Sec. 2.2 displacements) is inside the frame and valid.  Its flux
     estimate is psi_i / phi_i with variance 1 / phi_i (the single-image case
     of the Sec. 2.1.5 maximum-likelihood flux and its Fisher information).
  2. Flux model.  The flux follows a random walk in time with variance q per
     day (q = 0: a constant flux), started from a flat prior.
  3. Filter.  The Kalman filter in information form (J = 1/variance,
     H = mean/variance) runs forward over the observations in image order and
     backward in reverse order.  Between consecutive observations the
     prediction step widens the variance by q * dtau:
         d = 1 + (q * dtau) * J,   J <- J / d,   H <- H / d,
     with dtau the difference of the two tau_i = t_i - t_0; an update adds
     (phi_i, psi_i) to (J, H).  The estimate at observation k that does not
     use observation k itself combines the forward prediction into k with the
     backward prediction into k: J_k = Jf_k + Jb_k, H_k = Hf_k + Hb_k.
  4. Outlier test.  The residual psi_k/phi_k - H_k/J_k has variance
     1/phi_k + 1/J_k, so its squared standardised value is
         r_k = (a * a) / ((phi_k * J_k) * (J_k + phi_k)),  a = psi_k * J_k - phi_k * H_k
     (0 where J_k = 0, i.e. no other observation, or phi_k = 0).  An estimate
     pulled by an outlier is not a best fit, so outliers leave one at a time:
     the observation with the largest r_k (the lowest image index among equal
     values) is dropped if r_k > c^2 (c = 5 in the paper), the filter is run
     again on the observations left, and so on until every remaining one lies
     within c standard deviations of the estimate from the others.
  5. Refit.  Psi' and Phi' are the sums of psi_i and phi_i over the kept
     observations in increasing image order; nu' = Psi'/sqrt(Phi') and
     alpha' = Psi'/Phi' (Sec. 2.1.5), or nu' = -inf, alpha' = 0 when nothing
     with Phi' > 0 remains; n_obs' counts the kept observations.

Every step is a separate IEEE double operation in the order written above, so
that a reject decision is reproducible exactly from the same float32 planes.
Candidates are vectorised; images run in a Python loop.
"""
from __future__ import annotations

import numpy as np

from .core import displacements, scores

__all__ = ["light_curves", "light_curves_at", "kalman_loo", "residual_ratio", "clip", "refit",
           "filter_curves", "lightcurve_filter"]


def light_curves(psi, phi, ok, t, vel, ys, xs, js):
    """Per-image values along each candidate trajectory (Sec. 2.2, Sec. 3.3).

    psi, phi, ok: planes [N][H][W] and their validity.  Candidate c starts at
    (xs[c], ys[c]) with velocity index js[c]; an index outside the grid gives
    a candidate with no observations.  Returns lc_psi, lc_phi (float64 [C][N],
    zero where not observed) and obs (bool [C][N]).
    """
    psi = np.asarray(psi, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    ok = np.asarray(ok, dtype=bool)
    n, h, w = psi.shape
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    js = np.asarray(js, dtype=np.int64)
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    disp = displacements(t, vel)
    good = (js >= 0) & (js < vel.shape[0])
    d = disp[np.where(good, js, 0)]                      # [C][N][2]
    yy = ys[:, None] + d[:, :, 1]
    xx = xs[:, None] + d[:, :, 0]
    inb = good[:, None] & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
    img = np.broadcast_to(np.arange(n)[None, :], inb.shape)
    lc_psi = np.zeros(inb.shape)
    lc_phi = np.zeros(inb.shape)
    obs = np.zeros(inb.shape, dtype=bool)
    lc_psi[inb] = psi[img[inb], yy[inb], xx[inb]]
    lc_phi[inb] = phi[img[inb], yy[inb], xx[inb]]
    obs[inb] = ok[img[inb], yy[inb], xx[inb]]
    lc_psi[~obs] = 0.0
    lc_phi[~obs] = 0.0
    return lc_psi, lc_phi, obs


def light_curves_at(plane_fn, n, h, w, t, vel, ys, xs, js):
    """As light_curves, evaluating the planes only at the visited pixels:
    plane_fn(i, yy, xx) -> (psi, phi, valid) for in-frame pixels of image i."""
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    js = np.asarray(js, dtype=np.int64)
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    disp = displacements(t, vel)
    good = (js >= 0) & (js < vel.shape[0])
    d = disp[np.where(good, js, 0)]
    lc_psi = np.zeros((js.size, n))
    lc_phi = np.zeros((js.size, n))
    obs = np.zeros((js.size, n), dtype=bool)
    for i in range(n):
        yy = ys + d[:, i, 1]
        xx = xs + d[:, i, 0]
        inb = good & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
        if not inb.any():
            continue
        ps, ph, ok = plane_fn(i, yy[inb], xx[inb])
        sel = np.nonzero(inb)[0]
        ok = np.asarray(ok, dtype=bool)
        obs[sel, i] = ok
        lc_psi[sel[ok], i] = np.asarray(ps, dtype=np.float64)[ok]
        lc_phi[sel[ok], i] = np.asarray(ph, dtype=np.float64)[ok]
    return lc_psi, lc_phi, obs


def _one_direction(lc_psi, lc_phi, obs, tau, q, order):
    """Information-form Kalman filter over the images in `order`: the prior
    (J, H) at each observation, before its own update (step 3)."""
    c, n = lc_psi.shape
    Jp = np.zeros((c, n))
    Hp = np.zeros((c, n))
    J = np.zeros(c)
    H = np.zeros(c)
    tp = np.zeros(c)
    seen = np.zeros(c, dtype=bool)
    for i in order:
        o = obs[:, i]
        if q > 0:
            pred = o & seen
            dtau = np.abs(tau[i] - tp)
            s = q * dtau
            d = 1.0 + s * J
            J = np.where(pred, J / d, J)
            H = np.where(pred, H / d, H)
        Jp[:, i] = np.where(o, J, 0.0)
        Hp[:, i] = np.where(o, H, 0.0)
        J = np.where(o, J + lc_phi[:, i], J)
        H = np.where(o, H + lc_psi[:, i], H)
        tp = np.where(o, tau[i], tp)
        seen |= o
    return Jp, Hp


def kalman_loo(lc_psi, lc_phi, obs, tau, q):
    """(J_k, H_k): the filter's information about the flux at observation k
    from every other observation (step 3).  Zero where not observed."""
    n = lc_psi.shape[1]
    tau = np.asarray(tau, dtype=np.float64)
    Jf, Hf = _one_direction(lc_psi, lc_phi, obs, tau, q, range(n))
    Jb, Hb = _one_direction(lc_psi, lc_phi, obs, tau, q, range(n - 1, -1, -1))
    return Jf + Jb, Hf + Hb


def residual_ratio(lc_psi, lc_phi, obs, J, H):
    """Squared standardised residual r_k of each observation against the
    estimate from the others (step 4); 0 where it is not defined."""
    a = lc_psi * J - lc_phi * H
    d = (lc_phi * J) * (J + lc_phi)
    pos = obs & (d > 0)
    return np.where(pos, (a * a) / np.where(pos, d, 1.0), 0.0)


def clip(lc_psi, lc_phi, obs, tau, q, sigma_cut):
    """Observations dropped by the iterated outlier test (steps 3 and 4)."""
    c2 = float(sigma_cut) * float(sigma_cut)
    tau = np.asarray(tau, dtype=np.float64)
    keep = obs.copy()
    rows = np.arange(obs.shape[0])
    active = np.ones(obs.shape[0], dtype=bool)
    while active.any():
        J, H = kalman_loo(lc_psi, lc_phi, keep, tau, q)
        r = residual_ratio(lc_psi, lc_phi, keep, J, H)
        worst = np.argmax(r, axis=1)          # first index among equal maxima
        drop = active & (r[rows, worst] > c2)
        keep[rows[drop], worst[drop]] = False
        active = drop
    return obs & ~keep


def refit(lc_psi, lc_phi, keep):
    """nu', alpha', n_obs' from the kept observations, summed in image order (step 5)."""
    c, n = lc_psi.shape
    P = np.zeros(c)
    F = np.zeros(c)
    for i in range(n):
        P = np.where(keep[:, i], P + lc_psi[:, i], P)
        F = np.where(keep[:, i], F + lc_phi[:, i], F)
    nu, alpha = scores(P, F)
    return nu, alpha, keep.sum(axis=1)


def filter_curves(lc_psi, lc_phi, obs, t, sigma_cut=5.0, q=0.0):
    """Steps 3 to 5 on given light curves: dict(nu, alpha, nobs, rejected)."""
    t = np.asarray(t, dtype=np.float64)
    rej = clip(lc_psi, lc_phi, obs, t - t[0], q, sigma_cut)
    nu, alpha, nobs = refit(lc_psi, lc_phi, obs & ~rej)
    return dict(nu=nu, alpha=alpha, nobs=nobs, rejected=rej)


def lightcurve_filter(psi, phi, ok, t, vel, ys, xs, js, sigma_cut=5.0, q=0.0):
    """The whole filter for candidates (ys, xs, js).

    Returns dict(nu, alpha, nobs, rejected) with rejected a bool [C][N] mask
    of the dropped observations, plus the light curves (lc_psi, lc_phi, obs)
    for the tests.
    """
    lc_psi, lc_phi, obs = light_curves(psi, phi, ok, t, vel, ys, xs, js)
    out = filter_curves(lc_psi, lc_phi, obs, t, sigma_cut, q)
    out.update(lc_psi=lc_psi, lc_phi=lc_phi, obs=obs)
    return out
