"""Comparison of the HIP path's results with the FP64 oracle (test helper).

Tolerances (float32 arithmetic against the float64 definition):
  nu:     |nu_gpu - nu_ref| <= 1e-5 * max(1, |nu_ref|)
  alpha:  |alpha_gpu - alpha_ref| <= 1e-5 * max(|alpha_ref|, 1/sqrt(Phi_ref))
          (alpha = nu / sqrt(Phi), so the second term is the same bound in
          noise units; it keeps the test meaningful where Psi ~ 0)
  psi:    |psi_gpu - psi_ref| <= 1e-5 * max(1, |psi_ref|);  phi relative 1e-5
  velocity index and n_obs: exact.
Top-k sets must be equal except for entries whose reference nu is within the
nu tolerance of the reference k-th value (near-ties at the cut); the GPU list
must be strictly ordered by (its own nu descending, index ascending), and its
reference values must be non-increasing up to the tolerance.
"""
import numpy as np

RTOL = 1e-5


def tol_nu(ref):
    ref = np.asarray(ref, dtype=np.float64)
    return RTOL * np.maximum(1.0, np.abs(np.where(np.isfinite(ref), ref, 0.0)))


def to_numpy(res):
    return [r.detach().cpu().numpy() for r in res]


def check_planes(planes_gpu, psi, phi, ok):
    """planes_gpu float32 [N][H][W][2] against oracle psi, phi, valid [N][H][W]."""
    pg = planes_gpu[..., 0].astype(np.float64)
    fg = planes_gpu[..., 1]
    fbits = fg.view(np.uint32)
    pbits = planes_gpu[..., 0].view(np.uint32)
    assert np.all(fbits[~ok] == 0) and np.all(pbits[~ok] == 0), "invalid pixels must store +0"
    assert np.all(fbits[ok] != 0), "valid pixels must store a nonzero phi pattern"
    assert np.all(np.abs(pg - psi)[ok] <= (RTOL * np.maximum(1.0, np.abs(psi)))[ok]), \
        f"psi max err {np.max(np.abs(pg - psi)[ok]) if ok.any() else 0}"
    fgd = np.abs(fg.astype(np.float64))
    assert np.all(np.abs(fgd - phi)[ok] <= (RTOL * phi + 1e-30)[ok]), \
        f"phi max rel err {np.max((np.abs(fgd - phi) / np.maximum(phi, 1e-30))[ok])}"


def check_topk(gpu, all_nu, all_alpha, all_nobs, all_phi, ref_top, k):
    with np.errstate(invalid="ignore"):
        return _check_topk(gpu, all_nu, all_alpha, all_nobs, all_phi, ref_top, k)


def _check_topk(gpu, all_nu, all_alpha, all_nobs, all_phi, ref_top, k):
    """gpu = (nu, alpha, vel, nobs) arrays [P][k]; all_* are [V][P]; ref_top [P][k].

    Returns the number of pixels whose set differs from the reference by
    near-ties only (0 in most workloads)."""
    nu_g, al_g, j_g, n_g = [np.asarray(a) for a in gpu]
    P = nu_g.shape[0]
    V = all_nu.shape[0]
    assert nu_g.shape == (P, k) and ref_top.shape == (P, k)
    j_g = j_g.astype(np.int64)
    assert np.all((j_g >= 0) & (j_g < V)), "velocity index out of range"
    srt = np.sort(j_g, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]), "duplicate velocity within a pixel"
    pidx = np.arange(P)[:, None]
    nu_o = all_nu[j_g, pidx]
    al_o = all_alpha[j_g, pidx]
    n_o = all_nobs[j_g, pidx]
    phi_o = all_phi[j_g, pidx]
    bad = n_g.astype(np.int64) != n_o
    assert not bad.any(), f"n_obs differs at {np.argwhere(bad)[:5].tolist()}"
    inf_o = np.isneginf(nu_o)
    assert np.array_equal(np.isneginf(nu_g), inf_o), "-inf scores differ"
    assert np.all(al_g[inf_o] == 0)
    fin = ~inf_o
    err = np.abs(nu_g.astype(np.float64) - nu_o)
    assert np.all(err[fin] <= tol_nu(nu_o)[fin]), f"nu max err {err[fin].max()}"
    atol = RTOL * np.maximum(np.abs(al_o), 1.0 / np.sqrt(np.where(phi_o > 0, phi_o, 1.0)))
    aerr = np.abs(al_g.astype(np.float64) - al_o)
    assert np.all(aerr[fin] <= atol[fin]), f"alpha max err {aerr[fin].max()}"
    # GPU order is strict on its own values.
    a, b = nu_g[:, :-1], nu_g[:, 1:]
    ordered = (a > b) | ((a == b) & (j_g[:, :-1] < j_g[:, 1:]))
    assert np.all(ordered), "GPU list not ordered by (nu desc, index asc)"
    # ...and consistent with the reference up to tolerance.
    dec = nu_o[:, :-1] - nu_o[:, 1:] >= -tol_nu(nu_o[:, :-1])
    dec |= inf_o[:, 1:]
    assert np.all(dec), "GPU order contradicts the reference beyond tolerance"
    # Sets equal up to near-ties at the cut.
    nu_k = all_nu[ref_top[:, k - 1], np.arange(P)]
    tk = np.where(np.isfinite(nu_k), tol_nu(nu_k), 0.0)
    in_ref = (j_g[:, :, None] == ref_top[:, None, :]).any(-1)
    extra_ok = nu_o >= (nu_k - tk)[:, None]
    assert np.all(extra_ok | in_ref), "GPU keeps a trajectory clearly below the k-th"
    in_gpu = (ref_top[:, :, None] == j_g[:, None, :]).any(-1)
    nu_ref_top = all_nu[ref_top, pidx]
    missing_ok = nu_ref_top <= (nu_k + tk)[:, None]
    assert np.all(missing_ok | in_gpu), "GPU drops a trajectory clearly above the k-th"
    return int((~in_ref).any(axis=1).sum())


def oracle_full_as_pixels(ref):
    """Reshape oracle.search() output to the [V][P] / [P][k] form check_topk takes."""
    V, H, W = ref["all_nu"].shape
    P = H * W
    return (ref["all_nu"].reshape(V, P), ref["all_alpha"].reshape(V, P),
            ref["all_nobs"].reshape(V, P), ref["all_Phi"].reshape(V, P),
            ref["vel"].reshape(P, -1))
