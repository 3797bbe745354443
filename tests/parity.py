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


def member(ja, jb, n_vel):
    """bool [P][ka]: whether ja[p, a] is among jb[p, :] (integer indices in
    [0, n_vel)), without the [P][ka][kb] comparison cube."""
    ja = np.asarray(ja, dtype=np.int64)
    jb = np.asarray(jb, dtype=np.int64)
    P = ja.shape[0]
    base = np.arange(P, dtype=np.int64)[:, None] * n_vel
    kb = np.sort((jb + base).ravel())
    ka = (ja + base).ravel()
    pos = np.minimum(np.searchsorted(kb, ka), kb.size - 1)
    return (kb[pos] == ka).reshape(ja.shape)


def match(ja, jb, n_vel):
    """For every ja[p, a] the column b with jb[p, b] == ja[p, a], or -1."""
    ja = np.asarray(ja, dtype=np.int64)
    jb = np.asarray(jb, dtype=np.int64)
    P, kb_ = jb.shape
    base = np.arange(P, dtype=np.int64)[:, None] * n_vel
    flat = (jb + base).ravel()
    order = np.argsort(flat, kind="stable")
    srt = flat[order]
    ka = (ja + base).ravel()
    pos = np.minimum(np.searchsorted(srt, ka), srt.size - 1)
    found = srt[pos] == ka
    col = np.where(found, order[pos] % kb_, -1)
    return col.reshape(ja.shape)


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
    in_ref = member(j_g, ref_top, V)
    extra_ok = nu_o >= (nu_k - tk)[:, None]
    assert np.all(extra_ok | in_ref), "GPU keeps a trajectory clearly below the k-th"
    in_gpu = member(ref_top, j_g, V)
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


def lp_kcand(lp, k, n_vel):
    """Candidates a 16-bit search keeps before the FP32 re-score selects k:
    k for FP16 (its top-k recall meets 0.999 at K' = K), about 1.25 k for
    BF16 (8 significant bits: at K' = K its recall falls just short)."""
    if lp == "bf16":
        return int(min(n_vel, 64, k + max(2, k // 4)))
    return int(k)


# Unit roundoff of the 16-bit formats (round to nearest even).
LP_U = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def lp_bound(ref, lp, n_img):
    """Bound [V][P] on |nu_16 - nu_FP64| of a 16-bit search: every stored value
    is within u of its float32 plane value (relative; FP16 values below its
    normal range within 2^-25 / s absolute, with s >= 2^13 / max|plane|), the
    float32 planes within 1e-5, and the float32 sums add n_img rounding
    errors; first-order propagation through nu = Psi / sqrt(Phi), doubled."""
    V = ref["all_nu"].shape[0]
    nu = ref["all_nu"].reshape(V, -1)
    phi = ref["all_Phi"].reshape(V, -1)
    S = ref["all_Sabs"].reshape(V, -1)
    e = LP_U[lp] + 1e-5 + n_img * 2.0 ** -24
    tiny = 0.0
    if lp == "f16":
        tiny = n_img * 2.0 ** -25 * max(np.abs(ref["psi"]).max(), ref["phi"].max()) / 2.0 ** 13
    safe = np.where(phi > 0, phi, 1.0)
    dpsi = e * S + tiny
    dphi = e * phi + tiny
    fin = np.isfinite(nu)
    bound = dpsi / np.sqrt(safe) + np.where(fin, np.abs(nu), 0.0) * dphi / (2.0 * safe)
    return 2.0 * bound + tol_nu(nu)


def check_lp_candidates(cand, s, ref, lp, k_cand):
    """The 16-bit search's own lists, before any re-score: exact n_obs and
    velocity indices in range, nu within the propagated 16-bit bound of the
    oracle, and the kept set equal to the oracle's best k_cand up to entries
    within that bound of the k_cand-th value."""
    H, W = s.img.shape[1:]
    P = H * W
    nu_g, al_g, j_g, n_g = [a.reshape(P, k_cand) for a in cand]
    V = ref["all_nu"].shape[0]
    all_nu = ref["all_nu"].reshape(V, P)
    j = j_g.astype(np.int64)
    assert np.all((j >= 0) & (j < V))
    srt = np.sort(j, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1])
    pidx = np.arange(P)[:, None]
    assert np.array_equal(n_g.astype(np.int64), ref["all_nobs"].reshape(V, P)[j, pidx])
    nu_o = all_nu[j, pidx]
    inf_o = np.isneginf(nu_o)
    assert np.array_equal(np.isneginf(nu_g), inf_o)
    bound = lp_bound(ref, lp, s.img.shape[0])
    b_g = bound[j, pidx]
    err = np.abs(nu_g.astype(np.float64) - np.where(inf_o, 0.0, nu_o))
    assert np.all(err[~inf_o] <= b_g[~inf_o]), \
        f"16-bit nu outside its bound: worst ratio {np.max(err[~inf_o] / b_g[~inf_o]):.3f}"
    # the set: the oracle's k_cand-th value per pixel and the band around it
    with np.errstate(invalid="ignore"):
        kth = -np.partition(-all_nu, k_cand - 1, axis=0)[k_cand - 1]
        band = np.where(np.isfinite(bound), bound, 0.0).max(axis=0) * 2.0
        kth_f = np.where(np.isfinite(kth), kth, -np.inf)
        assert np.all(inf_o | (nu_o >= (kth_f - band)[:, None]))
        above = all_nu > (kth_f + band)[None, :]
        kept_above = (nu_o > (kth_f + band)[:, None]).sum(axis=1)
        assert np.array_equal(above.sum(axis=0), kept_above)
    rel = np.abs(nu_g.astype(np.float64) - nu_o) / np.maximum(1.0, np.abs(nu_o))
    return float(np.max(np.where(inf_o, 0.0, rel)))


def check_rescored(res, plain, s, ref, k):
    """Re-scored lists: every value meets the FP32 tolerances against the
    oracle with exact n_obs, equals the plain FP32 path bitwise wherever both
    keep the trajectory, is strictly ordered, and the tie-tolerant recall of
    the oracle's top k (an entry counts when the oracle ranks it in its top k
    or within the nu tolerance of its k-th value) is at least 0.999."""
    H, W = s.img.shape[1:]
    P = H * W
    all_nu, all_al, all_no, all_phi, top = oracle_full_as_pixels(ref)
    nu_g, al_g, j_g, n_g = [a.reshape(P, k) for a in res]
    pidx = np.arange(P)[:, None]
    nu_o = all_nu[j_g, pidx]
    fin = np.isfinite(nu_o)
    assert np.array_equal(n_g.astype(np.int64), all_no[j_g, pidx])
    assert np.all(np.abs(nu_g - nu_o)[fin] <= tol_nu(nu_o)[fin])
    al_o = all_al[j_g, pidx]
    phi_o = all_phi[j_g, pidx]
    atol = RTOL * np.maximum(np.abs(al_o), 1.0 / np.sqrt(np.where(phi_o > 0, phi_o, 1.0)))
    assert np.all(np.abs(al_g - al_o)[fin] <= atol[fin])
    with np.errstate(invalid="ignore"):
        a_, b_ = nu_g[:, :-1], nu_g[:, 1:]
        assert np.all((a_ > b_) | ((a_ == b_) & (j_g[:, :-1] < j_g[:, 1:])))
    p = [a.reshape(P, k) for a in plain]
    V = all_nu.shape[0]
    col = match(j_g, p[2], V)
    rows, slots = np.nonzero(col >= 0)
    for fg, fp in zip((nu_g, al_g, n_g), (p[0], p[1], p[3])):
        assert fg[rows, slots].tobytes() == fp[rows, col[rows, slots]].tobytes()
    kth = all_nu[top[:, k - 1], np.arange(P)]
    lim = np.where(np.isfinite(kth), kth - tol_nu(kth), -np.inf)
    in_top = member(j_g, top, V)
    with np.errstate(invalid="ignore"):
        ok = in_top | (nu_o >= lim[:, None])
    return float(ok.mean())


def check_band(gpu, orc, k):
    """A band of start pixels of the GPU's ranked top-k lists against the C
    oracle's ranked best k_out >= k (tests/..., oracle.cref.search_rows), both
    [B][W][...]: the same rules as check_topk, decided from the oracle's lists
    alone (a GPU entry must be among the oracle's best k_out).
    Returns a dict of counts and worst errors for the caller's summary."""
    nu_g, al_g, j_g, n_g = [np.asarray(a).reshape(-1, k) for a in gpu]
    ko = orc["nu"].shape[-1]
    o_nu = orc["nu"].reshape(-1, ko)
    o_al = orc["alpha"].reshape(-1, ko)
    o_phi = orc["Phi"].reshape(-1, ko)
    o_n = orc["nobs"].reshape(-1, ko)
    o_j = orc["vel"].reshape(-1, ko).astype(np.int64)
    P = nu_g.shape[0]
    j_g = j_g.astype(np.int64)
    n_vel = int(max(o_j.max(), j_g.max())) + 1
    col = match(j_g, o_j, n_vel)
    missing = col < 0
    if missing.any():
        p, a = np.argwhere(missing)[0]
        raise AssertionError(f"GPU keeps velocity {j_g[p, a]} at pixel {p} of the band, "
                             f"outside the oracle's best {ko}")
    rows = np.arange(P)[:, None]
    nu_o, al_o, ph_o, n_o = (x[rows, col] for x in (o_nu, o_al, o_phi, o_n))
    assert np.array_equal(n_g.astype(np.int64), n_o.astype(np.int64)), "n_obs differs"
    inf_o = np.isneginf(nu_o)
    assert np.array_equal(np.isneginf(nu_g), inf_o), "-inf scores differ"
    assert np.all(al_g[inf_o] == 0)
    fin = ~inf_o
    err = np.abs(nu_g.astype(np.float64) - nu_o)
    tn = tol_nu(nu_o)
    assert np.all(err[fin] <= tn[fin]), f"nu max err {err[fin].max()}"
    atol = RTOL * np.maximum(np.abs(al_o), 1.0 / np.sqrt(np.where(ph_o > 0, ph_o, 1.0)))
    aerr = np.abs(al_g.astype(np.float64) - al_o)
    assert np.all(aerr[fin] <= atol[fin]), f"alpha max err {aerr[fin].max()}"
    with np.errstate(invalid="ignore"):
        a_, b_ = nu_g[:, :-1], nu_g[:, 1:]
        assert np.all((a_ > b_) | ((a_ == b_) & (j_g[:, :-1] < j_g[:, 1:]))), \
            "GPU list not ordered by (nu desc, index asc)"
        dec = (nu_o[:, :-1] - nu_o[:, 1:] >= -tol_nu(nu_o[:, :-1])) | inf_o[:, 1:]
        assert np.all(dec), "GPU order contradicts the oracle beyond tolerance"
        kth = o_nu[:, k - 1]
        tk = np.where(np.isfinite(kth), tol_nu(kth), 0.0)
        in_top = col < k
        assert np.all(in_top | (nu_o >= (kth - tk)[:, None])), \
            "GPU keeps a trajectory clearly below the k-th"
        # every one of the oracle's top k clearly above its k-th value is kept
        kept = member(o_j[:, :k], j_g, n_vel)
        assert np.all(kept | (o_nu[:, :k] <= (kth + tk)[:, None])), \
            "GPU drops a trajectory clearly above the k-th"
        # the oracle's lists must reach past the ambiguous entries
        if ko > k:
            last = o_nu[:, ko - 1]
            amb = np.isfinite(kth) & (last >= kth - tk) & ~in_top.all(axis=1)
            assert not amb.any(), "oracle list too short to decide a near-tie"
    recalled = in_top | (nu_o >= (kth - tk)[:, None])
    return dict(pixels=int(P), entries=int(P * k), recalled=int(recalled.sum()),
                near_tie_pixels=int((~in_top).any(axis=1).sum()),
                nu_err=float(np.max(np.where(fin, err / np.maximum(1.0, np.abs(nu_o)), 0.0))),
                alpha_err=float(np.max(np.where(fin, aerr / atol, 0.0))))
