"""The parity checkers themselves (CPU): they accept the oracle's own results
rounded to float32, and reject a planted wrong value, a dropped best
trajectory, a wrong n_obs and a 16-bit error beyond its bound."""
import numpy as np
import pytest

import oracle
from paper_1901_02492_amd import synth
from tests import parity


@pytest.fixture(scope="module")
def case():
    s = synth.random_stack(301, n=7, h=12, w=40, n_vel=30, k=6, psf_size=5, vmax=12.0, tmax=2.0)
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, s.k)
    disp = oracle.displacements(s.t, s.vel)
    ok = oracle.validity(s.img, s.var, s.mask)
    ref["all_Sabs"] = oracle.trajectory_sums(np.abs(ref["psi"]), ref["phi"], ok, disp)[0]
    P = s.img.shape[1] * s.img.shape[2]
    res = [ref["nu"].astype(np.float32), ref["alpha"].astype(np.float32),
           ref["vel"].astype(np.int32), ref["nobs"].astype(np.int16)]
    return s, ref, [r.reshape(P, s.k) for r in res]


def test_member_and_match():
    ja = np.array([[3, 1, 7], [0, 2, 5]])
    jb = np.array([[7, 3, 2], [5, 9, 1]])
    assert parity.member(ja, jb, 10).tolist() == [[True, False, True], [False, False, True]]
    assert parity.match(ja, jb, 10).tolist() == [[1, -1, 0], [-1, -1, 0]]


def test_check_topk_accepts_oracle_and_rejects_mistakes(case):
    s, ref, res = case
    full = parity.oracle_full_as_pixels(ref)
    parity.check_topk(res, *full, s.k)
    bad = [r.copy() for r in res]
    bad[0][5, 0] += 1e-3 * max(1.0, abs(float(bad[0][5, 0])))
    with pytest.raises(AssertionError):
        parity.check_topk(bad, *full, s.k)
    bad = [r.copy() for r in res]
    bad[3][9, 2] += 1
    with pytest.raises(AssertionError):
        parity.check_topk(bad, *full, s.k)
    # drop the best trajectory of a pixel whose 1st and k+1-th values differ clearly
    all_nu = full[0]
    srt = -np.sort(-all_nu, axis=0)
    p = int(np.argmax(srt[0] - srt[s.k]))
    j_out = int(np.argsort(-all_nu[:, p], kind="stable")[s.k])
    bad = [r.copy() for r in res]
    bad[2][p] = np.concatenate([bad[2][p, 1:], [j_out]])
    order = np.argsort(-all_nu[bad[2][p], p], kind="stable")
    bad[2][p] = bad[2][p][order]
    bad[0][p] = all_nu[bad[2][p], p].astype(np.float32)
    bad[1][p] = full[1][bad[2][p], p].astype(np.float32)
    bad[3][p] = full[2][bad[2][p], p].astype(np.int16)
    with pytest.raises(AssertionError):
        parity.check_topk(bad, *full, s.k)


def test_check_lp_candidates_bound(case):
    s, ref, res = case
    # the oracle's own values pass; values moved by 3x the 16-bit bound do not
    parity.check_lp_candidates([r.copy() for r in res], s, ref, "bf16", s.k)
    V = ref["all_nu"].shape[0]
    P = res[0].shape[0]
    bound = parity.lp_bound(ref, "bf16", s.img.shape[0])
    j = res[2].astype(np.int64)
    b = bound[j, np.arange(P)[:, None]]
    bad = [r.copy() for r in res]
    fin = np.isfinite(bad[0])
    p, a = np.argwhere(fin)[0]
    bad[0][p, a] = np.float32(bad[0][p, a] + 3.0 * b[p, a])
    with pytest.raises(AssertionError):
        parity.check_lp_candidates(bad, s, ref, "bf16", s.k)
    assert V == s.vel.shape[0]


def test_check_rescored_recall(case):
    s, ref, res = case
    recall = parity.check_rescored(res, res, s, ref, s.k)
    assert recall == 1.0
    bad = [r.copy() for r in res]
    bad[1][3, 1] = np.float32(bad[1][3, 1] * 1.01 + 1.0)
    with pytest.raises(AssertionError):
        parity.check_rescored(bad, res, s, ref, s.k)
