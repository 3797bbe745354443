"""Pins of the threshold/clustering oracle against facts that do not come from it.

* Its groups are scikit-learn's DBSCAN clusters with min_samples = 1 on the
  same coordinates (random points kept away from the eps boundary).
* Groups are unions of chains: points on a line spaced just under eps form
  one group, spaced just over eps form singletons.
* The representative is the group's best nu; ties go to the smallest (y, x, j).
* Threshold hits are exactly the trajectories whose score reaches m.
"""
import numpy as np
import pytest

import oracle
from oracle import cluster as oc
from paper_1901_02492_amd import synth


def _partition(labels):
    groups = {}
    for i, l in enumerate(labels):
        groups.setdefault(int(l), []).append(i)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_groups_equal_sklearn_dbscan_min_samples_1(seed):
    from sklearn.cluster import DBSCAN
    rng = np.random.default_rng(seed)
    n = 400
    xs = rng.integers(0, 60, n)
    ys = rng.integers(0, 60, n)
    vel = rng.uniform(-30.0, 30.0, (50, 2))
    js = rng.integers(0, 50, n)
    s, eps = 0.37, 4.3
    f = oc.features(xs, ys, js, vel, s)
    d = np.sqrt(((f[:, None, :] - f[None, :, :]) ** 2).sum(axis=2))
    near = np.abs(d - eps) < 1e-6
    assert not near.any()                       # no pair sits on the boundary
    lab_sk = DBSCAN(eps=eps, min_samples=1).fit(f).labels_
    lab = oc.components(oc.pairs_within(f, eps))
    assert _partition(lab) == _partition(lab_sk)
    assert len(set(lab.tolist())) > 20 and len(set(lab.tolist())) < n


def test_chains_join_and_gaps_split():
    vel = np.zeros((1, 2))
    xs = np.arange(10) * 3
    ys = np.zeros(10, dtype=np.int64)
    js = np.zeros(10, dtype=np.int64)
    f = oc.features(xs, ys, js, vel, 1.0)
    assert len(set(oc.components(oc.pairs_within(f, 3.0)).tolist())) == 1
    assert len(set(oc.components(oc.pairs_within(f, 2.999)).tolist())) == 10
    # Velocity differences count as s * dv pixels.
    vel2 = np.array([[0.0, 0.0], [10.0, 0.0]])
    f2 = oc.features([0, 0], [0, 0], [0, 1], vel2, 0.2)     # 2 px apart
    assert oc.pairs_within(f2, 2.0)[0, 1] and not oc.pairs_within(f2, 1.99)[0, 1]


def test_representative_is_best_nu_with_ordered_ties():
    xs = np.array([5, 4, 6, 9])
    ys = np.array([1, 1, 0, 1])
    js = np.array([3, 2, 7, 0])
    nu = np.array([12.0, 12.0, 11.0, 30.0], dtype=np.float32)
    labels = np.array([0, 0, 0, 3])
    rep = oc.representatives(labels, nu, xs, ys, js)
    # hits 0 and 1 tie on nu; (y, x) = (1, 4) < (1, 5) wins.
    assert rep.tolist() == [1, 1, 1, 3]


def test_threshold_hits_are_the_trajectories_at_or_above_m():
    s = synth.small_stack()
    ref = oracle.search(s.img, s.var, s.mask, s.t, s.psf, s.vel, 1)
    nu = ref["all_nu"]
    m = 8.0
    ys, xs, js = oc.threshold_hits(nu, m)
    assert ys.size == int((nu >= m).sum()) and ys.size > 0
    assert (nu[js, ys, xs] >= m).all()
    # The source at (20, 30) moving (40, 25) px/d is among them.
    j_true = int(np.nonzero((s.vel[:, 0] == 40.0) & (s.vel[:, 1] == 20.0))[0][0])
    assert any((y, x, j) == (30, 20, j_true) for y, x, j in zip(ys, xs, js))


@pytest.mark.parametrize("seed,eps,s", [(0, 2.0, 0.5), (1, 3.0, 1.0), (2, 1.0, 0.0),
                                        (3, 0.0, 1.0), (4, 4.0, 2.24)])
def test_sparse_pairs_equal_the_dense_test(seed, eps, s):
    """The k-d tree candidate pairs with the exact test give the dense test's
    groups and representatives, on integer positions and a coarse velocity
    grid where distances of exactly eps are common (they join)."""
    rng = np.random.default_rng(900 + seed)
    n = 1500
    vel = np.stack(np.meshgrid(np.arange(-3.0, 4.0), np.arange(-2.0, 3.0)), -1).reshape(-1, 2)
    xs = rng.integers(0, 40, n)
    ys = rng.integers(0, 30, n)
    js = rng.integers(0, vel.shape[0], n)
    nu = rng.integers(0, 5, n).astype(np.float32)       # many ties
    rep_d, lab_d = oc.cluster(xs, ys, js, nu, vel, s, eps)
    rep_s, lab_s = oc.cluster_sparse(xs, ys, js, nu, vel, s, eps)
    assert np.array_equal(lab_d, lab_s)
    assert np.array_equal(rep_d, rep_s)
    d = oc.pairs_within(oc.features(xs, ys, js, vel, s), eps)
    p = oc.pairs_within_sparse(oc.features(xs, ys, js, vel, s), eps)
    assert p.shape[0] == int(np.triu(d, 1).sum())


def test_sparse_clustering_puts_out_of_grid_hits_alone():
    vel = np.array([[0.0, 0.0], [1.0, 0.0]])
    xs, ys = np.array([5, 5, 5]), np.array([7, 7, 8])
    js = np.array([0, 7, 1])
    nu = np.array([1.0, 9.0, 2.0], np.float32)
    rep, lab = oc.cluster_sparse(xs, ys, js, nu, vel, 1.0, 2.0)
    assert lab.tolist() == [0, 1, 0] and rep.tolist() == [2, 1, 2]
