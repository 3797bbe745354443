"""FP64 CPU oracle of threshold mode and duplicate clustering (test
infrastructure only).

Nothing in the product path imports, calls or links this module: only the
tests, the package smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library.

What is computed:

  1. Threshold mode (Sec. 2.2 and Sec. 3.2: every trajectory whose nu reaches
     the threshold is kept, nu >= 10 in the HiTS search).  A hit is a start
     pixel (x, y) and velocity index j with nu(x, y, j) >= m; the search's
     own scores (Sec. 2.1.5) decide.
  2. Duplicate clustering (Sec. 3.3, last paragraph: trajectories are grouped
     by start pixel and velocity with DBSCAN and the most likely one of each
     group is kept).  The paper gives no DBSCAN parameters; the reading used
     is DBSCAN with min_samples = 1, under which every hit is a core point
     and the groups are the connected components of the graph joining hits
     within distance eps.  The distance is Euclidean over (x, y, s*vx, s*vy),
     the velocity scaled by a time s (days) so that it is a position offset:
         d2 = ((dx*dx + dy*dy) + du*du) + dv*dv,
         dx = x - x', dy = y - y', du = s*vx - s*vx', dv = s*vy - s*vy'
     in IEEE double in that order; two hits are joined when d2 <= eps*eps.
     The representative of a group is its hit with the largest nu (as stored
     in float32), ties to the smallest (y, x, j).
"""
from __future__ import annotations

import numpy as np

__all__ = ["threshold_hits", "features", "pairs_within", "components", "representatives",
           "cluster", "pairs_within_sparse", "components_sparse", "cluster_sparse"]


def threshold_hits(all_nu, m):
    """(ys, xs, js) of every trajectory with nu >= m, from per-trajectory
    scores all_nu [V][H][W] (step 1), in (y, x, j) order."""
    js, ys, xs = np.nonzero(np.asarray(all_nu) >= m)
    order = np.lexsort((js, xs, ys))
    return ys[order], xs[order], js[order]


def features(xs, ys, js, vel, s):
    """Clustering coordinates (x, y, s*vx, s*vy) in float64 [n][4]."""
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    js = np.asarray(js, dtype=np.int64)
    return np.stack([np.asarray(xs, dtype=np.float64), np.asarray(ys, dtype=np.float64),
                     s * vel[js, 0], s * vel[js, 1]], axis=1)


def pairs_within(f, eps):
    """Boolean [n][n]: d2 <= eps^2 with d2 summed in the order of step 2."""
    dx = f[:, None, 0] - f[None, :, 0]
    dy = f[:, None, 1] - f[None, :, 1]
    du = f[:, None, 2] - f[None, :, 2]
    dv = f[:, None, 3] - f[None, :, 3]
    d2 = ((dx * dx + dy * dy) + du * du) + dv * dv
    return d2 <= float(eps) * float(eps)


def components(adj):
    """Connected components of a symmetric adjacency matrix by union-find;
    each node's label is the smallest node index of its component."""
    n = adj.shape[0]
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    ii, jj = np.nonzero(np.triu(adj, 1))
    for a, b in zip(ii.tolist(), jj.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            lo, hi = min(ra, rb), max(ra, rb)
            parent[hi] = lo
    return np.array([find(a) for a in range(n)], dtype=np.int64)


def representatives(labels, nu32, xs, ys, js):
    """For every hit, the index of its group's representative: the largest
    float32 nu, ties to the smallest (y, x, j)."""
    n = labels.size
    best = {}
    for i in range(n):
        key = (-float(nu32[i]), int(ys[i]), int(xs[i]), int(js[i]))
        lab = int(labels[i])
        if lab not in best or key < best[lab][0]:
            best[lab] = (key, i)
    return np.array([best[int(labels[i])][1] for i in range(n)], dtype=np.int64)


def cluster(xs, ys, js, nu32, vel, s, eps):
    """Step 2 for hits (xs, ys, js) with float32 scores nu32: returns the
    representative index of every hit and the component labels."""
    f = features(xs, ys, js, vel, s)
    labels = components(pairs_within(f, eps))
    return representatives(labels, nu32, xs, ys, js), labels


def pairs_within_sparse(f, eps):
    """The pairs (a, b), a < b, with d2 <= eps^2 (step 2's test, in its order),
    for many hits: candidate pairs from a k-d tree query at a radius slightly
    above eps (a library routine), each then decided by the exact test."""
    from scipy.spatial import cKDTree
    f = np.asarray(f, dtype=np.float64)
    ok = np.all(np.isfinite(f), axis=1)
    idx = np.nonzero(ok)[0]
    if idx.size < 2:
        return np.zeros((0, 2), dtype=np.int64)
    tree = cKDTree(f[idx])
    cand = tree.query_pairs(r=float(eps) * (1.0 + 1e-9) + 1e-300, output_type="ndarray")
    if cand.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    a, b = idx[cand[:, 0]], idx[cand[:, 1]]
    d = f[a] - f[b]
    d2 = ((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]) + d[:, 3] * d[:, 3]
    keep = d2 <= float(eps) * float(eps)
    lo, hi = np.minimum(a, b)[keep], np.maximum(a, b)[keep]
    return np.stack([lo, hi], axis=1)


def components_sparse(n, pairs):
    """Connected components of n nodes joined by `pairs` (a library routine);
    each node's label is the smallest node index of its component."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    g = coo_matrix((np.ones(pairs.shape[0]), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    smallest = np.full(lab.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(smallest, lab, np.arange(n))
    return smallest[lab]


def cluster_sparse(xs, ys, js, nu32, vel, s, eps):
    """cluster() for many hits: the same groups and representatives, with the
    pairs found by pairs_within_sparse instead of the dense n x n test."""
    js = np.asarray(js, dtype=np.int64)
    nv = np.asarray(vel).reshape(-1, 2).shape[0]
    bad = (js < 0) | (js >= nv)
    f = features(xs, ys, np.where(bad, 0, js), vel, s)
    f[bad] = np.nan                             # outside the grid: a group of its own
    labels = components_sparse(f.shape[0], pairs_within_sparse(f, eps))
    return representatives(labels, nu32, xs, ys, js), labels
