"""Literal-loop brute force of the search, for tiny stacks only (test helper).

Written directly from the definitions (Sec. 2.1.5 planes, coadd and scores;
Sec. 2.2 linear trajectories) with pure-Python loops and no array slicing, so
that it shares no structure with the vectorised oracle it pins.
"""
import math


def _valid(img, var, mask, i, y, x):
    a, v = float(img[i][y][x]), float(var[i][y][x])
    return (mask is None or int(mask[i][y][x]) == 0) and math.isfinite(a) \
        and math.isfinite(v) and v > 0


def planes(img, var, mask, psf):
    n, h, w = len(img), len(img[0]), len(img[0][0])
    ph, pw = len(psf), len(psf[0])
    cy, cx = ph // 2, pw // 2
    psi = [[[0.0] * w for _ in range(h)] for _ in range(n)]
    phi = [[[0.0] * w for _ in range(h)] for _ in range(n)]
    ok = [[[False] * w for _ in range(h)] for _ in range(n)]
    for i in range(n):
        for y in range(h):
            for x in range(w):
                if not _valid(img, var, mask, i, y, x):
                    continue
                ok[i][y][x] = True
                s1 = s2 = 0.0
                for u in range(ph):
                    for v in range(pw):
                        yy, xx = y + u - cy, x + v - cx
                        if 0 <= yy < h and 0 <= xx < w and _valid(img, var, mask, i, yy, xx):
                            tv = float(psf[u][v])
                            s1 += float(img[i][yy][xx]) / float(var[i][yy][xx]) * tv
                            s2 += tv * tv / float(var[i][yy][xx])
                psi[i][y][x] = s1
                phi[i][y][x] = s2
    return psi, phi, ok


def search(img, var, mask, t, psf, vel, k):
    """Returns (per-trajectory dict keyed by (y, x, j) -> (Psi, Phi, n, nu, alpha),
    top-k dict keyed by (y, x) -> list of j)."""
    n, h, w = len(img), len(img[0]), len(img[0][0])
    psi, phi, ok = planes(img, var, mask, psf)
    t0 = float(t[0])
    traj = {}
    top = {}
    for y in range(h):
        for x in range(w):
            scored = []
            for j in range(len(vel)):
                vx, vy = float(vel[j][0]), float(vel[j][1])
                P = F = 0.0
                c = 0
                for i in range(n):
                    tau = float(t[i]) - t0
                    px = x + math.floor(vx * tau + 0.5)
                    py = y + math.floor(vy * tau + 0.5)
                    if 0 <= px < w and 0 <= py < h and ok[i][py][px]:
                        P += psi[i][py][px]
                        F += phi[i][py][px]
                        c += 1
                if F > 0:
                    nu, al = P / math.sqrt(F), P / F
                else:
                    nu, al = -math.inf, 0.0
                traj[(y, x, j)] = (P, F, c, nu, al)
                scored.append((nu, j))
            scored.sort(key=lambda e: (-e[0], e[1]))
            top[(y, x)] = [j for _, j in scored[:k]]
    return traj, top
