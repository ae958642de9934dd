"""Plain FP64 oracle of the treecode far field (a fast, approximate evaluation of the
far-field sum of eq. (single_layer); the paper leaves fast summation out of scope,
Section 4.1, and names the fast multipole method as the way to O(M) cost).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

What it computes, for points z_j = x_j + i y_j (targets = sources) with weighted forces
F_j = w_j (f_x + i f_y)_j and u = u_x + i u_y:

  u(z_i) = 1/(4 pi mu) sum_{j not in ves(i)} [ -F_j ln|z_i - z_j| + F_j / 2
                                              + (z_i - z_j) conj(F_j / (z_i - z_j)) / 2 ],

which is the Stokeslet sum written with complex numbers: (r.F) r / |r|^2 = F/2 + r conj(F/r)/2
for r = z_i - z_j.  Grouping sources into boxes with centre c and zeta_j = z_j - c, every term is
an analytic function of w = z - c outside the box, expanded in powers of t = 1/w with the power
moments M_k[q] = sum_j q_j zeta_j^k of three charge sets, F, conj(F) and conj(zeta) F: the far
contribution of a box is
    -M_0[F] ln|w| + 1/2 sum_{k=1}^p (M_k[F] t^k + conj(M_k[conj F] t^k)) / k
    + M_0[F] / 2 + (w conj(Phi) - conj(Psi)) / 2,
with Phi = sum_{k=0}^p M_k[F] t^(k+1) (the Cauchy sum of F) and Psi = sum_{k=0}^p
M_k[conj(zeta) F] t^(k+1), truncated after order p.

The tree is a uniform quadtree of depth L over the bounding square of the points (side the larger
extent, centred on the bounding box; a point on the upper edge belongs to the last box).  A target
in leaf B takes, at every level l = 2..L, the boxes of its level-l ancestor's interaction list
(children of the parent's 3 x 3 neighbourhood that are not adjacent to the ancestor) through their
expansions, and the sources of the 3 x 3 leaves around B directly.  Sources of the target's own
vesicle are skipped in the direct part; those lying outside the 3 x 3 leaves, which the expansions
included, are subtracted exactly.  Moments here are summed directly from the points of each box at
each level (no translations), and every quantity is FP64.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Tree:
    x0: float       # lower-left corner of the root square
    y0: float
    side: float     # root square side
    depth: int      # leaf level L
    ix: np.ndarray  # leaf coordinates of every point
    iy: np.ndarray

    def width(self, level):
        return self.side / (1 << level)

    def center(self, level, bx, by):
        w = self.width(level)
        return (self.x0 + (bx + 0.5) * w) + 1j * (self.y0 + (by + 0.5) * w)


def build_tree(X, depth):
    """Uniform quadtree of the given depth over the bounding square of X (2, P)."""
    x, y = np.asarray(X[0], np.float64), np.asarray(X[1], np.float64)
    xlo, xhi, ylo, yhi = x.min(), x.max(), y.min(), y.max()
    side = max(xhi - xlo, yhi - ylo)
    if side == 0.0:
        side = 1.0
    x0 = 0.5 * (xlo + xhi) - 0.5 * side
    y0 = 0.5 * (ylo + yhi) - 0.5 * side
    n = 1 << depth
    wl = side / n
    ix = np.clip(np.floor((x - x0) / wl), 0, n - 1).astype(np.int64)
    iy = np.clip(np.floor((y - y0) / wl), 0, n - 1).astype(np.int64)
    return Tree(x0, y0, side, depth, ix, iy)


def box_moments(z, q, centers, box, nbox, p):
    """M[b, k] = sum_{j in box b} q_j (z_j - c_b)^k, k = 0..p."""
    zeta = z - centers[box]
    pw = np.cumprod(np.concatenate([np.ones((z.size, 1), complex), np.repeat(zeta[:, None], p, axis=1)], axis=1),
                    axis=1)
    M = np.zeros((nbox, p + 1), complex)
    np.add.at(M, box, q[:, None] * pw)
    return M


def far_terms(w, MF, MFc, MPsi):
    """Velocity (times 4 pi mu) at offsets w from box centres given the three moment rows."""
    p = MF.shape[-1] - 1
    t = 1.0 / w
    k = np.arange(1, p + 1)
    tk = t[..., None] ** np.arange(0, p + 2)  # t^0 .. t^(p+1)
    logpart = -MF[..., 0] * np.log(np.abs(w))
    series = 0.5 * (np.sum(MF[..., 1:] / k * tk[..., 1:p + 1], axis=-1)
                    + np.conj(np.sum(MFc[..., 1:] / k * tk[..., 1:p + 1], axis=-1)))
    Phi = np.sum(MF * tk[..., 1:], axis=-1)
    Psi = np.sum(MPsi * tk[..., 1:], axis=-1)
    return logpart + series + 0.5 * MF[..., 0] + 0.5 * (w * np.conj(Phi) - np.conj(Psi))


def direct_terms(zt, zs, F):
    """Stokeslet terms (times 4 pi mu) in real arithmetic, summed over the last axis."""
    r = zt - zs
    rx, ry = r.real, r.imag
    q = rx * rx + ry * ry
    dot = rx * F.real + ry * F.imag
    lg = -0.5 * np.log(q)
    return np.sum(lg * F.real + dot * rx / q, axis=-1) + 1j * np.sum(lg * F.imag + dot * ry / q, axis=-1)


def interaction_offsets():
    """Candidate source boxes relative to a target box: children of the parent's 3 x 3
    neighbourhood; returned as (dx, dy) from the parent's first child, plus adjacency test."""
    return [(a, b) for a in range(-2, 4) for b in range(-2, 4)]


def near_part(tree, z, F, ves, offsets, target):
    """Direct part (times 4 pi mu) shared by every tree method here: the sources of the 3 x 3 leaves
    around each target's leaf, own vesicle skipped, minus the own-vesicle sources outside those leaves
    (which the expansions included).  Zero at targets not selected."""
    P = z.size
    depth = tree.depth
    u = np.zeros(P, complex)
    # 3 x 3 leaves, own vesicle skipped
    n = 1 << depth
    leaf = tree.ix * n + tree.iy
    order_ = np.argsort(leaf, kind="stable")
    starts = np.searchsorted(leaf[order_], np.arange(n * n + 1))
    for lx in range(n):
        for ly in range(n):
            tgt = order_[starts[lx * n + ly]:starts[lx * n + ly + 1]]
            tgt = tgt[target[tgt]]
            if tgt.size == 0:
                continue
            src = np.concatenate([order_[starts[jx * n + jy]:starts[jx * n + jy + 1]]
                                  for jx in range(max(lx - 1, 0), min(lx + 2, n))
                                  for jy in range(max(ly - 1, 0), min(ly + 2, n))])
            keep = ves[src][None, :] != ves[tgt][:, None]
            Fm = np.where(keep, F[src][None, :], 0.0)
            zs = np.where(keep, z[src][None, :], z[tgt][:, None] + 1.0)  # masked terms: F = 0, r = 1
            u[tgt] += direct_terms(z[tgt][:, None], zs, Fm)
    # own-vesicle sources that the expansions included: subtract them exactly
    for v in range(len(offsets) - 1):
        a, b = int(offsets[v]), int(offsets[v + 1])
        if b - a < 2 or not target[a:b].any():
            continue
        far = (np.abs(tree.ix[a:b, None] - tree.ix[None, a:b]) > 1) | (np.abs(tree.iy[a:b, None] - tree.iy[None, a:b]) > 1)
        if not far.any():
            continue
        Fm = np.where(far, F[None, a:b], 0.0)
        zs = np.where(far, z[None, a:b], z[a:b, None] + 1.0)
        u[a:b] -= direct_terms(z[a:b, None], zs, Fm)
    return u


def treecode(X, f, w, offsets, mu, order, depth, sel=None):
    """Treecode far field of all points on themselves, own vesicle excluded: (2, P), or
    (2, len(sel)) at the targets sel only (the tree and moments still use every point)."""
    X = np.asarray(X, np.float64)
    P = X.shape[1]
    z = X[0] + 1j * X[1]
    F = np.asarray(w, np.float64) * (f[0] + 1j * f[1])
    ves = np.repeat(np.arange(len(offsets) - 1), np.diff(np.asarray(offsets, np.int64)))
    tree = build_tree(X, depth)
    p = order
    target = np.zeros(P, bool)
    target[np.arange(P) if sel is None else np.asarray(sel)] = True
    u = np.zeros(P, complex)
    for l in range(2, depth + 1):
        n = 1 << l
        bx, by = tree.ix >> (depth - l), tree.iy >> (depth - l)
        box = bx * n + by
        cx = tree.x0 + (np.arange(n) + 0.5) * tree.width(l)
        cy = tree.y0 + (np.arange(n) + 0.5) * tree.width(l)
        centers = (cx[:, None] + 1j * cy[None, :]).ravel()
        zeta = z - centers[box]
        MF = box_moments(z, F, centers, box, n * n, p)
        MFc = box_moments(z, np.conj(F), centers, box, n * n, p)
        MPsi = box_moments(z, np.conj(zeta) * F, centers, box, n * n, p)
        for a, b in interaction_offsets():
            sx = 2 * (bx >> 1) + a
            sy = 2 * (by >> 1) + b
            ok = (sx >= 0) & (sx < n) & (sy >= 0) & (sy < n) & ((np.abs(sx - bx) > 1) | (np.abs(sy - by) > 1))
            ok &= target
            if not ok.any():
                continue
            s = sx[ok] * n + sy[ok]
            u[ok] += far_terms(z[ok] - centers[s], MF[s], MFc[s], MPsi[s])
    u += near_part(tree, z, F, ves, offsets, target)
    u /= 4.0 * np.pi * mu
    if sel is not None:
        u = u[np.asarray(sel)]
    return np.stack([u.real, u.imag])


def truncation_bound(X, f, w, offsets, mu, order, depth):
    """Per-target bound on |treecode - exact sum| from the truncated series: for a box S of
    radius rho (largest |zeta_j|) seen at |w| from its centre, x = rho / |w| < 1, the dropped
    terms are at most sum_S |F_j| x^(p+1) [1 / ((p+1)(1-x)) + (1+x) / (2 (1-x))] / (4 pi mu)."""
    X = np.asarray(X, np.float64)
    P = X.shape[1]
    z = X[0] + 1j * X[1]
    F = np.asarray(w, np.float64) * (f[0] + 1j * f[1])
    tree = build_tree(X, depth)
    p = order
    bound = np.zeros(P)
    for l in range(2, depth + 1):
        n = 1 << l
        bx, by = tree.ix >> (depth - l), tree.iy >> (depth - l)
        box = bx * n + by
        cx = tree.x0 + (np.arange(n) + 0.5) * tree.width(l)
        cy = tree.y0 + (np.arange(n) + 0.5) * tree.width(l)
        centers = (cx[:, None] + 1j * cy[None, :]).ravel()
        absF = np.zeros(n * n)
        np.add.at(absF, box, np.abs(F))
        rho = np.zeros(n * n)
        np.maximum.at(rho, box, np.abs(z - centers[box]))
        for a, b in interaction_offsets():
            sx = 2 * (bx >> 1) + a
            sy = 2 * (by >> 1) + b
            ok = (sx >= 0) & (sx < n) & (sy >= 0) & (sy < n) & ((np.abs(sx - bx) > 1) | (np.abs(sy - by) > 1))
            s = sx[ok] * n + sy[ok]
            x = rho[s] / np.abs(z[ok] - centers[s])
            bound[ok] += absF[s] * x ** (p + 1) * (1.0 / ((p + 1) * (1 - x)) + (1 + x) / (2 * (1 - x)))
    return bound / (4.0 * np.pi * mu)
