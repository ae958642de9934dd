"""Plain FP64 oracle of the fast-multipole far field (a fast, approximate evaluation of the far-field
sum of eq. (single_layer); the paper evaluates the sum directly, names the fast multipole method as
the route to O(M) cost and leaves it out of scope, Section 4.1).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The tree, the interaction lists, the direct part and the own-vesicle correction are those of the
treecode (oracle.treecode).  The two differ in how a far box S acts on a target z whose level-l
ancestor is the box T, S in T's interaction list: the treecode evaluates the truncated multipole
series of S at z; the fast multipole method replaces every analytic function in that series by its
Taylor polynomial of degree p about the centre c_T of T, and evaluates the polynomial at z.

With complex numbers (z = x + i y, F_j = w_j (f_x + i f_y)_j, u = u_x + i u_y, r = z - z_j) the
Stokeslet term times 4 pi mu is -F ln|r| + F/2 + r conj(F/r)/2.  Since 2 ln|r| = log r + conj(log r)
(for any branch of log r) and r conj(F/r) = z conj(F/r) - conj(conj(z_j) F / r), a box of sources acts
through four analytic functions of z,
    A = sum_j F_j log(z - z_j),        Q = sum_j conj(F_j) log(z - z_j),
    Phi = sum_j F_j / (z - z_j),       G = sum_j conj(z_j) F_j / (z - z_j),
as  u = -A/2 - conj(Q)/2 + z conj(Phi)/2 - conj(G)/2 + M_0[F]/2,  the same branch of log in A and Q
(its imaginary part then cancels).  About the box centre c, with the power moments
M_k[q] = sum_j q_j (z_j - c)^k, the multipole series truncated after order p (the treecode's) are
    A = M_0[F] log(z - c) - sum_{m=1}^p M_m[F] / m (z - c)^-m,    Q the same with conj F,
    Phi = sum_{m=1}^{p+1} M_{m-1}[F] (z - c)^-m,                  G = sum_{m=1}^{p+1} M_{m-1}[conj(z_j) F] (z - c)^-m.
Their Taylor coefficients of order l about c_T, with D = c_T - c, follow from the derivatives:
    (z - c)^-m :  (-1)^l C(m + l - 1, l) D^-(m + l);
    log(z - c) :  log D  (l = 0),   (-1)^(l - 1) D^-l / l  (l >= 1),
with the principal log D (any fixed branch would do).  Moments are summed directly from the points
of every box at every level, each level's Taylor polynomials are evaluated about that level's
ancestor (no translation between levels), and everything is FP64.
"""
from math import comb

import numpy as np

from .treecode import box_moments, build_tree, interaction_offsets, near_part


def taylor_coeffs(lam, alpha, D, p):
    """Taylor coefficients of orders 0..p about c_T of  lam log(z - c) + sum_{m>=1} alpha_m (z - c)^-m,
    D = c_T - c.  lam (n,), alpha (n, mmax) for m = 1..mmax, D (n,); returns (n, p + 1)."""
    lam = np.asarray(lam, complex)
    alpha = np.asarray(alpha, complex)
    D = np.asarray(D, complex)
    mmax = alpha.shape[1]
    m = np.arange(1, mmax + 1)
    Dinv = 1.0 / D
    out = np.zeros((D.size, p + 1), complex)
    for l in range(p + 1):
        binom = np.array([float(comb(mm + l - 1, l)) for mm in m])
        out[:, l] = (-1.0) ** l * np.sum(alpha * binom[None, :] * Dinv[:, None] ** (m[None, :] + l), axis=1)
    out[:, 0] += lam * np.log(D)
    for l in range(1, p + 1):
        out[:, l] += lam * (-1.0) ** (l - 1) * Dinv ** l / l
    return out


def multipole_coeffs(MF, MFc, MG, p):
    """(lam, alpha) of A, Q, Phi, G for boxes with moment rows MF = M_k[F], MFc = M_k[conj F],
    MG = M_k[conj(z_j) F], k = 0..p; alpha over m = 1..p+1."""
    nbox = MF.shape[0]
    m = np.arange(1, p + 1)
    aA = np.zeros((nbox, p + 1), complex)
    aA[:, :p] = -MF[:, 1:] / m
    aQ = np.zeros((nbox, p + 1), complex)
    aQ[:, :p] = -MFc[:, 1:] / m
    zero = np.zeros(nbox, complex)
    return {"A": (MF[:, 0], aA), "Q": (MFc[:, 0], aQ), "Phi": (zero, MF.copy()), "G": (zero, MG.copy())}


def polyval(c, zeta):
    """sum_l c[..., l] zeta^l."""
    p = c.shape[-1] - 1
    return np.sum(c * zeta[..., None] ** np.arange(p + 1), axis=-1)


def fmm(X, f, w, offsets, mu, order, depth, sel=None):
    """Fast-multipole far field of all points on themselves, own vesicle excluded: (2, P), or
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
        MF = box_moments(z, F, centers, box, n * n, p)
        MFc = box_moments(z, np.conj(F), centers, box, n * n, p)
        MG = box_moments(z, np.conj(z) * F, centers, box, n * n, p)
        coef = multipole_coeffs(MF, MFc, MG, p)
        # Taylor polynomials about the centres of the boxes that hold a selected target, summed over
        # each box's interaction list
        tb = np.unique(box[target])
        tx, ty = tb // n, tb % n
        loc = {key: np.zeros((tb.size, p + 1), complex) for key in coef}
        K = np.zeros(tb.size, complex)
        for a, b in interaction_offsets():
            sx = 2 * (tx >> 1) + a
            sy = 2 * (ty >> 1) + b
            ok = (sx >= 0) & (sx < n) & (sy >= 0) & (sy < n) & ((np.abs(sx - tx) > 1) | (np.abs(sy - ty) > 1))
            if not ok.any():
                continue
            s = sx[ok] * n + sy[ok]
            D = centers[tb[ok]] - centers[s]
            for key, (lam, alpha) in coef.items():
                loc[key][ok] += taylor_coeffs(lam[s], alpha[s], D, p)
            K[ok] += MF[s, 0]
        # evaluate at the selected targets
        idx = np.flatnonzero(target)
        row = np.searchsorted(tb, box[idx])
        zeta = z[idx] - centers[box[idx]]
        Av, Qv, Pv, Gv = (polyval(loc[key][row], zeta) for key in ("A", "Q", "Phi", "G"))
        u[idx] += -0.5 * Av - 0.5 * np.conj(Qv) + 0.5 * z[idx] * np.conj(Pv) - 0.5 * np.conj(Gv) + 0.5 * K[row]
    u += near_part(tree, z, F, ves, offsets, target)
    u /= 4.0 * np.pi * mu
    if sel is not None:
        u = u[np.asarray(sel)]
    return np.stack([u.real, u.imag])


def truncation_bound(X, f, w, offsets, mu, order, depth, n_radii=16):
    """Per-target bound on |fmm - exact sum|.  For a target z with ancestor T (centre c_T, r = |z - c_T|)
    and a box S of its interaction list (centre c, radius rho = max |z_j - c|, Q = sum_S |F_j|,
    D = |c_T - c|), the error is the multipole truncation at z (the treecode's term, with
    x = rho / |z - c|) plus the Taylor remainder of the truncated series.  In exact arithmetic the
    latter is -dA/2 - conj(dQ)/2 + (z - c) conj(dPhi)/2 - conj(dPsi)/2 with Psi = G - conj(c) Phi, and for
    each function, analytic on the disc |z' - c_T| < D, Cauchy's estimate on a circle of radius R,
    r < R <= D - rho, gives |d.| <= max_circle |.| (r/R)^(p+1) / (1 - r/R); on that circle
    s = |z' - c| >= D - R, y = rho / s <= 1 and
      |A|, |Q| <= Q (max(|ln s|, |ln(D + R)|) + 3 pi / 2 + sum_{m=1}^p y^m / m),
      |Phi| <= Q / s sum_{k=0}^p y^k,   |Psi| <= Q sum_{k=1}^{p+1} y^k.
    The smallest bound over n_radii radii is taken."""
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
        r = np.abs(z - centers[box])
        for a, b in interaction_offsets():
            sx = 2 * (bx >> 1) + a
            sy = 2 * (by >> 1) + b
            ok = (sx >= 0) & (sx < n) & (sy >= 0) & (sy < n) & ((np.abs(sx - bx) > 1) | (np.abs(sy - by) > 1))
            ok &= absF[np.where(ok, sx * n + sy, 0)] > 0  # boxes without force contribute nothing
            s_ = sx[ok] * n + sy[ok]
            q, rh, rt = absF[s_], rho[s_], r[ok]
            x = rh / np.abs(z[ok] - centers[s_])
            mult = q * x ** (p + 1) * (1.0 / ((p + 1) * (1 - x)) + (1 + x) / (2 * (1 - x)))
            D = np.abs(centers[box[ok]] - centers[s_])
            best = np.full(q.size, np.inf)
            for k in range(1, n_radii + 1):
                R = rt + (D - rh - rt) * k / n_radii
                s = D - R
                y = np.minimum(rh / s, 1.0)
                ys = y[:, None] ** np.arange(0, p + 2)
                logs = np.maximum(np.abs(np.log(s)), np.abs(np.log(D + R))) + 1.5 * np.pi
                mA = q * (logs + np.sum(ys[:, 1:p + 1] / np.arange(1, p + 1), axis=1))
                mPhi = q / s * np.sum(ys[:, :p + 1], axis=1)
                mPsi = q * np.sum(ys[:, 1:p + 2], axis=1)
                ratio = rt / R
                tail = ratio ** (p + 1) / (1 - ratio)
                cand = tail * (mA + 0.5 * (D + rt) * mPhi + 0.5 * mPsi)
                best = np.minimum(best, np.where(R > rt, cand, np.inf))
            bound[ok] += mult + best
    return bound / (4.0 * np.pi * mu)
