"""Seeded synthetic vesicle suspensions shaped like the paper's workloads.

This module only builds *inputs*: membrane points, force densities, arclength
quadrature weights and the vesicle partition.  It contains none of the
far-field arithmetic, so both the CPU oracle and the GPU path can take their
inputs from it.

Shapes follow the paper's setting (Section 2, "Vesicle flows"): every vesicle is
a closed curve sampled at N points alpha_k = 2*pi*k/N, counter-clockwise.  As
in the paper's experiments the membranes are ellipses of perimeter 2*pi
(reduced area nu = 4*pi*A/L^2, which for L = 2*pi is simply a*b).  The trapezoid
rule of Section 2.2.1 needs the arclength element, so the weight of point k is
w_k = |X'(alpha_k)| * 2*pi/N, evaluated analytically for the ellipse.

Layout (the layout the C-ABI consumes):
  X        float64 [2][P]   planar SoA, row 0 = x, row 1 = y
  f        float64 [2][P]   force density (not multiplied by w)
  w        float64 [P]
  offsets  int32   [M+1]    vesicle v owns points offsets[v] .. offsets[v+1]-1
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
import tempfile

import numpy as np
from scipy.optimize import brentq
from scipy.spatial import cKDTree
from scipy.special import ellipe

GENERATOR_VERSION = 4
BASE_SEED = 260625569
PERIMETER = 2.0 * np.pi


@dataclasses.dataclass
class Suspension:
    X: np.ndarray          # (2, P) float64
    f: np.ndarray          # (2, P) float64
    w: np.ndarray          # (P,) float64
    offsets: np.ndarray    # (M+1,) int32
    mu: float
    box: float
    centers: np.ndarray    # (M, 2) ellipse centres
    axes: np.ndarray       # (M, 2) semi-axes (a, b)
    angles: np.ndarray     # (M,) rotation angles

    @property
    def n_points(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_vesicles(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def cross_pairs(self) -> int:
        """Number of cross-vesicle (target, source) pairs: P^2 - sum_v N_v^2."""
        n = self.sizes()
        return int(self.n_points) ** 2 - int(np.sum(n * n))


@dataclasses.dataclass
class Batch:
    """Several independent suspensions concatenated (vesicle- and point-wise)."""
    X: np.ndarray
    f: np.ndarray
    w: np.ndarray
    vesicle_offsets: np.ndarray      # (V+1,) int32, global point offsets
    suspension_offsets: np.ndarray   # (S+1,) int32, vesicle index ranges
    mu: np.ndarray                   # (S,) float64
    members: list

    @property
    def n_points(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_suspensions(self) -> int:
        return int(self.suspension_offsets.shape[0] - 1)

    def cross_pairs(self) -> int:
        return int(sum(s.cross_pairs() for s in self.members))


# ----------------------------------------------------------------------------- shapes

def ellipse_axes(nu: float, perimeter: float = PERIMETER) -> tuple[float, float]:
    """Semi-axes (a >= b) of the ellipse with the given perimeter and reduced area.

    Reduced area is 4*pi*A/L^2; with A = pi*a*b and L = perimeter this gives
    a*b = nu*(L/(2*pi))^2.  The perimeter is 4*a*E(1 - b^2/a^2) with E the
    complete elliptic integral of the second kind (parameter convention).
    """
    s = perimeter / (2.0 * np.pi)
    ab = nu * s * s
    if nu >= 1.0:
        return s, s

    def g(a):
        return 4.0 * a * ellipe(1.0 - (ab / a) ** 2 / a ** 2) - perimeter

    lo = np.sqrt(ab) * (1.0 + 1e-12)
    a = brentq(g, lo, 4.0 * s, xtol=1e-15, rtol=1e-15, maxiter=200)
    return float(a), float(ab / a)


def ellipse_curve(center, a, b, phi, n):
    """Points and arclength weights of a rotated ellipse at alpha_k = 2*pi*k/n."""
    if n == 0:
        return np.zeros((2, 0)), np.zeros(0), np.zeros(0)
    th = 2.0 * np.pi * np.arange(n) / n
    c, s = np.cos(phi), np.sin(phi)
    ex, ey = a * np.cos(th), b * np.sin(th)
    x = center[0] + c * ex - s * ey
    y = center[1] + s * ex + c * ey
    speed = np.sqrt((a * np.sin(th)) ** 2 + (b * np.cos(th)) ** 2)
    return np.stack([x, y]), speed * (2.0 * np.pi / n), th


def fourier_force(rng, n, th, kmin, kmax, std_fn):
    """Smooth random force density: per component sum_k alpha_k cos(k th) + beta_k sin(k th)."""
    f = np.zeros((2, n))
    for comp in range(2):
        for k in range(kmin, kmax + 1):
            sd = std_fn(k)
            f[comp] += rng.normal(0.0, sd) * np.cos(k * th)
            if k > 0:
                f[comp] += rng.normal(0.0, sd) * np.sin(k * th)
    return f


def make_force_free(f, w):
    """Remove the arc-weighted mean so that sum_j w_j f_j = 0 (to rounding)."""
    return f - (f @ w)[:, None] / np.sum(w)


# ----------------------------------------------------------------------------- packing

def _extent(a, b, phi):
    c, s = np.cos(phi), np.sin(phi)
    return np.sqrt((a * c) ** 2 + (b * s) ** 2), np.sqrt((a * s) ** 2 + (b * c) ** 2)


_UNIT = {}


def _unit(n):
    if n not in _UNIT:
        th = 2.0 * np.pi * np.arange(n) / n
        _UNIT[n] = (np.cos(th), np.sin(th))
    return _UNIT[n]


def _sample(center, a, b, phi, n):
    """(x, y) of n boundary points of a rotated ellipse (same points as ellipse_curve)."""
    ct, st = _unit(n)
    c, s = np.cos(phi), np.sin(phi)
    ex, ey = a * ct, b * st
    return center[0] + c * ex - s * ey, center[1] + s * ex + c * ey


def _min_dist(p, q):
    dx = p[0][:, None] - q[0][None, :]
    dy = p[1][:, None] - q[1][None, :]
    return float(np.sqrt(np.min(dx * dx + dy * dy)))


def rsa_pack(rng, axes, box, gap, max_tries=10_000_000):
    """Random sequential addition of ellipses wholly inside [0, box]^2.

    Accepts a candidate only if its true boundary distance to every placed
    ellipse is >= gap.  Sampled point sets over-estimate the true distance by
    at most half the largest chord spacing of each curve (a * 2*pi/n), so a
    coarse 64-point test rejects certain overlaps and a 512-point test with
    that margin decides the rest.  Fails loudly instead of lowering the area
    fraction.
    """
    m = len(axes)
    amax = float(np.max(axes[:, 0]))
    cell = 2.0 * amax + gap
    ncell = max(1, int(box // cell))
    cell = box / ncell
    grid: dict = {}
    centers = np.zeros((m, 2))
    angles = np.zeros(m)
    coarse_n, fine_n = 64, 512
    coarse_pts, fine_pts = [None] * m, [None] * m
    tries = 0
    for v in range(m):
        a, b = axes[v]
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError(f"RSA failed to place vesicle {v}/{m} within {max_tries} tries")
            phi = rng.uniform(0.0, 2.0 * np.pi)
            hx, hy = _extent(a, b, phi)
            if 2 * hx >= box or 2 * hy >= box:
                raise RuntimeError("box too small for one vesicle")
            c = np.array([rng.uniform(hx, box - hx), rng.uniform(hy, box - hy)])
            ci, cj = int(c[0] // cell), int(c[1] // cell)
            nbrs = []
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    nbrs.extend(grid.get((ci + di, cj + dj), ()))
            ok = True
            close = []
            for u in nbrs:
                dc = float(np.hypot(centers[u, 0] - c[0], centers[u, 1] - c[1]))
                if dc >= a + axes[u, 0] + gap:
                    continue
                if dc < axes[u, 1] + b:  # inscribed circles overlap
                    ok = False
                    break
                close.append(u)
            if ok and close:
                cpts = _sample(c, a, b, phi, coarse_n)
                fpts = None
                for u in close:
                    if coarse_pts[u] is None:
                        coarse_pts[u] = _sample(centers[u], axes[u, 0], axes[u, 1], angles[u], coarse_n)
                    dco = _min_dist(cpts, coarse_pts[u])
                    if dco < gap:
                        ok = False
                        break
                    margin_c = 0.5 * (a + axes[u, 0]) * 2.0 * np.pi / coarse_n
                    if dco - margin_c >= gap:
                        continue
                    if fpts is None:
                        fpts = np.stack(_sample(c, a, b, phi, fine_n), axis=1)
                    if fine_pts[u] is None:
                        fine_pts[u] = cKDTree(np.stack(_sample(centers[u], axes[u, 0], axes[u, 1], angles[u],
                                                               fine_n), axis=1))
                    margin_f = 0.5 * (a + axes[u, 0]) * 2.0 * np.pi / fine_n
                    if float(fine_pts[u].query(fpts, k=1)[0].min()) - margin_f < gap:
                        ok = False
                        break
            if ok:
                centers[v] = c
                angles[v] = phi
                grid.setdefault((ci, cj), []).append(v)
                break
    return centers, angles


# ----------------------------------------------------------------------------- assembly

def _assemble(rng, centers, axes, angles, n_per, force_kind, net_force_std, mu, box):
    m = len(centers)
    n_per = np.broadcast_to(np.asarray(n_per, dtype=np.int64), (m,))
    offsets = np.zeros(m + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(n_per)
    P = int(offsets[-1])
    X = np.empty((2, P))
    f = np.empty((2, P))
    w = np.empty(P)
    for v in range(m):
        n = int(n_per[v])
        pts, wv, th = ellipse_curve(centers[v], axes[v, 0], axes[v, 1], angles[v], n)
        if force_kind == "k4":
            fv = fourier_force(rng, n, th, 0, 4, lambda k: 1.0)
        elif force_kind == "k16inv":
            fv = fourier_force(rng, n, th, 1, 16, lambda k: 1.0 / k)
        else:
            raise ValueError(force_kind)
        if n == 0:
            continue
        fv = make_force_free(fv, wv)
        if net_force_std > 0.0:
            Fnet = rng.normal(0.0, net_force_std, size=2)
            fv = fv + Fnet[:, None] / np.sum(wv)
        s, e = offsets[v], offsets[v + 1]
        X[:, s:e] = pts
        f[:, s:e] = fv
        w[s:e] = wv
    if P >= 2 ** 31:
        raise ValueError("suspension too large for int32 offsets")
    return Suspension(X=X, f=f, w=w, offsets=offsets.astype(np.int32), mu=float(mu), box=float(box),
                      centers=centers, axes=np.asarray(axes, dtype=np.float64), angles=angles)


def grid_suspension(seed, nx=4, ny=4, n=32, spacing=3.0, jitter=0.05, nu=0.65, mu=1.0):
    """Ellipses on a jittered nx-by-ny grid (spacing 3 > 2a + 0.1, so no overlap)."""
    rng = np.random.default_rng(seed)
    a, b = ellipse_axes(nu)
    m = nx * ny
    centers = np.array([[spacing * (i + 0.5), spacing * (j + 0.5)] for j in range(ny) for i in range(nx)], dtype=np.float64)
    centers += rng.uniform(-jitter, jitter, size=centers.shape)
    angles = rng.uniform(0.0, 2.0 * np.pi, size=m)
    axes = np.tile([a, b], (m, 1))
    return _assemble(rng, centers, axes, angles, n, "k4", 0.0, mu, spacing * max(nx, ny))


def rsa_suspension(seed, m, n, phi, nu=0.65, gap=0.1, force_kind="k4", net_force_std=0.0, mu=1.0):
    """m ellipses of perimeter 2*pi placed by RSA at area fraction phi (box side from phi)."""
    rng = np.random.default_rng(seed)
    if np.isscalar(nu):
        nus = np.full(m, float(nu))
    else:
        nus = rng.uniform(nu[0], nu[1], size=m)
    axes = np.array([ellipse_axes(float(x)) for x in nus]) if not np.isscalar(nu) else np.tile(ellipse_axes(float(nu)), (m, 1))
    area = float(np.sum(np.pi * axes[:, 0] * axes[:, 1]))
    box = float(np.sqrt(area / phi))
    centers, angles = rsa_pack(rng, axes, box, gap)
    return _assemble(rng, centers, axes, angles, n, force_kind, net_force_std, mu, box)


def smooth_field(seed, points, n_modes=8, length=4.0):
    """A seeded smooth random vector field at points (2, Q): a sum of n_modes plane waves
    a_m cos(k_m . x + p_m) with wavelengths between length and 2 length.  Stands in for the
    layer velocities that the paper's near-field networks predict."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    kmag = 2.0 * np.pi / (length * rng.uniform(1.0, 2.0, n_modes))
    k = kmag[:, None] * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    amp = rng.normal(size=(2, n_modes))
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    pts = np.asarray(points, dtype=np.float64)
    return amp @ np.cos(k @ pts + phase[:, None])


def batch_of(members, mus=None) -> Batch:
    X = np.concatenate([s.X for s in members], axis=1)
    f = np.concatenate([s.f for s in members], axis=1)
    w = np.concatenate([s.w for s in members])
    voff = [0]
    soff = [0]
    for s in members:
        base = voff[-1]
        voff.extend((base + s.offsets[1:].astype(np.int64)).tolist())
        soff.append(soff[-1] + s.n_vesicles)
    mu = np.array([s.mu for s in members], dtype=np.float64) if mus is None else np.asarray(mus, dtype=np.float64)
    return Batch(X=X, f=f, w=w, vesicle_offsets=np.asarray(voff, dtype=np.int32),
                 suspension_offsets=np.asarray(soff, dtype=np.int32), mu=mu, members=list(members))


# ----------------------------------------------------------------------------- the workloads

def config_seed(k: int, sub: int = 0) -> int:
    return BASE_SEED + 100 * k + sub


def make_config(k: int, variant: str = "force_free", n_suspensions: int = 64):
    """The five synthetic workloads.

    0: 16 x 32 on a jittered 4x4 grid (spacing 3), forces k <= 4, force-free.
    1: 2000 x 128 by RSA at 30% area fraction, gap 0.1, forces k <= 4.
    2: 8000 x 64 by RSA at 35%, reduced areas U[0.6, 0.9], 1/k^2 spectrum k <= 16;
       variant "force_free" or "net_force" (net force per vesicle N(0, 0.01)).
    3: 64 independent suspensions, M log-uniform in [10, 1500], N in {32, 64, 128},
       area fraction U[0.20, 0.35]; returns a Batch.
    4: 512 x 64 by RSA at 30%, forces k <= 4.
    """
    if k == 0:
        return grid_suspension(config_seed(0))
    if k == 1:
        return rsa_suspension(config_seed(1), 2000, 128, 0.30)
    if k == 2:
        net = 0.1 if variant == "net_force" else 0.0
        return rsa_suspension(config_seed(2, 1 if net else 0), 8000, 64, 0.35, nu=(0.6, 0.9),
                              force_kind="k16inv", net_force_std=net)
    if k == 3:
        rng = np.random.default_rng(config_seed(3))
        ms = np.rint(np.exp(rng.uniform(np.log(10.0), np.log(1500.0), size=n_suspensions))).astype(int)
        ns = rng.choice([32, 64, 128], size=n_suspensions)
        phis = rng.uniform(0.20, 0.35, size=n_suspensions)
        members = [rsa_suspension(config_seed(3, 1 + s), int(ms[s]), int(ns[s]), float(phis[s]))
                   for s in range(n_suspensions)]
        return batch_of(members)
    if k == 4:
        return rsa_suspension(config_seed(4), 512, 64, 0.30)
    raise ValueError(f"unknown workload {k}")


def target_field(k: int, P: int) -> np.ndarray:
    """Seeded random target velocity field u* (iid N(0,1) per component) for the adjoint loss."""
    rng = np.random.default_rng(config_seed(k, 99))
    return rng.normal(0.0, 1.0, size=(2, P))


def sample_targets(P: int, fraction: float, seed: int) -> np.ndarray:
    """Sorted seeded subset of target indices (e.g. the 1% parity sample)."""
    rng = np.random.default_rng(seed)
    count = max(1, int(round(P * fraction)))
    return np.sort(rng.choice(P, size=count, replace=False)).astype(np.int64)


def _cache_dir() -> str:
    d = os.environ.get("VESNET_SYNTH_CACHE", os.path.join(tempfile.gettempdir(), "vesnet_synth_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def load_config(k: int, variant: str = "force_free"):
    """make_config with an on-disk npz cache keyed by (workload, variant, generator version)."""
    if k == 3:
        key = f"cfg{k}_{variant}_v{GENERATOR_VERSION}"
    else:
        key = f"cfg{k}_{variant}_v{GENERATOR_VERSION}"
    tag = hashlib.sha1(key.encode()).hexdigest()[:10]
    path = os.path.join(_cache_dir(), f"{key}_{tag}.npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            if k == 3:
                members = []
                for s in range(int(z["n_members"])):
                    members.append(Suspension(X=z[f"X{s}"], f=z[f"f{s}"], w=z[f"w{s}"], offsets=z[f"o{s}"],
                                              mu=float(z[f"mu{s}"]), box=float(z[f"box{s}"]),
                                              centers=z[f"c{s}"], axes=z[f"a{s}"], angles=z[f"t{s}"]))
                return batch_of(members)
            return Suspension(X=z["X"], f=z["f"], w=z["w"], offsets=z["offsets"], mu=float(z["mu"]),
                              box=float(z["box"]), centers=z["centers"], axes=z["axes"], angles=z["angles"])
        except Exception:
            pass
    obj = make_config(k, variant)
    tmp = path + f".tmp{os.getpid()}.npz"
    if k == 3:
        arrs = {"n_members": np.int64(len(obj.members))}
        for s, m in enumerate(obj.members):
            arrs.update({f"X{s}": m.X, f"f{s}": m.f, f"w{s}": m.w, f"o{s}": m.offsets, f"mu{s}": m.mu,
                         f"box{s}": m.box, f"c{s}": m.centers, f"a{s}": m.axes, f"t{s}": m.angles})
        np.savez(tmp, **arrs)
    else:
        np.savez(tmp, X=obj.X, f=obj.f, w=obj.w, offsets=obj.offsets, mu=obj.mu, box=obj.box,
                 centers=obj.centers, axes=obj.axes, angles=obj.angles)
    os.replace(tmp, path)
    return obj
