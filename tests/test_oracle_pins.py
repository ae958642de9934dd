"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each test targets a plausible mistake in the oracle (a dropped or sign-flipped
term, a missing identity, a wrong prefactor, weights taken at the wrong index,
a wrong exclusion) and is independent of the oracle's own code: closed forms
of the continuous integral eq. (single_layer) for a circle, the divergence-free
property of the Stokeslet (eq. (incomp)), the nullity of the single layer of
the normal, reciprocity, invariances, and exact scaling laws.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import suspension as S


def _lone_targets(x):
    """Targets that belong to no source vesicle (exclusion id -1)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return x, -np.ones(x.shape[1], dtype=np.int32)


def _circle(a, n, center=(0.0, 0.0)):
    th = 2.0 * np.pi * np.arange(n) / n
    y = np.stack([center[0] + a * np.cos(th), center[1] + a * np.sin(th)])
    return y, np.full(n, 2.0 * np.pi * a / n), th


# ----------------------------------------------------------------------------- single pairs

@pytest.mark.parametrize("r,f,expected", [
    ((1.0, 0.0), (1.0, 0.0), (1.0 / (4 * np.pi), 0.0)),                 # ln 1 = 0, rr-term = f
    ((2.0, 0.0), (0.0, 1.0), (0.0, -np.log(2.0) / (4 * np.pi))),       # r . f = 0: pure log term
    ((np.e, 0.0), (1.0, 0.0), (0.0, 0.0)),                              # -ln e f + f = 0 exactly
    ((0.0, 1.0), (1.0, 0.0), (0.0, 0.0)),                               # ln 1 = 0 and r . f = 0
])
def test_single_pair_closed_forms(r, f, expected):
    """One source, one target, w = 1, mu = 1: u = (1/4 pi)(-ln|r| f + (r.f) r/|r|^2)."""
    t, excl = _lone_targets(np.array(r)[:, None])
    u = O.farfield(t, np.zeros((2, 1)), np.array(f)[:, None], np.ones(1), 1.0, excl, np.zeros(1, np.int32))
    np.testing.assert_allclose(u[:, 0], expected, atol=1e-16)


def test_golden_single_pairs():
    """Hand-derived single-pair values stored under tests/golden (with derivations)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "single_pairs.txt")
    rows = np.loadtxt(path, comments="#")
    for rx, ry, fx, fy, mu, ux, uy in rows:
        t, excl = _lone_targets(np.array([[rx], [ry]]))
        u = O.farfield(t, np.zeros((2, 1)), np.array([[fx], [fy]]), np.ones(1), mu, excl, np.zeros(1, np.int32))
        np.testing.assert_allclose(u[:, 0], [ux, uy], rtol=0, atol=2e-15)


# ----------------------------------------------------------------------------- circle closed forms

@pytest.mark.parametrize("a,mu", [(0.8, 1.7), (1.3, 1.0), (2.0, 0.5)])
def test_circle_uniform_force_interior(a, mu):
    """Inside a circle of radius a the single layer of a uniform density f0 is
    (a/(4 mu))(1 - 2 ln a) f0: the log potential of the circle is 2 pi a ln a
    inside, and the rr-kernel integrates to pi a I (its e^{2i phi} part is a
    contour integral with no pole inside).  The trapezoid rule converges
    geometrically for targets off the curve."""
    y, w, _ = _circle(a, 96)
    f0 = np.array([0.3, -1.1])
    f = np.tile(f0[:, None], (1, y.shape[1]))
    pts = np.array([[0.0, 0.0], [0.3 * a, -0.2 * a], [-0.45 * a, 0.1 * a]]).T
    t, excl = _lone_targets(pts)
    u = O.farfield(t, y, f, w, mu, excl, np.zeros(y.shape[1], np.int32))
    expect = (a / (4 * mu)) * (1 - 2 * np.log(a)) * f0
    np.testing.assert_allclose(u, np.tile(expect[:, None], (1, pts.shape[1])), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("z", [complex(2.5, 1.0), complex(-1.7, -2.9), complex(0.2, 3.3)])
def test_circle_uniform_force_exterior(z):
    """Outside (|z| > a): log part -2 pi a ln|z| f0, rr part pi a f0 + (1/2) M(C) f0 with
    C = 2 pi a (z/conj(z) - a^2/conj(z)^2) (residue at a^2/conj(z)) and
    M(C) = [[Re C, Im C], [Im C, -Re C]]."""
    a, mu = 1.1, 1.3
    y, w, _ = _circle(a, 128)
    f0 = np.array([-0.7, 0.45])
    f = np.tile(f0[:, None], (1, y.shape[1]))
    t, excl = _lone_targets(np.array([[z.real], [z.imag]]))
    u = O.farfield(t, y, f, w, mu, excl, np.zeros(y.shape[1], np.int32))[:, 0]
    C = 2 * np.pi * a * (z / np.conj(z) - a * a / np.conj(z) ** 2)
    M = np.array([[C.real, C.imag], [C.imag, -C.real]])
    expect = (-2 * np.pi * a * np.log(abs(z)) * f0 + np.pi * a * f0 + 0.5 * M @ f0) / (4 * np.pi * mu)
    np.testing.assert_allclose(u, expect, rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------------------------- nullity of the normal

@pytest.mark.parametrize("where", ["outside", "inside"])
def test_single_layer_of_normal_vanishes(where):
    """Each column of the Stokeslet is divergence-free, so the single layer of the
    unit normal of a closed curve vanishes off the curve.  On an ellipse the
    weights |X'| 2 pi/N vary along the curve, so weights taken at the target
    instead of the source would break this."""
    a, b = S.ellipse_axes(0.65)
    n = 128
    X, w, th = S.ellipse_curve((0.3, -0.2), a, b, 0.7, n)
    # outward normal: rotate the tangent X'(theta) by -90 degrees and normalise
    c, s = np.cos(0.7), np.sin(0.7)
    tx, ty = -a * np.sin(th), b * np.cos(th)
    Tx, Ty = c * tx - s * ty, s * tx + c * ty
    nrm = np.hypot(Tx, Ty)
    nvec = np.stack([Ty / nrm, -Tx / nrm])
    if where == "outside":
        pts = np.array([[3.0, 0.5], [-2.5, 2.0], [0.0, -4.0]]).T
    else:
        pts = np.array([[0.3, -0.2], [0.5, -0.1], [0.1, -0.25]]).T
    t, excl = _lone_targets(pts)
    u = O.farfield(t, X, nvec, w, 1.0, excl, np.zeros(n, np.int32))
    assert np.max(np.abs(u)) < 1e-12
    # the uniform force on the same curve does not vanish (the test has teeth)
    u2 = O.farfield(t, X, np.tile([[1.0], [0.0]], (1, n)), w, 1.0, excl, np.zeros(n, np.int32))
    assert np.max(np.abs(u2)) > 1e-2


# ----------------------------------------------------------------------------- divergence

def test_divergence_free():
    """eq. (incomp): the induced field is divergence-free off the membranes."""
    s = S.make_config(0)
    vid = O.vesicle_ids(s.offsets)
    pts = np.array([[1.5, 1.5], [4.4, 7.6], [10.5, 3.0], [6.0, 6.0]]).T
    h = 1e-4
    div = []
    scale = []
    for k in range(pts.shape[1]):
        p = pts[:, k]
        stencil = np.array([p + [h, 0], p - [h, 0], p + [0, h], p - [0, h]]).T
        t, excl = _lone_targets(stencil)
        u = O.farfield(t, s.X, s.f, s.w, 1.0, excl, vid)
        dudx = (u[0, 0] - u[0, 1]) / (2 * h)
        dvdy = (u[1, 2] - u[1, 3]) / (2 * h)
        div.append(dudx + dvdy)
        scale.append(abs(dudx) + abs(dvdy))
    div = np.abs(np.array(div))
    assert np.all(div < 1e-6 * np.maximum(np.array(scale), 1e-3)), (div, scale)


# ----------------------------------------------------------------------------- reciprocity

def test_weighted_reciprocity():
    """G is symmetric and even and the exclusion is symmetric, so
    sum_i w_i g_i . u_i[f] = sum_j w_j f_j . u_j[g] for any two densities."""
    s = S.make_config(0)
    rng = np.random.default_rng(5)
    g = rng.normal(size=s.f.shape)
    uf = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    ug = O.farfield_suspension(s.X, g, s.w, s.offsets, 1.0)
    lhs = np.sum(s.w * np.sum(g * uf, axis=0))
    rhs = np.sum(s.w * np.sum(s.f * ug, axis=0))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1e-300) + 1e-14


# ----------------------------------------------------------------------------- invariances and scaling

def test_translation_and_rotation():
    s = S.make_config(0)
    u = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    ut = O.farfield_suspension(s.X + np.array([[1000.25], [-333.5]]), s.f, s.w, s.offsets, 1.0)
    np.testing.assert_allclose(ut, u, atol=1e-10 * np.abs(u).max())
    th = 0.9
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    ur = O.farfield_suspension(R @ s.X, R @ s.f, s.w, s.offsets, 1.0)
    np.testing.assert_allclose(ur, R @ u, atol=1e-14 * np.abs(u).max() * 10)


def test_scaling_force_free_and_net_force():
    """(X, w) -> (sX, sw): -ln|s r| = -ln s - ln|r|, so
    u_s = s u - (s ln s / (4 pi mu)) * sum over other vesicles of sum_j w_j f_j.
    For force-free vesicles the second term vanishes."""
    s = S.make_config(0)
    sc = 3.7
    mu = 1.0
    u = O.farfield_suspension(s.X, s.f, s.w, s.offsets, mu)
    us = O.farfield_suspension(sc * s.X, s.f, sc * s.w, s.offsets, mu)
    np.testing.assert_allclose(us, sc * u, atol=1e-13 * np.abs(u).max())
    # give every vesicle a net force
    rng = np.random.default_rng(11)
    f = s.f.copy()
    Fv = rng.normal(size=(2, s.n_vesicles))
    for v in range(s.n_vesicles):
        a, b = s.offsets[v], s.offsets[v + 1]
        f[:, a:b] += Fv[:, v:v + 1] / np.sum(s.w[a:b])
    u = O.farfield_suspension(s.X, f, s.w, s.offsets, mu)
    us = O.farfield_suspension(sc * s.X, f, sc * s.w, s.offsets, mu)
    total = Fv.sum(axis=1)
    vid = O.vesicle_ids(s.offsets)
    others = total[:, None] - Fv[:, vid]
    expect = sc * u - sc * np.log(sc) / (4 * np.pi * mu) * others
    np.testing.assert_allclose(us, expect, atol=1e-12 * np.abs(u).max())


def test_linearity_and_viscosity():
    s = S.make_config(0)
    rng = np.random.default_rng(3)
    g = rng.normal(size=s.f.shape)
    u1 = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    u2 = O.farfield_suspension(s.X, g, s.w, s.offsets, 1.0)
    u12 = O.farfield_suspension(s.X, 2.0 * s.f - 0.5 * g, s.w, s.offsets, 1.0)
    np.testing.assert_allclose(u12, 2.0 * u1 - 0.5 * u2, atol=1e-13 * np.abs(u12).max())
    u_mu = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 2.5)
    np.testing.assert_allclose(u_mu, u1 / 2.5, rtol=1e-14, atol=1e-16)


def test_far_field_is_one_stokeslet():
    """Seen from distance R, a vesicle acts as one Stokeslet of its net force at its
    centre: |u - G(x - c) F| = O(1/R), so R * error stays bounded and settles."""
    a, b = S.ellipse_axes(0.65)
    X, w, th = S.ellipse_curve((0.0, 0.0), a, b, 0.4, 64)
    f = np.stack([1.0 + 0.3 * np.cos(th), -0.5 + 0.2 * np.sin(2 * th)])
    F = f @ w
    errs = []
    for R in (1e2, 1e3, 1e4):
        x = np.array([[R * 0.6], [R * 0.8]])
        t, excl = _lone_targets(x)
        u = O.farfield(t, X, f, w, 1.0, excl, np.zeros(64, np.int32))[:, 0]
        r = x[:, 0]
        G = (-np.log(np.linalg.norm(r)) * np.eye(2) + np.outer(r, r) / (r @ r)) / (4 * np.pi)
        errs.append(R * np.linalg.norm(u - G @ F))
    assert errs[0] < 1.0
    assert abs(errs[1] - errs[2]) < 0.02 * errs[2] + 1e-9
    assert abs(errs[0] - errs[1]) < 0.1 * errs[1] + 1e-9


def test_trapezoid_refinement_converges():
    """For far targets the N-point sum on an analytic curve with analytic density
    converges geometrically to the integral: N and 4N agree to ~1e-13."""
    a, b = S.ellipse_axes(0.65)
    pts = np.array([[4.0, 1.0], [-3.0, 3.5]]).T
    t, excl = _lone_targets(pts)
    out = []
    for n in (64, 256):
        X, w, th = S.ellipse_curve((0.0, 0.0), a, b, 0.3, n)
        f = np.stack([np.cos(th) + 0.2 * np.sin(3 * th), np.sin(2 * th)])
        out.append(O.farfield(t, X, f, w, 1.0, excl, np.zeros(n, np.int32)))
    np.testing.assert_allclose(out[0], out[1], atol=1e-13)


# ----------------------------------------------------------------------------- exclusion

def test_own_vesicle_excluded():
    """u at a vesicle's points does not depend on that vesicle's own density, and
    equals the sum over the other vesicles evaluated with no exclusion."""
    s = S.make_config(0)
    u = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    v = 5
    a, b = s.offsets[v], s.offsets[v + 1]
    f2 = s.f.copy()
    f2[:, a:b] = 17.0
    u2 = O.farfield_suspension(s.X, f2, s.w, s.offsets, 1.0)
    np.testing.assert_array_equal(u2[:, a:b], u[:, a:b])
    keep = np.r_[0:a, b:s.n_points]
    t, excl = _lone_targets(s.X[:, a:b])
    u3 = O.farfield(t, s.X[:, keep], s.f[:, keep], s.w[keep], 1.0, excl, np.zeros(keep.size, np.int32))
    np.testing.assert_allclose(u3, u[:, a:b], rtol=0, atol=1e-15 * np.abs(u).max())


def test_coincident_points_rejected():
    X = np.array([[0.0, 0.0], [0.0, 0.0]])
    with pytest.raises(ValueError):
        O.farfield_suspension(X, np.ones((2, 2)), np.ones(2), np.array([0, 1, 2], np.int32), 1.0)


# ----------------------------------------------------------------------------- gradients

def _loss(X, f, w, offsets, mu, ustar):
    u = O.farfield_suspension(X, f, w, offsets, mu)
    return 0.5 * np.sum((u - ustar) ** 2), u


def _small_case():
    susp = S.rsa_suspension(12345, 6, 16, 0.2)
    rng = np.random.default_rng(1)
    ustar = rng.normal(size=(2, susp.n_points))
    return susp, ustar


def test_gradient_vs_central_differences():
    """Analytic oracle gradient (dL/dX over both roles, dL/df, dL/dw) against
    central differences of the oracle's own forward sum, h = 1e-6."""
    s, ustar = _small_case()
    mu = 1.3
    L0, u = _loss(s.X, s.f, s.w, s.offsets, mu, ustar)
    g = u - ustar
    gr = O.grad_suspension(s.X, s.f, s.w, s.offsets, mu, g)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(20):
        c, k = rng.integers(2), rng.integers(s.n_points)
        for name, arr, an in (("X", s.X, gr["grad_X"][c, k]), ("f", s.f, gr["grad_f"][c, k])):
            Xp, Xm = arr.copy(), arr.copy()
            Xp[c, k] += h
            Xm[c, k] -= h
            if name == "X":
                Lp, _ = _loss(Xp, s.f, s.w, s.offsets, mu, ustar)
                Lm, _ = _loss(Xm, s.f, s.w, s.offsets, mu, ustar)
            else:
                Lp, _ = _loss(s.X, Xp, s.w, s.offsets, mu, ustar)
                Lm, _ = _loss(s.X, Xm, s.w, s.offsets, mu, ustar)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (name, c, k, fd, an)
        wp, wm = s.w.copy(), s.w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (_loss(s.X, s.f, wp, s.offsets, mu, ustar)[0] - _loss(s.X, s.f, wm, s.offsets, mu, ustar)[0]) / (2 * h)
        assert abs(fd - gr["grad_w"][k]) <= 2e-6 * max(1.0, abs(gr["grad_w"][k]))


def _complex_loss(X, f, w, offsets, mu, ustar):
    """Complex-analytic rewrite of the loss for the complex-step derivative
    (no abs/conj; ln|r| = 0.5 ln(rx^2 + ry^2) is analytic)."""
    vid = O.vesicle_ids(offsets)
    rx = X[0][:, None] - X[0][None, :]
    ry = X[1][:, None] - X[1][None, :]
    mask = vid[:, None] != vid[None, :]
    r2 = np.where(mask, rx * rx + ry * ry, 1.0)
    lnr = 0.5 * np.log(r2)
    Fx, Fy = w * f[0], w * f[1]
    rdotF = rx * Fx[None, :] + ry * Fy[None, :]
    ux = np.sum(np.where(mask, -lnr * Fx[None, :] + rdotF * rx / r2, 0.0), axis=1) / (4 * np.pi * mu)
    uy = np.sum(np.where(mask, -lnr * Fy[None, :] + rdotF * ry / r2, 0.0), axis=1) / (4 * np.pi * mu)
    return 0.5 * np.sum((ux - ustar[0]) ** 2 + (uy - ustar[1]) ** 2), np.stack([ux, uy])


def test_gradient_vs_complex_step():
    """Complex step (h = 1e-30) pins the oracle gradient to ~1e-13.  The complex
    rewrite is first checked against the oracle at real inputs."""
    s, ustar = _small_case()
    mu = 0.8
    L0, u = _loss(s.X, s.f, s.w, s.offsets, mu, ustar)
    Lc, uc = _complex_loss(s.X, s.f, s.w, s.offsets, mu, ustar)
    np.testing.assert_allclose(uc, u, rtol=1e-12, atol=1e-14)
    gr = O.grad_suspension(s.X, s.f, s.w, s.offsets, mu, u - ustar)
    rng = np.random.default_rng(9)
    h = 1e-30
    for _ in range(25):
        c, k = rng.integers(2), rng.integers(s.n_points)
        Xc = s.X.astype(np.complex128)
        Xc[c, k] += 1j * h
        d = np.imag(_complex_loss(Xc, s.f, s.w, s.offsets, mu, ustar)[0]) / h
        assert abs(d - gr["grad_X"][c, k]) <= 1e-11 * max(1.0, abs(d))
        fc = s.f.astype(np.complex128)
        fc[c, k] += 1j * h
        d = np.imag(_complex_loss(s.X, fc, s.w, s.offsets, mu, ustar)[0]) / h
        assert abs(d - gr["grad_f"][c, k]) <= 1e-11 * max(1.0, abs(d))
        wc = s.w.astype(np.complex128)
        wc[k] += 1j * h
        d = np.imag(_complex_loss(s.X, s.f, wc, s.offsets, mu, ustar)[0]) / h
        assert abs(d - gr["grad_w"][k]) <= 1e-11 * max(1.0, abs(d))


def test_adjoint_of_f_is_forward_on_g():
    """By reciprocity, dL/df_j = w_j (G g)_j: the forward operator applied to g."""
    s, ustar = _small_case()
    rng = np.random.default_rng(4)
    g = rng.normal(size=s.f.shape)
    gr = O.grad_suspension(s.X, s.f, s.w, s.offsets, 1.0, g)
    ug = O.farfield_suspension(s.X, g, np.ones_like(s.w), s.offsets, 1.0)
    np.testing.assert_allclose(gr["v"], ug, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gr["grad_f"], s.w * ug, rtol=1e-13, atol=1e-15)
