"""Pins of the near-field layer and RBF interpolation oracle (Section 3.3,
Algorithm 4 CreateNearLayers / interpolateInNearField) against closed forms,
exact geometry and an independent library interpolator."""
import numpy as np
import pytest
from scipy.interpolate import RBFInterpolator

from oracle import nearfield_rbf as NR
from synth import suspension as S

EPS = np.finfo(float).eps
# the node layout read from Section 3.3: layer l of a vesicle sits at d = (l - 2) h / 2
ORDER = (-1.0, -0.5, 0.0, 0.5, 1.0)


def _circle(n, R, c, clockwise=False):
    a = 2 * np.pi * np.arange(n) / n
    if clockwise:
        a = -a
    X = np.array(c, dtype=float)[:, None] + R * np.stack([np.cos(a), np.sin(a)])
    w = np.full(n, 2 * np.pi * R / n)
    return X, w


def _ellipse(n, nu=0.65, rot=0.4, shift=(3.0, -1.0)):
    a, b = S.ellipse_axes(nu)
    t = 2 * np.pi * np.arange(n) / n
    c, s = np.cos(rot), np.sin(rot)
    R = np.array([[c, -s], [s, c]])
    X = R @ np.stack([a * np.cos(t), b * np.sin(t)]) + np.array(shift)[:, None]
    w = np.hypot(a * np.sin(t), b * np.cos(t)) * 2 * np.pi / n
    tang = R @ np.stack([-a * np.sin(t), b * np.cos(t)])
    tang /= np.hypot(*tang)
    outward = np.stack([tang[1], -tang[0]])
    return X, w, outward


@pytest.mark.parametrize("clockwise", [False, True])
@pytest.mark.parametrize("n", [7, 32, 33])
def test_circle_layers_are_concentric(n, clockwise):
    """On a circle of radius R the layer d lies on the circle of radius R + d h, each node on the
    ray from the centre through its membrane point, h = 2 pi R / N, for either orientation."""
    R, c = 1.3, (0.5, -2.0)
    X, w = _circle(n, R, c, clockwise)
    nodes, h = NR.vesicle_layers(X, w)
    assert h == pytest.approx(2 * np.pi * R / n, rel=1e-15)
    assert nodes.shape == (2, 5 * n)
    rel = X - np.array(c)[:, None]
    for l, d in enumerate(ORDER):
        blk = nodes[:, l * n:(l + 1) * n] - np.array(c)[:, None]
        np.testing.assert_allclose(blk, rel * (R + d * h) / R, atol=1e-13)
    # the middle layer is the membrane itself
    np.testing.assert_allclose(nodes[:, 2 * n:3 * n], X, atol=1e-15)


def test_ellipse_layers_follow_the_exact_normal():
    """Spectral tangent of a smooth curve: layers sit along the analytic outward normal."""
    n = 64
    X, w, outward = _ellipse(n)
    nodes, h = NR.vesicle_layers(X, w)
    assert h == pytest.approx(w.mean(), rel=1e-15)
    for l, d in enumerate(ORDER):
        np.testing.assert_allclose(nodes[:, l * n:(l + 1) * n], X + d * h * outward, atol=1e-10)


def test_near_layers_layout_and_empty_vesicles():
    X1, w1, _ = _ellipse(16)
    X2, w2 = _circle(9, 0.8, (10.0, 0.0), clockwise=True)
    X = np.concatenate([X1, X2], axis=1)
    w = np.concatenate([w1, w2])
    offsets = np.array([0, 16, 16, 25])
    layers, h = NR.near_layers(X, w, offsets)
    np.testing.assert_array_equal(layers[:, :80], NR.vesicle_layers(X1, w1)[0])
    np.testing.assert_array_equal(layers[:, 80:], NR.vesicle_layers(X2, w2)[0])
    assert h[1] == 0.0 and h[2] == pytest.approx(2 * np.pi * 0.8 / 9)


def test_two_node_closed_form():
    """Two nodes at distance r: K = [[1, g], [g, 1]], g = exp(-r^2 / width^2), so
    c = (u1 - g u2, u2 - g u1) / (1 - g^2), and s at the midpoint is g^(1/4) (c1 + c2)."""
    nodes = np.array([[0.0, 0.6], [0.0, 0.0]])
    u = np.array([[1.0, -2.0], [0.5, 3.0]])
    width = 0.7
    g = np.exp(-0.36 / width ** 2)
    c = NR.vesicle_fit(nodes, u, width)
    expect = np.stack([u[:, 0] - g * u[:, 1], u[:, 1] - g * u[:, 0]], axis=1) / (1 - g * g)
    np.testing.assert_allclose(c, expect, rtol=1e-14)
    mid = NR.vesicle_eval(nodes, c, np.array([[0.3], [0.0]]), width)
    np.testing.assert_allclose(mid[:, 0], np.exp(-0.09 / width ** 2) * (expect[:, 0] + expect[:, 1]), rtol=1e-14)


@pytest.mark.parametrize("eps", [0.75, 1.0])
def test_fit_matches_library_interpolator(eps):
    """scipy's RBFInterpolator with the Gaussian kernel exp(-(r/width)^2) and no polynomial part
    solves the same interpolation problem by its own route; values at near-zone points agree to
    the conditioning of K (derived bound 10 eps_mach cond(K))."""
    rng = np.random.default_rng(11)
    n = 32
    X, w, outward = _ellipse(n)
    nodes, h = NR.vesicle_layers(X, w)
    U = rng.normal(size=(2, 5 * n))
    width = eps * h
    c = NR.vesicle_fit(nodes, U, width)
    Q = X[:, :8] + rng.uniform(-1, 1, (2, 8)) * h
    s = NR.vesicle_eval(nodes, c, Q, width)
    ref = RBFInterpolator(nodes.T, U.T, kernel="gaussian", epsilon=1 / width, degree=-1)(Q.T).T
    kappa = np.linalg.cond(NR.kernel_matrix(nodes, width))
    assert np.abs(s - ref).max() <= 10 * EPS * kappa * np.abs(U).max()


def test_interpolates_the_nodes():
    rng = np.random.default_rng(12)
    X, w, _ = _ellipse(24)
    nodes, h = NR.vesicle_layers(X, w)
    U = rng.normal(size=(2, 120))
    c = NR.vesicle_fit(nodes, U, 0.75 * h)
    kappa = np.linalg.cond(NR.kernel_matrix(nodes, 0.75 * h))
    np.testing.assert_allclose(NR.vesicle_eval(nodes, c, nodes, 0.75 * h), U, atol=10 * EPS * kappa)


def test_smooth_field_converges_under_refinement():
    """Gaussian interpolation converges exponentially under refinement at a fixed shape (Section
    3.3): a smooth field (a Stokeslet centred well away from the vesicle) sampled on the five
    layers of ever finer discretisations, with the width held at 0.75 h of the coarsest one,
    is reproduced in the near zone with an error that falls by orders of magnitude."""
    src, F = np.array([4.0, 3.0]), np.array([0.7, -0.4])

    def field(x):
        r = x - src[:, None]
        q = (r ** 2).sum(0)
        return (-0.5 * np.log(q) * F[:, None] + (r * F[:, None]).sum(0) / q * r) / (4 * np.pi)

    a, b = S.ellipse_axes(0.65)
    rng = np.random.default_rng(5)
    tq = rng.uniform(0, 2 * np.pi, 300)
    tang = np.stack([-a * np.sin(tq), b * np.cos(tq)])
    tang /= np.hypot(*tang)
    errs = []
    width = None
    for n in (16, 24, 32, 40):
        X, w, _ = _ellipse(n, shift=(0.0, 0.0), rot=0.0)
        nodes, h = NR.vesicle_layers(X, w)
        if width is None:
            width = 0.75 * h
            # queries inside the thinnest band (|d| <= h of the finest vesicle)
            Q = np.stack([a * np.cos(tq), b * np.sin(tq)]) + rng.uniform(-0.39, 0.39, 300) * h * np.stack(
                [tang[1], -tang[0]])
            u = field(Q)
        c = NR.vesicle_fit(nodes, field(nodes), width)
        errs.append(np.abs(NR.vesicle_eval(nodes, c, Q, width) - u).max() / np.abs(u).max())
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert errs[-1] < errs[0] / 100, errs


def test_eval_near_sums_over_pairs():
    rng = np.random.default_rng(13)
    X1, w1, _ = _ellipse(12, shift=(0.0, 0.0))
    X2, w2, _ = _ellipse(12, shift=(0.0, 1.2))
    X = np.concatenate([X1, X2], axis=1)
    w = np.concatenate([w1, w2])
    offsets = np.array([0, 12, 24])
    layers, h = NR.near_layers(X, w, offsets)
    U = rng.normal(size=(2, 120))
    coeffs = NR.rbf_fit(layers, U, w, offsets, 1.0)
    T = rng.normal(size=(2, 3)) * 0.3
    both = NR.rbf_eval_near(layers, coeffs, w, offsets, 1.0, T, [(0, 0), (0, 1), (2, 1)])
    s0 = NR.vesicle_eval(layers[:, :60], coeffs[:, :60], T, h[0])
    s1 = NR.vesicle_eval(layers[:, 60:], coeffs[:, 60:], T, h[1])
    # the sums over 60 nodes are formed in different orders: bound 60 eps_mach sum_a |phi_a c_a|
    def bound(nodes, c, x, hv):
        d = x[:, :, None] - nodes[:, None, :]
        return 60 * EPS * (np.abs(c) @ NR.gaussian(d[0] ** 2 + d[1] ** 2, 1.0 * hv).T)

    np.testing.assert_array_less(np.abs(both[:, 0] - s0[:, 0] - s1[:, 0]),
                                 bound(layers[:, :60], coeffs[:, :60], T, h[0])[:, 0] + bound(layers[:, 60:], coeffs[:, 60:], T, h[1])[:, 0])
    np.testing.assert_array_equal(both[:, 1], 0.0)
    np.testing.assert_array_less(np.abs(both[:, 2] - s1[:, 2]), bound(layers[:, 60:], coeffs[:, 60:], T, h[1])[:, 2])
    np.testing.assert_array_equal(NR.rbf_eval_near(layers, coeffs, w, offsets, 1.0, T, np.zeros((0, 2), int)), 0.0)
