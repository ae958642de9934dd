"""Pins of the membrane-force oracle (eq. (elastic_force), spectral arclength
derivatives of Section 2.2.1) against closed forms and exact invariants."""
import numpy as np
import pytest

from oracle import spectral as SP
from synth import suspension as S


@pytest.mark.parametrize("n", [8, 9, 32, 33])
def test_derivative_of_trig_polynomials(n):
    """d/dalpha of cos(k a) and sin(k a) is exact for |k| < N/2; the even-N Nyquist mode maps to zero."""
    a = 2 * np.pi * np.arange(n) / n
    for k in range(0, (n - 1) // 2 + 1):
        np.testing.assert_allclose(SP.spectral_derivative(np.cos(k * a)), -k * np.sin(k * a), atol=1e-12 * max(1, k))
        np.testing.assert_allclose(SP.spectral_derivative(np.sin(k * a)), k * np.cos(k * a), atol=1e-12 * max(1, k))
    if n % 2 == 0:
        np.testing.assert_allclose(SP.spectral_derivative(np.cos(n // 2 * a)), 0.0, atol=1e-12)


@pytest.mark.parametrize("n", [16, 31, 64])
def test_circle_closed_form(n):
    """Circle of radius R: X_s = t, X_ss = -(X - c)/R^2, X_ssss = (X - c)/R^4, so with constant
    sigma the force is (-kappa_b/R^4 - sigma/R^2)(X - c); w = 2 pi R / N."""
    R, kb, sig, c = 1.7, 0.8, 0.35, np.array([[0.4], [-2.0]])
    a = 2 * np.pi * np.arange(n) / n
    X = c + R * np.stack([np.cos(a), np.sin(a)])
    f, w = SP.vesicle_force(X, np.full(n, sig), kb)
    # rounding of X (eps |X|) is amplified by at most (N/2) per spectral derivative
    tol = 4 * np.finfo(float).eps * np.abs(X).max() * (n / 2) ** 4
    np.testing.assert_allclose(f, (-kb / R ** 4 - sig / R ** 2) * (X - c), atol=tol)
    np.testing.assert_allclose(w, 2 * np.pi * R / n, rtol=1e-13)


def _ellipse_curvature(theta, a, b):
    return a * b / ((a * np.sin(theta)) ** 2 + (b * np.cos(theta)) ** 2) ** 1.5


def test_ellipse_bending_force_frenet():
    """On an ellipse X = (a cos t, b sin t): X_ssss = (k_ss - k^3) n - 3 k k_s T (Frenet, with
    T the unit tangent and n the inward unit normal), with the curvature k(t) in closed form and
    its arclength derivatives by the complex step applied to that closed form."""
    a, b = S.ellipse_axes(0.65)
    n = 256
    t = 2 * np.pi * np.arange(n) / n
    X = np.stack([a * np.cos(t), b * np.sin(t)])
    f, w = SP.vesicle_force(X, np.zeros(n), 1.0)
    J = np.sqrt((a * np.sin(t)) ** 2 + (b * np.cos(t)) ** 2)
    h = 1e-20
    k = _ellipse_curvature(t, a, b)
    kt = np.imag(_ellipse_curvature(t + 1j * h, a, b)) / h

    def ks_of(tt):
        # k_s = k_t / J as an analytic function of t (for the second complex step)
        Jc = np.sqrt((a * np.sin(tt)) ** 2 + (b * np.cos(tt)) ** 2)
        dk = -1.5 * a * b * (2 * a * a * np.sin(tt) * np.cos(tt) - 2 * b * b * np.cos(tt) * np.sin(tt)) / Jc ** 5
        return dk / Jc

    ks = kt / J
    np.testing.assert_allclose(ks, ks_of(t), rtol=1e-12, atol=1e-12)
    kss = np.imag(ks_of(t + 1j * h)) / h / J
    T = np.stack([-a * np.sin(t), b * np.cos(t)]) / J
    nrm = np.stack([-T[1], T[0]])  # tangent rotated by +90 degrees: inward for a counter-clockwise curve
    xssss = (kss - k ** 3) * nrm - 3 * k * ks * T
    np.testing.assert_allclose(f, -xssss, atol=1e-8 * np.abs(xssss).max())
    np.testing.assert_allclose(w.sum(), 2 * np.pi, rtol=1e-12)  # perimeter 2 pi


def test_bending_force_is_force_free_and_torque_free():
    """-kappa_b X_ssss integrates to zero (exactly on the grid: the spectral derivative has no mean
    mode) and has zero torque (to spectral accuracy) on any smooth closed curve."""
    rng = np.random.default_rng(3)
    n = 64
    t = 2 * np.pi * np.arange(n) / n
    r = 1.0 + 0.15 * np.cos(2 * t) + 0.07 * np.sin(3 * t) + 0.03 * np.cos(5 * t)
    X = np.stack([r * np.cos(t), r * np.sin(t)]) + rng.normal(size=(2, 1))
    f, w = SP.vesicle_force(X, np.zeros(n), 2.0)
    F = (f * w).sum(axis=1)
    assert np.abs(F).max() < 1e-10 * np.abs(f * w).sum()
    torque = np.sum(w * (X[0] * f[1] - X[1] * f[0]))
    assert abs(torque) < 1e-6 * np.sum(w * np.hypot(*X) * np.hypot(*f))


def test_constant_tension_on_circle_gives_laplace_pressure():
    """(sigma X_s)_s with constant sigma is sigma * curvature * inward normal."""
    n = 40
    a = 2 * np.pi * np.arange(n) / n
    R = 0.9
    X = R * np.stack([np.cos(a), np.sin(a)])
    f, _ = SP.vesicle_force(X, np.full(n, 2.0), 0.0)
    np.testing.assert_allclose(f, -2.0 / R ** 2 * X, atol=1e-12)
