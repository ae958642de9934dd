"""Pins of the fast-multipole oracle: its Taylor coefficients against contour integrals of the
expanded functions (a route that shares no formula with them), the exact far-field sum (the plain C
oracle) within the derived truncation bound and at high order, exactness without expansions, the
treecode within both bounds, and a single far box against its direct sum."""
import numpy as np
import pytest

from oracle import fmm as FM
from oracle import oracle as O
from oracle import treecode as TC
from synth import suspension as S


@pytest.fixture(scope="module")
def susp():
    return S.rsa_suspension(5, 120, 24, 0.3)


@pytest.fixture(scope="module")
def exact(susp):
    return O.farfield_suspension(susp.X, susp.f, susp.w, susp.offsets, susp.mu)


def test_taylor_coefficients_against_contour_integral():
    """c_l = (1 / 2 pi i) closed integral of g(z) / (z - c_T)^(l+1) dz on a circle of radius |D|/2 about
    c_T, by the trapezoidal rule with 128 nodes (aliasing below 2^-100 of the scale), with
    g = lam log(z - c) + sum_m alpha_m (z - c)^-m evaluated pointwise; log(z - c) is taken as
    log D + log(1 + zeta / D) (principal logs, Re(1 + zeta / D) > 0 on the disc), the branch the
    coefficients use.  Arguments of D on all four quadrants and on the negative real axis."""
    rng = np.random.default_rng(3)
    p, mmax, K = 14, 15, 128
    D = np.array([2.0 + 0.5j, -1.5 + 2.0j, -3.0 - 0.2j, 0.4 - 2.5j, -2.0 + 0.0j])
    lam = rng.normal(size=D.size) + 1j * rng.normal(size=D.size)
    alpha = (rng.normal(size=(D.size, mmax)) + 1j * rng.normal(size=(D.size, mmax))) * 0.7 ** np.arange(mmax)
    got = FM.taylor_coeffs(lam, alpha, D, p)
    theta = 2 * np.pi * np.arange(K) / K
    for i, d in enumerate(D):
        r = abs(d) / 2
        zeta = r * np.exp(1j * theta)
        g = lam[i] * (np.log(d) + np.log(1 + zeta / d))
        g = g + sum(alpha[i, m - 1] * (zeta + d) ** (-m) for m in range(1, mmax + 1))
        scale = np.abs(g).max()
        for l in range(p + 1):
            c = np.mean(g * zeta ** (-l))
            assert abs(got[i, l] - c) <= 1e-12 * scale / r ** l, (i, l, got[i, l], c)


def test_single_far_box_against_direct_terms():
    """One box of sources and targets in a box two widths away: at order 40 the Taylor polynomials of
    the four functions reproduce the direct Stokeslet sum to rounding; at order 6 within the bound."""
    rng = np.random.default_rng(7)
    wd = 1.0
    c = 0.3 - 0.2j
    zs = c + wd * (rng.uniform(-0.5, 0.5, 30) + 1j * rng.uniform(-0.5, 0.5, 30))
    F = rng.normal(size=30) + 1j * rng.normal(size=30)
    cT = c + wd * (2.0 + 1.0j)
    zt = cT + wd * (rng.uniform(-0.5, 0.5, 20) + 1j * rng.uniform(-0.5, 0.5, 20))
    ref = np.array([TC.direct_terms(z, zs, F) for z in zt])
    box = np.zeros(30, int)
    centers = np.array([c])
    for p, tol in ((40, 1e-13), (6, None)):
        MF = TC.box_moments(zs, F, centers, box, 1, p)
        MFc = TC.box_moments(zs, np.conj(F), centers, box, 1, p)
        MG = TC.box_moments(zs, np.conj(zs) * F, centers, box, 1, p)
        coef = FM.multipole_coeffs(MF, MFc, MG, p)
        loc = {k: FM.taylor_coeffs(lam, al, np.array([cT - c]), p)[0] for k, (lam, al) in coef.items()}
        zeta = zt - cT
        got = (-0.5 * FM.polyval(loc["A"], zeta) - 0.5 * np.conj(FM.polyval(loc["Q"], zeta))
               + 0.5 * zt * np.conj(FM.polyval(loc["Phi"], zeta)) - 0.5 * np.conj(FM.polyval(loc["G"], zeta))
               + 0.5 * MF[0, 0])
        err = np.abs(got - ref).max()
        if tol is not None:
            assert err <= tol * np.abs(ref).max(), err
        else:
            assert 1e-14 * np.abs(ref).max() < err < 0.05 * np.abs(ref).max()  # truncated, not wrong


@pytest.mark.parametrize("depth", [0, 1])
def test_without_expansions_equals_direct_sum(susp, exact, depth):
    u = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 8, depth)
    assert np.abs(u - exact).max() <= 1e-13 * np.abs(exact).max()


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_truncation_bound_and_convergence(susp, exact, depth):
    """The error against the exact sum stays within the derived bound (plus rounding) and falls
    with the order."""
    errs = []
    for p in (4, 8, 16):
        u = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
        b = FM.truncation_bound(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
        err = np.abs(u - exact).max(axis=0)
        assert np.all(err <= b + 1e-13 * np.abs(exact).max()), (p, (err / b).max())
        errs.append(err.max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4 * np.abs(exact).max()


def test_high_order_reaches_rounding(susp, exact):
    u = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 45, 3)
    assert np.abs(u - exact).max() <= 1e-12 * np.abs(exact).max()


def test_agrees_with_treecode_within_both_bounds(susp):
    p, depth = 10, 4
    a = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
    b = TC.treecode(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
    bound = (FM.truncation_bound(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
             + TC.truncation_bound(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth))
    diff = np.abs(a - b).max(axis=0)
    assert np.all(diff <= bound + 1e-13 * np.abs(b).max())
    assert diff.max() > 0.0  # two different approximations


def test_selected_targets_match_full_evaluation(susp):
    sel = np.array([0, 5, 17, 400, 1999, susp.n_points - 1])
    full = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 12, 4)
    part = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 12, 4, sel=sel)
    assert np.array_equal(part, full[:, sel])
