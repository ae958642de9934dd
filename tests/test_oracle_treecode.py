"""Pins of the treecode oracle: the exact far-field sum (the plain C oracle) within the
truncation bound of the expansions, exactness without expansions or at high order, and
the expansion of a single box against its direct sum."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import treecode as TC
from synth import suspension as S


@pytest.fixture(scope="module")
def susp():
    return S.rsa_suspension(5, 120, 24, 0.3)


@pytest.fixture(scope="module")
def exact(susp):
    return O.farfield_suspension(susp.X, susp.f, susp.w, susp.offsets, susp.mu)


@pytest.mark.parametrize("depth", [0, 1])
def test_without_expansions_equals_direct_sum(susp, exact, depth):
    """Depth 0 and 1 have no interaction lists: every pair is direct, own vesicle skipped."""
    u = TC.treecode(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 8, depth)
    assert np.abs(u - exact).max() <= 1e-13 * np.abs(exact).max()


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_truncation_bound_and_convergence(susp, exact, depth):
    """The error against the exact sum stays within the derived bound of the dropped series
    terms (plus rounding), and falls with the order."""
    errs = []
    for p in (4, 8, 16):
        u = TC.treecode(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
        b = TC.truncation_bound(susp.X, susp.f, susp.w, susp.offsets, susp.mu, p, depth)
        err = np.abs(u - exact).max(axis=0)
        assert np.all(err <= b + 1e-13 * np.abs(exact).max()), (p, (err / b).max())
        errs.append(err.max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5 * np.abs(exact).max()


def test_high_order_reaches_rounding(susp, exact):
    u = TC.treecode(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 45, 3)
    assert np.abs(u - exact).max() <= 1e-13 * np.abs(exact).max()


def test_single_box_expansion_against_direct_terms():
    """The far terms of one box of sources, from its three moment sets, reproduce the direct
    Stokeslet sum of that box at a distant point to the size of the first dropped term."""
    rng = np.random.default_rng(7)
    c = 0.3 - 0.2j
    zs = c + (rng.uniform(-0.5, 0.5, 30) + 1j * rng.uniform(-0.5, 0.5, 30))
    F = rng.normal(size=30) + 1j * rng.normal(size=30)
    zt = np.array([4.0 + 1.0j, -3.0 - 2.5j, 0.1 + 5.0j])
    ref = np.array([TC.direct_terms(z, zs, F) for z in zt])
    box = np.zeros(30, int)
    centers = np.array([c])
    zeta = zs - c
    for p in (10, 30):
        M = [TC.box_moments(zs, q, centers, box, 1, p)[0] for q in (F, np.conj(F), np.conj(zeta) * F)]
        got = np.array([TC.far_terms(z - c, *M) for z in zt])
        x = np.abs(zeta).max() / np.abs(zt - c)
        # dropped terms, plus rounding of sums whose terms are bounded by sum |F| (1 + |ln|w||)
        rounding = 64 * np.finfo(float).eps * np.abs(F).sum() * (1 + np.abs(np.log(np.abs(zt - c))))
        assert np.all(np.abs(got - ref) <= np.abs(F).sum() * x ** (p + 1) * 3 / (1 - x) + rounding)


def test_tree_assignment():
    """Bounding square centred on the points' box, side the larger extent; the upper edge
    belongs to the last box."""
    X = np.array([[0.0, 4.0, 2.0, 4.0], [1.0, 1.0, 2.0, 3.0]])
    t = TC.build_tree(X, 2)
    assert t.side == 4.0 and t.x0 == 0.0 and t.y0 == 0.0
    np.testing.assert_array_equal(t.ix, [0, 3, 2, 3])
    np.testing.assert_array_equal(t.iy, [1, 1, 2, 3])


def test_translation_leaves_the_result(susp):
    """The tree follows the points, so a rigid shift changes only rounding."""
    u0 = TC.treecode(susp.X, susp.f, susp.w, susp.offsets, susp.mu, 12, 3)
    u1 = TC.treecode(susp.X + np.array([[1000.0], [-500.0]]), susp.f, susp.w, susp.offsets, susp.mu, 12, 3)
    assert np.abs(u1 - u0).max() <= 1e-9 * np.abs(u0).max()
