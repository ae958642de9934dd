"""Pins of the oracle's near-field masked far field (masks of Section 4.1,
FindNearFieldPoints of Algorithm 4, near-field rule of Section 2.2)."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import suspension as S


def _two_circles(gap_over_h, n=32, a=1.0):
    """Two circles whose facing points (theta = 0 on the left circle, theta = pi on
    the right) are gap_over_h * h apart, h = 2 pi a / n the spacing of each."""
    h = 2 * np.pi * a / n
    D = 2 * a + gap_over_h * h
    th = 2 * np.pi * np.arange(n) / n
    left = np.stack([a * np.cos(th), a * np.sin(th)])
    right = np.stack([D + a * np.cos(th), a * np.sin(th)])
    X = np.concatenate([left, right], axis=1)
    w = np.full(2 * n, 2 * np.pi * a / n)
    f = np.concatenate([np.stack([np.cos(th), 0.3 * np.sin(2 * th)])] * 2, axis=1)
    return X, f, w, np.array([0, n, 2 * n], np.int32), n


@pytest.mark.parametrize("ratio", [0.999, 0.5])
def test_near_pair_is_masked(ratio):
    """The facing points sit closer than h: each circle is near the facing point of
    the other, so that point's masked velocity is zero (only two vesicles)."""
    X, f, w, off, n = _two_circles(ratio)
    u, pairs = O.nearmasked_suspension(X, f, w, off, 1.0)
    assert np.all(u[:, 0] == 0.0) and np.all(u[:, n + n // 2] == 0.0)
    got = {tuple(p) for p in pairs.tolist()}
    assert (0, 1) in got and (n + n // 2, 0) in got
    # a point on the far side of the left circle is farther than h from the right circle
    assert (n // 2, 1) not in got


def test_far_pair_is_kept():
    """Facing points just beyond h: nothing is near and the masked sum equals the
    plain far field."""
    X, f, w, off, n = _two_circles(1.001)
    u, pairs = O.nearmasked_suspension(X, f, w, off, 1.0)
    assert pairs.shape[0] == 0
    np.testing.assert_array_equal(u, O.farfield_suspension(X, f, w, off, 1.0))


def test_masked_sum_decomposes():
    """Masked sum = plain far field minus, for every near pair, that vesicle's own
    trapezoid sum at the target (computed with the plain oracle on one vesicle)."""
    s = S.rsa_suspension(31, 40, 32, 0.40, gap=0.02)
    u, pairs = O.nearmasked_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    assert pairs.shape[0] > 10
    full = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    expect = full.copy()
    for i, v in pairs:
        a, b = s.offsets[v], s.offsets[v + 1]
        t = s.X[:, i:i + 1]
        ui = O.farfield(t, s.X[:, a:b], s.f[:, a:b], s.w[a:b], s.mu, np.array([-1], np.int32),
                        np.zeros(b - a, np.int32))
        expect[:, i] -= ui[:, 0]
    np.testing.assert_allclose(u, expect, rtol=0, atol=1e-13 * np.abs(full).max())


def test_near_decision_matches_brute_force_distance():
    """Near pairs equal the brute-force set {(i, v): min_j |x_i - y_j| <= mean spacing of v}."""
    s = S.rsa_suspension(32, 25, 32, 0.40, gap=0.02)
    _, pairs = O.nearmasked_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    vid = O.vesicle_ids(s.offsets)
    expect = set()
    for v in range(s.n_vesicles):
        a, b = s.offsets[v], s.offsets[v + 1]
        h = s.w[a:b].sum() / (b - a)
        d = np.sqrt(((s.X[:, :, None] - s.X[:, None, a:b]) ** 2).sum(axis=0)).min(axis=1)
        for i in np.nonzero((d <= h) & (vid != v))[0]:
            expect.add((int(i), v))
    assert {tuple(p) for p in pairs.tolist()} == expect
