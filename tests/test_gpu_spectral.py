"""GPU parity of the membrane force and trapezoid weights (eq. (elastic_force),
spectral derivatives of Section 2.2.1), and of the full step force -> far field."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import spectral as SP
from synth import suspension as S
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


def _curves(sizes, seed):
    """Smooth random closed curves (perturbed ellipses) of the given point counts, far apart."""
    rng = np.random.default_rng(seed)
    X, off = [], [0]
    for k, n in enumerate(sizes):
        t = 2 * np.pi * np.arange(n) / n
        a, b = rng.uniform(0.8, 1.4), rng.uniform(0.4, 0.8)
        r = 1.0 + 0.05 * np.cos(3 * t + rng.uniform(0, 6)) + 0.03 * np.sin(5 * t)
        x = np.stack([a * r * np.cos(t), b * r * np.sin(t)])
        phi = rng.uniform(0, 2 * np.pi)
        R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
        X.append(R @ x + np.array([[5.0 * k], [3.0 * (k % 2)]]))
        off.append(off[-1] + n)
    return np.concatenate(X, axis=1), np.asarray(off, np.int32)


def _exact_shift(X, off, shift):
    """Points that are exactly representable both as given and translated by shift: each coordinate
    is rounded to the grid of x + shift first, so the translated curve is the same curve."""
    Xr = (X + shift) - shift
    return Xr, Xr + shift


def _centred_reference(X, sigma, kappa_b, off):
    """The oracle on every curve moved to its own first point (f and w do not depend on the
    translation), so the reference's rounding scales with the curve's extent only."""
    f = np.empty_like(X)
    w = np.empty(X.shape[1])
    for v in range(len(off) - 1):
        a, b = off[v], off[v + 1]
        if b > a:
            fv, wv = SP.elastic_force(X[:, a:b] - X[:, a:a + 1], sigma[a:b], kappa_b, np.array([0, b - a]))
            f[:, a:b], w[a:b] = fv, wv
    return f, w


def _check_force(V, X, off, sizes, sigma, kappa_b, label):
    """GPU force and weights against the centred oracle.  Bars: the rounding of the points relative to
    the first point (size e = extent of the curve) amplified by at most N/2 per derivative, four of
    them, for f; and e N log2 N 2 pi / N for |X_alpha| 2 pi / N: neither grows with the translation."""
    import torch
    ref_f, ref_w = _centred_reference(X, sigma, kappa_b, off)
    f, w = V.elastic_force(torch.tensor(X, device="cuda"), off, kappa_b, torch.tensor(sigma, device="cuda"))
    torch.cuda.synchronize()
    f, w = f.cpu().numpy(), w.cpu().numpy()
    for v, n in enumerate(sizes):
        a, b = off[v], off[v + 1]
        if n < 3:
            continue
        ext = np.abs(X[:, a:b] - X[:, a:a + 1]).max()
        tol = 64 * EPS * ext * (n / 2) ** 4 + 64 * EPS * np.abs(ref_f[:, a:b]).max()
        df = np.abs(f[:, a:b] - ref_f[:, a:b]).max()
        say(f"{label} N={n}: max |df| {df:.3e} (bound {tol:.3e}), rel {df / np.abs(ref_f[:, a:b]).max():.3e}")
        assert df <= tol
        atol_w = 16 * EPS * ext * n * max(1.0, np.log2(n)) * (2 * np.pi / n)
        np.testing.assert_allclose(w[a:b], ref_w[a:b], rtol=0, atol=atol_w)


@pytest.mark.parametrize("shift", [0.0, 1000.0])
def test_elastic_force_parity_across_sizes(shift):
    """N = 4 .. 1024 (one wavefront per vesicle and the workgroup kernel), in place and translated
    by +1000: the bar depends on each curve's extent, not on its distance from the origin."""
    import paper_2606_25569_amd as V
    sizes = [4, 7, 8, 31, 32, 64, 128, 255, 1000, 1024]
    X, off = _curves(sizes, 5)
    X0, X1 = _exact_shift(X, off, shift)
    rng = np.random.default_rng(6)
    sigma = rng.normal(size=X.shape[1])
    _check_force(V, X1, off, sizes, sigma, 0.7, f"elastic +{shift:g}")


@pytest.mark.parametrize("sizes", [
    [3, 17, 33, 63, 64, 65, 5, 40, 1, 64],        # mean <= 64: one point per lane (R = 1), 65 -> workgroup kernel
    [65, 100, 127, 128, 129, 70, 99, 101],        # mean in (64, 128]: two points per lane (R = 2)
    [129, 200, 255, 256, 257, 130, 203, 131],     # mean in (128, 256]: four points per lane (R = 4)
])
def test_elastic_force_wavefront_forms(sizes):
    """Partitions whose mean size selects each one-wavefront form: sizes that are not multiples of the
    points per lane, lanes past the last point, and vesicles just above the wavefront capacity that
    fall to the workgroup kernel (the 2000 x 128 workload takes the R = 2 form)."""
    import paper_2606_25569_amd as V
    X, off = _curves(sizes, 31 + len(sizes))
    X0, X1 = _exact_shift(X, off, 1000.0)
    rng = np.random.default_rng(7)
    sigma = rng.normal(size=X.shape[1])
    _check_force(V, X1, off, sizes, sigma, 1.1, f"wavefront mean {int(np.mean(sizes))}")


def test_elastic_force_zero_tension_and_degenerate_sizes():
    import torch
    import paper_2606_25569_amd as V
    X, off = _curves([32, 2, 1100, 16], 9)
    Xd = torch.tensor(X, device="cuda")
    f0, w0 = V.elastic_force(Xd, off, 1.3, None)
    f1, w1 = V.elastic_force(Xd, off, 1.3, torch.zeros(X.shape[1], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    f0, f1, w0 = f0.cpu().numpy(), f1.cpu().numpy(), w0.cpu().numpy()
    assert np.isfinite(f0[:, :32]).all() and np.isfinite(f0[:, -16:]).all()
    np.testing.assert_array_equal(f0[:, :32], f1[:, :32])
    assert np.isnan(f0[:, 32:34]).all()              # two points: no tangent
    assert np.isnan(f0[:, 34:34 + 1100]).all() and np.isnan(w0[34:34 + 1100]).all()  # above 1024 points


def _force_error_bound(X, f, off):
    """Per point: the bounds of _check_force on f and on w (the GPU force differs from the oracle's by
    at most these)."""
    tf = np.zeros(X.shape[1])
    tw = np.zeros(X.shape[1])
    for v in range(len(off) - 1):
        a, b = off[v], off[v + 1]
        n = b - a
        ext = np.abs(X[:, a:b] - X[:, a:a + 1]).max()
        tf[a:b] = 64 * EPS * ext * (n / 2) ** 4 + 64 * EPS * np.abs(f[:, a:b]).max()
        tw[a:b] = 16 * EPS * ext * n * max(1.0, np.log2(n)) * (2 * np.pi / n)
    return tf, tw


@pytest.mark.parametrize("tension", ["smooth", "rough"])
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32c", 1e-5)])
def test_force_then_far_field(prec, bar, tension):
    """One solver step's explicit part on 16 x 32: membrane force and weights on the GPU, then the
    far-field sum, against the oracle doing both steps.  The GPU force may differ from the oracle's
    by the spectral bounds of _check_force (dF_j on w f, per point), and the sum carries such a
    difference to target i as at most c sum_j (|ln r_ij| + 1) dF_j; the bar is the sum's own (relative
    to max |u|) plus that propagated bound, which matters when the tension is rough: then the force
    is dominated by wavenumbers near N/2, whose far fields cancel, and max |u| is small next to |f|."""
    import torch
    import paper_2606_25569_amd as V
    s = S.make_config(0)
    rng = np.random.default_rng(12)
    sigma = np.empty(s.n_points)
    for v in range(s.n_vesicles):
        a, b = s.offsets[v], s.offsets[v + 1]
        t = 2 * np.pi * np.arange(b - a) / (b - a)
        if tension == "smooth":
            # membrane tension varies on the vesicle scale
            sigma[a:b] = 1.0 + 0.3 * np.cos(2 * t + rng.uniform(0, 2 * np.pi)) + 0.1 * np.sin(t)
        else:
            sigma[a:b] = 1.0 + rng.standard_normal(b - a)
    f_ref, w_ref = SP.elastic_force(s.X, sigma, 0.5, s.offsets)
    u_ref = O.farfield_suspension(s.X, f_ref, w_ref, s.offsets, s.mu)
    X = torch.tensor(s.X, device="cuda")
    f, w = V.elastic_force(X, s.offsets, 0.5, torch.tensor(sigma, device="cuda"))
    u = V.farfield_forward(X, X, f, w, s.offsets, s.mu, prec)
    torch.cuda.synchronize()
    tf, tw = _force_error_bound(s.X, f_ref, s.offsets)
    dF = w_ref * tf + tw * np.abs(f_ref).max(axis=0) + tf * tw
    vid = np.repeat(np.arange(s.n_vesicles), np.diff(s.offsets))
    r = np.hypot(s.X[0][:, None] - s.X[0][None, :], s.X[1][:, None] - s.X[1][None, :])
    other = vid[:, None] != vid[None, :]
    K = np.where(other, np.abs(np.log(np.where(other, r, 1.0))) + 1.0, 0.0)
    prop = (K @ dF) / (4 * np.pi * s.mu)
    d = np.abs(u.cpu().numpy() - u_ref)
    scale = np.abs(u_ref).max()
    err = float(np.max(d - prop[None, :]) / scale)
    say(f"force -> far field {prec} {tension}: max rel err {d.max() / scale:.3e}, "
        f"propagated force bound {prop.max() / scale:.3e} of max|u|, excess {err:.3e}")
    assert err <= bar
