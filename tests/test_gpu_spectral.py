"""GPU parity of the membrane force and trapezoid weights (eq. (elastic_force),
spectral derivatives of Section 2.2.1), and of the full step force -> far field."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import spectral as SP
from synth import suspension as S
from tests.gpu_util import rel_err, say

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


def test_elastic_force_parity_across_sizes():
    import torch
    import paper_2606_25569_amd as V
    sizes = [4, 7, 8, 31, 32, 64, 128, 255, 1000, 1024]
    X, off = _curves(sizes, 5)
    rng = np.random.default_rng(6)
    sigma = rng.normal(size=X.shape[1])
    ref_f, ref_w = SP.elastic_force(X, sigma, 0.7, off)
    f, w = V.elastic_force(torch.tensor(X, device="cuda"), off, 0.7, torch.tensor(sigma, device="cuda"))
    torch.cuda.synchronize()
    f, w = f.cpu().numpy(), w.cpu().numpy()
    for v, n in enumerate(sizes):
        a, b = off[v], off[v + 1]
        # rounding of the points, amplified by at most N/2 per derivative (four of them)
        tol = 64 * EPS * np.abs(X[:, a:b]).max() * (n / 2) ** 4 + 64 * EPS * np.abs(ref_f[:, a:b]).max()
        df = np.abs(f[:, a:b] - ref_f[:, a:b]).max()
        say(f"elastic N={n}: max |df| {df:.3e} (bound {tol:.3e}), rel {df / np.abs(ref_f[:, a:b]).max():.3e}")
        assert df <= tol
        # |X_alpha| is a sum of N terms of size up to |X| (global coordinates): rounding of order
        # eps |X| N log2(N), times 2 pi / N for the weight
        atol_w = 16 * EPS * np.abs(X[:, a:b]).max() * n * max(1.0, np.log2(n)) * (2 * np.pi / n)
        np.testing.assert_allclose(w[a:b], ref_w[a:b], rtol=0, atol=atol_w)


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


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("fp32c", 1e-5)])
def test_force_then_far_field(prec, bar):
    """One solver step's explicit part on 16 x 32: membrane force and weights on the GPU, then
    the far-field sum, against the oracle doing both steps."""
    import torch
    import paper_2606_25569_amd as V
    s = S.make_config(0)
    rng = np.random.default_rng(12)
    # a smooth tension per vesicle (membrane tension varies on the vesicle scale)
    sigma = np.empty(s.n_points)
    for v in range(s.n_vesicles):
        a, b = s.offsets[v], s.offsets[v + 1]
        t = 2 * np.pi * np.arange(b - a) / (b - a)
        sigma[a:b] = 1.0 + 0.3 * np.cos(2 * t + rng.uniform(0, 2 * np.pi)) + 0.1 * np.sin(t)
    f_ref, w_ref = SP.elastic_force(s.X, sigma, 0.5, s.offsets)
    u_ref = O.farfield_suspension(s.X, f_ref, w_ref, s.offsets, s.mu)
    X = torch.tensor(s.X, device="cuda")
    f, w = V.elastic_force(X, s.offsets, 0.5, torch.tensor(sigma, device="cuda"))
    u = V.farfield_forward(X, X, f, w, s.offsets, s.mu, prec)
    torch.cuda.synchronize()
    err, _ = rel_err(u.cpu().numpy(), u_ref)
    say(f"force -> far field {prec}: {err:.3e}")
    assert err <= bar
