"""GPU parity of the adjoint for one point array (targets = sources) through the C-ABI entry
vesnet_farfield_stokeslet_backward_points, against the oracle's gradient.

Under fp32c and fp64 each unordered pair of points in different vesicles is evaluated once (the
symmetric forms of the forward; float64 on global coordinates); the two gathers remain for separate
target and source arrays (tests/test_gpu_backward.py).
Bars: 1e-5 (fp32c) and 1e-12 (fp64) in max-norm error relative to the largest component, per
output.  The cases cover one, two and three targets per thread (small problems take one), ragged and
empty vesicles, vesicles longer than a block, several blocks of both parities, a translated
suspension, the partial requests and the zero cases.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import suspension as S
from tests.gpu_util import rel_err, say
from tests.test_gpu_symmetric import _ragged_suspension

pytestmark = pytest.mark.gpu

BARS = {"fp32c": 1e-5, "fp64": 1e-12}


@pytest.fixture(scope="module")
def V():
    import paper_2606_25569_amd as V
    return V


def _g(s, seed):
    return np.random.default_rng(seed).standard_normal((2, s.n_points))


def _points(V, s, g, prec, need=(True, True, True)):
    import torch
    X = torch.tensor(s.X, device="cuda")
    f = torch.tensor(s.f, device="cuda")
    w = torch.tensor(s.w, device="cuda")
    gd = torch.tensor(g, device="cuda")
    out = V.farfield_backward_points(X, f, w, s.offsets, s.mu, gd, prec, need)
    torch.cuda.synchronize()
    return [None if a is None else a.cpu().numpy() for a in out]


def _check(s, got, ref, prec, tag, sel=None):
    names = ("grad_X", "grad_f", "grad_w")
    for name, a in zip(names, got):
        if a is None:
            continue
        if sel is not None:
            a = a[..., sel]
        err, rms = rel_err(a, ref[name])
        say(f"{tag} {name} {prec}: max rel err {err:.3e} rms {rms:.3e}")
        assert err <= BARS[prec], (name, err)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_config0(V, prec):
    s = S.make_config(0)
    g = _g(s, 10)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g)
    _check(s, _points(V, s, g, prec), ref, prec, "cfg0")


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_ragged_partition(V, prec):
    s = _ragged_suspension()
    g = _g(s, 11)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g)
    _check(s, _points(V, s, g, prec), ref, prec, "ragged")


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
@pytest.mark.parametrize("m", [90, 131])
def test_many_blocks_odd_and_even(V, m, prec):
    rng = np.random.default_rng(m)
    s = _ragged_suspension(seed=m, sizes=list(rng.integers(1, 90, size=m)), spacing=4.5)
    g = _g(s, m)
    sel = S.sample_targets(s.n_points, 0.25, m)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g, select=sel)
    _check(s, _points(V, s, g, prec), ref, prec, f"many blocks m={m}", sel)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_vesicle_larger_than_block(V, prec):
    rng = np.random.default_rng(8)
    sizes = np.array([2500, 7, 1030, 33])
    centers = np.array([[0.0, 0.0], [30.0, 0.0], [0.0, 30.0], [30.0, 30.0]])
    axes = np.array([[10.0, 4.0], [1.2, 0.5], [6.0, 3.0], [1.3, 0.4]])
    s = S._assemble(rng, centers, axes, rng.uniform(0, 6.28, 4), sizes, "k4", 0.2, 1.0, 40.0)
    g = _g(s, 12)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g)
    _check(s, _points(V, s, g, prec), ref, prec, "large vesicle")


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_large_translation(V, prec):
    s = _ragged_suspension()
    s.X = s.X + np.array([[1000.0], [-1000.0]])
    g = _g(s, 13)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g)
    _check(s, _points(V, s, g, prec), ref, prec, "+1000")


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_config4_sampled(V, prec):
    """512 x 64 at 30% (two targets per thread under fp32c), 400 sampled points."""
    s = S.load_config(4)
    g = _g(s, 14)
    sel = S.sample_targets(s.n_points, 400 / s.n_points, 4141)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g, select=sel)
    _check(s, _points(V, s, g, prec), ref, prec, "cfg4", sel)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_default_shape_of_large_problems(V, prec):
    """About 38,000 points in 400 vesicles of 60 .. 129 points: large enough for the compensated adjoint's
    three targets per thread (768-point blocks, at least four units per compute unit), 400 sampled points."""
    rng = np.random.default_rng(21)
    s = _ragged_suspension(seed=21, sizes=list(rng.integers(60, 130, size=400)), spacing=4.5)
    g = _g(s, 21)
    sel = S.sample_targets(s.n_points, 400 / s.n_points, 2121)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, g, select=sel)
    say(f"large adjoint: P={s.n_points}")
    _check(s, _points(V, s, g, prec), ref, prec, "large", sel)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_partial_requests_agree(V, prec):
    """grad_force and grad_weights alone, or with the positions, give the same values up to the order
    of the float64 atomic additions (fp32c: the position gradient then goes to the workspace)."""
    s = _ragged_suspension(seed=5)
    g = _g(s, 15)
    full = _points(V, s, g, prec)
    only_f = _points(V, s, g, prec, (False, True, False))
    only_w = _points(V, s, g, prec, (False, False, True))
    assert only_f[0] is None and only_f[2] is None and only_w[1] is None
    assert rel_err(only_f[1], full[1])[0] <= BARS[prec]
    assert rel_err(only_w[2], full[2])[0] <= BARS[prec]


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_zero_cases(V, prec):
    """Zero dL/du gives zero gradients; one vesicle has no cross pairs at all."""
    s = S.make_config(0)
    for a in _points(V, s, np.zeros((2, s.n_points)), prec):
        assert np.all(a == 0.0)
    a, b = S.ellipse_axes(0.65)
    X, w, th = S.ellipse_curve((0.0, 0.0), a, b, 0.0, 40)
    s1 = S.Suspension(X=X, f=np.stack([np.cos(th), np.sin(th)]), w=w, offsets=np.array([0, 40], np.int32), mu=1.0,
                      box=4.0, centers=np.zeros((1, 2)), axes=np.array([[a, b]]), angles=np.zeros(1))
    for a in _points(V, s1, _g(s1, 16), prec):
        assert np.all(a == 0.0)


def test_autograd_takes_the_points_form_for_one_tensor(V):
    """farfield_stokeslet(X, X, ...) differentiates X through the points entry; passing a copy as
    the sources takes the two gathers.  Both match the oracle."""
    import torch
    s = _ragged_suspension(seed=9)
    ustar = np.random.default_rng(17).standard_normal((2, s.n_points))
    u = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    ref = O.grad_suspension(s.X, s.f, s.w, s.offsets, s.mu, u - ustar)
    for same in (True, False):
        X = torch.tensor(s.X, device="cuda", requires_grad=True)
        f = torch.tensor(s.f, device="cuda", requires_grad=True)
        w = torch.tensor(s.w, device="cuda")
        for prec in ("fp32c", "fp64"):
            X.grad = None
            f.grad = None
            Y = X if same else X * 1.0
            out = V.farfield_stokeslet(X, Y, f, w, s.offsets, s.mu, precision=prec)
            (0.5 * ((out - torch.tensor(ustar, device="cuda")) ** 2).sum()).backward()
            torch.cuda.synchronize()
            for name, a in (("grad_X", X.grad), ("grad_f", f.grad)):
                err, _ = rel_err(a.cpu().numpy(), ref[name])
                say(f"autograd same={same} {prec} {name}: {err:.3e}")
                assert err <= BARS[prec], (same, prec, name, err)
