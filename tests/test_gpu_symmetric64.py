"""GPU parity of the symmetric float64 forward (each unordered pair evaluated once, two-word
fixed-point accumulation) against the CPU oracle, through the C-ABI.

pair_form 2 forces the form; the automatic choice takes it for one point array in float64 when the
problem is large enough.  Bar: <= 1e-12 in max-norm error relative to max |u| (component-wise), as for
the direct float64 kernel.  The sums are added as fixed-point integers, so repeated calls agree bit for
bit.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import suspension as S
from tests.gpu_util import dev_inputs, rel_err, say
from tests.test_gpu_symmetric import _ragged_suspension

pytestmark = pytest.mark.gpu

BAR = 1e-12


@pytest.fixture(scope="module")
def V():
    import paper_2606_25569_amd as V
    return V


def _sym64(V, s, T=None):
    import torch
    X, f, w = dev_inputs(s)
    cfg = {"pair_form": 2}
    if T:
        cfg["targets_per_thread"] = T
    out = V.farfield_forward(X, X, f, w, s.offsets, s.mu, precision="fp64", config=cfg)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_config0(V, T):
    s = S.make_config(0)
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    err, rms = rel_err(_sym64(V, s, T), ref)
    say(f"symmetric fp64 cfg0 T={T}: {err:.3e} rms {rms:.3e}")
    assert err <= BAR


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_ragged_partition(V, T):
    """Empty, single-point and odd-sized vesicles; one block holds the whole suspension."""
    s = _ragged_suspension()
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    err, _ = rel_err(_sym64(V, s, T), ref)
    say(f"symmetric fp64 ragged T={T}: {err:.3e}")
    assert err <= BAR


@pytest.mark.parametrize("m", [90, 131])
def test_many_blocks_odd_and_even(V, m):
    """Several blocks of both parities of the block count; vesicles straddle block boundaries."""
    rng = np.random.default_rng(m)
    sizes = list(rng.integers(1, 90, size=m))
    s = _ragged_suspension(seed=m, sizes=sizes, spacing=4.5)
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    for T in (1, 2, 3, 4):
        err, _ = rel_err(_sym64(V, s, T), ref)
        say(f"symmetric fp64 many blocks m={m} T={T}: {err:.3e}")
        assert err <= BAR


def test_vesicle_larger_than_block(V):
    """A vesicle of 2500 points covers several blocks of 256, 512 and 1024 points."""
    rng = np.random.default_rng(8)
    sizes = np.array([2500, 7, 1030, 33])
    centers = np.array([[0.0, 0.0], [30.0, 0.0], [0.0, 30.0], [30.0, 30.0]])
    axes = np.array([[10.0, 4.0], [1.2, 0.5], [6.0, 3.0], [1.3, 0.4]])
    s = S._assemble(rng, centers, axes, rng.uniform(0, 6.28, 4), sizes, "k4", 0.2, 1.0, 40.0)
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    for T in (1, 2, 4):
        err, _ = rel_err(_sym64(V, s, T), ref)
        say(f"symmetric fp64 large vesicle T={T}: {err:.3e}")
        assert err <= BAR


def test_large_translation(V):
    """Every point shifted by (+1000, -1000): float64 on global coordinates keeps the bar."""
    s = _ragged_suspension()
    s.X = s.X + np.array([[1000.0], [-1000.0]])
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    err, _ = rel_err(_sym64(V, s, 2), ref)
    say(f"symmetric fp64 +1000: {err:.3e}")
    assert err <= BAR


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_scaled_suspension(V, scale):
    """Coordinates and weights scaled by 1e-6 and 1e6: |r|^2 spans exponents of about -40 and +40, where the
    logarithm's e ln 2 term dominates; every float64 form (symmetric at T = 1 and the default, direct) within
    the bar of the oracle."""
    import torch
    s = _ragged_suspension(seed=9)
    s.X = s.X * scale
    s.w = s.w * scale
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    for cfg in ({"pair_form": 2, "targets_per_thread": 1}, {"pair_form": 2}, {"pair_form": 1}):
        X, f, w = dev_inputs(s)
        out = V.farfield_forward(X, X, f, w, s.offsets, s.mu, precision="fp64", config=cfg)
        torch.cuda.synchronize()
        err, _ = rel_err(out.cpu().numpy(), ref)
        say(f"fp64 scaled x{scale:g} {cfg}: {err:.3e}")
        assert err <= BAR


def test_single_vesicle_and_zero_force(V):
    a, b = S.ellipse_axes(0.65)
    X, w, th = S.ellipse_curve((0.0, 0.0), a, b, 0.0, 40)
    s = S.Suspension(X=X, f=np.stack([np.cos(th), np.sin(th)]), w=w, offsets=np.array([0, 40], np.int32), mu=1.0,
                     box=4.0, centers=np.zeros((1, 2)), axes=np.array([[a, b]]), angles=np.zeros(1))
    assert np.all(_sym64(V, s, 1) == 0.0)
    s2 = S.make_config(0)
    s2.f = np.zeros_like(s2.f)
    assert np.all(_sym64(V, s2, 2) == 0.0)


def test_bitwise_repeatable(V):
    """Two-word fixed-point accumulation: the result does not depend on the order of the atomics."""
    s = _ragged_suspension(seed=3, sizes=list(np.random.default_rng(3).integers(1, 90, size=120)), spacing=4.5)
    a = _sym64(V, s, 1)
    for _ in range(3):
        assert np.array_equal(_sym64(V, s, 1), a)


def test_automatic_choice(V):
    """One float64 point array large enough for the symmetric form takes it; separate arrays and
    pair_form 1 take the direct form; all within the bar of each other."""
    import torch
    s = _ragged_suspension(seed=5, sizes=list(np.random.default_rng(5).integers(60, 130, size=400)), spacing=4.5)
    X, f, w = dev_inputs(s)
    auto = V.farfield_forward(X, X, f, w, s.offsets, s.mu, precision="fp64")
    forced = V.farfield_forward(X, X, f, w, s.offsets, s.mu, precision="fp64", config={"pair_form": 2})
    direct = V.farfield_forward(X, X, f, w, s.offsets, s.mu, precision="fp64", config={"pair_form": 1})
    torch.cuda.synchronize()
    assert torch.equal(auto, forced)
    assert rel_err(auto.cpu().numpy(), direct.cpu().numpy())[0] <= BAR


def test_config1_sampled_full_size(V):
    """2000 x 128 (256,000 points) in the default float64 form, on the seeded 1% sample."""
    s = S.load_config(1)
    sel = S.sample_targets(s.n_points, 0.01, 101)
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)
    err, rms = rel_err(_sym64(V, s)[:, sel], ref)
    say(f"cfg1 symmetric fp64: max rel err {err:.3e}  rms {rms:.3e}")
    assert err <= BAR


@pytest.mark.parametrize("variant", ["force_free", "net_force"])
def test_config2_precision_study(V, variant):
    """8000 x 64 at 35% on a 1% target sample."""
    s = S.load_config(2, variant)
    sel = S.sample_targets(s.n_points, 0.01, 202)
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)
    err, rms = rel_err(_sym64(V, s)[:, sel], ref)
    say(f"cfg2 {variant} symmetric fp64: max rel err {err:.3e}  rms {rms:.3e}")
    assert err <= BAR
