"""GPU parity of the fast-multipole far field: against the fast-multipole oracle of the same depth
and order (same tree; the GPU translates multipole series into Taylor polynomials box to box and
re-centres them down the levels, the oracle forms every level's polynomials from directly summed
moments), and against the exact sum within the oracle's truncation bound."""
import numpy as np
import pytest

from oracle import fmm as FM
from oracle import oracle as O
from synth import suspension as S
from tests.gpu_util import dev_inputs, rel_err, say

pytestmark = pytest.mark.gpu


def _run(s, order, depth):
    import torch
    import paper_2606_25569_amd as V
    X, f, w = dev_inputs(s)
    u = V.farfield_fmm(X, f, w, s.offsets, s.mu, order, depth)
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.fixture(scope="module")
def susp():
    return S.rsa_suspension(5, 120, 24, 0.3)


@pytest.fixture(scope="module")
def exact(susp):
    return O.farfield_suspension(susp.X, susp.f, susp.w, susp.offsets, susp.mu)


@pytest.mark.parametrize("depth", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("order", [8, 20])
def test_fmm_parity_with_oracle(susp, depth, order):
    """Same tree and order: the two differ by rounding only: 1e-12 of max|u|."""
    got = _run(susp, order, depth)
    ref = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, order, depth)
    err, rms = rel_err(got, ref)
    say(f"fmm depth={depth} order={order}: err vs oracle {err:.2e} (rms {rms:.1e})")
    assert err <= 1e-12


@pytest.mark.parametrize("depth,order", [(2, 1), (3, 48), (5, 3)])
def test_fmm_order_and_depth_extremes(susp, depth, order):
    """Order 1 and the largest order (whole-table LDS staging), and a tree deeper than the points need
    (many empty boxes and leaves)."""
    got = _run(susp, order, depth)
    ref = FM.fmm(susp.X, susp.f, susp.w, susp.offsets, susp.mu, order, depth)
    err, _ = rel_err(got, ref)
    say(f"fmm depth={depth} order={order}: err vs oracle {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("depth,order", [(3, 6), (3, 16), (4, 30)])
def test_fmm_within_truncation_bound(susp, exact, depth, order):
    got = _run(susp, order, depth)
    b = FM.truncation_bound(susp.X, susp.f, susp.w, susp.offsets, susp.mu, order, depth)
    err = np.abs(got - exact).max(axis=0)
    say(f"fmm depth={depth} order={order}: err vs exact {err.max() / np.abs(exact).max():.2e} of max|u|, "
        f"worst err/bound {(err / (b + 1e-300)).max():.2e}")
    assert np.all(err <= b + 1e-12 * np.abs(exact).max())


def _ragged():
    """Vesicles of 0 .. 130 points (empty ones, and single points whose spacing h_v = 2 pi) on a grid 4 apart."""
    rng = np.random.default_rng(9)
    sizes = [0, 1, 7, 33, 64, 130, 0, 90] * 8
    Xs, fs, ws, off = [], [], [], [0]
    for k, n in enumerate(sizes):
        a, b = S.ellipse_axes(0.65)
        t = 2 * np.pi * np.arange(n) / max(n, 1)
        c = np.array([[4.0 * (k % 6)], [4.0 * (k // 6)]])
        Xs.append(c + np.stack([a * np.cos(t), b * np.sin(t)]))
        fs.append(rng.normal(size=(2, n)))
        ws.append(np.full(n, 2 * np.pi / max(n, 1)))
        off.append(off[-1] + n)
    return S.Suspension(X=np.concatenate(Xs, 1), f=np.concatenate(fs, 1), w=np.concatenate(ws),
                        offsets=np.asarray(off, np.int32), mu=0.7, box=24.0, centers=None, axes=None, angles=None)


def test_fmm_ragged_partition_and_big_leaves():
    """Vesicles of 0 .. 130 points (one empty, one single point), and at depth 0 one leaf of every
    point (more than 2048 points: the unsorted-leaf path)."""
    s = _ragged()
    exact = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    assert s.n_points > 2048
    for depth in (0, 2, 3):
        got = _run(s, 24, depth)
        ref = FM.fmm(s.X, s.f, s.w, s.offsets, s.mu, 24, depth)
        err, _ = rel_err(got, ref)
        err_x, _ = rel_err(got, exact)
        say(f"fmm ragged depth={depth}: err vs oracle {err:.2e}, vs exact {err_x:.2e}")
        assert err <= 1e-12
        assert err_x <= 1e-8


def test_fmm_full_size_sampled():
    """2000 vesicles x 128 points at the default depth and order 30: 400 seeded targets against the
    fast-multipole oracle and the exact sum."""
    s = S.load_config(1)
    got = _run(s, 30, 6)
    sel = np.sort(np.random.default_rng(11).choice(s.n_points, 400, replace=False))
    exact = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu, select=sel)
    ref = FM.fmm(s.X, s.f, s.w, s.offsets, s.mu, 30, 6, sel=sel)
    scale = np.abs(exact).max()
    err_o = np.abs(got[:, sel] - ref).max() / scale
    err_x = np.abs(got[:, sel] - exact).max() / scale
    say(f"fmm 2000x128 depth 6 order 30: err vs oracle {err_o:.2e}, vs exact {err_x:.2e} of max|u|")
    assert err_o <= 1e-12
    assert err_x <= 1e-9


def test_fmm_deterministic_and_graph_replay(susp):
    """Leaves of at most 2048 points give bit-identical results on every call; the call launches
    kernels only, so it can be captured in a HIP graph, and every replay (with eager work in between)
    equals the eager result bit for bit."""
    import torch
    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    X, f, w = dev_inputs(susp)
    part = V.Partition(susp.offsets, "cuda")
    ws = torch.empty(L.lib().vesnet_fmm_workspace_bytes(susp.n_points, 4, 16), dtype=torch.uint8, device="cuda")
    out = torch.empty((2, susp.n_points), dtype=torch.float64, device="cuda")
    eager = V.farfield_fmm(X, f, w, part, susp.mu, 16, 4, out=out, workspace=ws).clone()
    again = V.farfield_fmm(X, f, w, part, susp.mu, 16, 4, out=torch.empty_like(out), workspace=ws)
    assert torch.equal(eager, again)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        V.farfield_fmm(X, f, w, part, susp.mu, 16, 4, out=out, workspace=ws)  # warm-up on the side stream
        with torch.cuda.graph(g, stream=s):
            V.farfield_fmm(X, f, w, part, susp.mu, 16, 4, out=out, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        out.fill_(float(k) - 7.0)
        V.farfield_treecode(X, f, w, part, susp.mu, 8, 3)  # unrelated eager work in between
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
    say("fmm: deterministic, 3 graph replays equal the eager call")


def _fmm_masked_ref(s, order, depth):
    """Fast-multipole oracle minus the near vesicles' exact sums (the plain direct oracle minus the masked one)."""
    plain = O.farfield_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    masked, pairs = O.nearmasked_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    return FM.fmm(s.X, s.f, s.w, s.offsets, s.mu, order, depth) - (plain - masked), pairs


@pytest.mark.parametrize("depth,order", [(0, 8), (2, 12), (3, 20), (4, 30)])
def test_fmm_nearmasked_parity(depth, order):
    """Dense suspension at gap 0.02 (every distance at least 1e-5 relative away from the spacing): the near
    pairs equal the oracle's exactly, and the masked field equals the fast-multipole oracle minus the near
    vesicles' exact sums within 1e-12 of max|u|."""
    import torch
    import paper_2606_25569_amd as V
    from tests.gpu_util import near_margin
    s = S.rsa_suspension(33, 120, 32, 0.40, gap=0.02)
    assert near_margin(s) > 1e-5
    ref, pairs_ref = _fmm_masked_ref(s, order, depth)
    assert pairs_ref.shape[0] > 20
    X, f, w = dev_inputs(s)
    out, pairs = V.farfield_fmm_nearmasked(X, f, w, s.offsets, s.mu, order, depth)
    torch.cuda.synchronize()
    got = {tuple(p) for p in pairs.cpu().numpy().tolist()}
    err, _ = rel_err(out.cpu().numpy(), ref)
    say(f"fmm nearmasked depth={depth} order={order}: err vs oracle {err:.2e}, {len(got)} near pairs")
    assert got == {tuple(p) for p in pairs_ref.tolist()}
    assert len(got) == pairs.shape[0]  # no pair twice
    assert err <= 1e-12


def test_fmm_nearmasked_small_list_and_determinism():
    """A list smaller than the pairs reports the full count and still masks completely: out equals the
    full-list call bit for bit, and repeated calls agree bit for bit."""
    import torch
    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    s = S.rsa_suspension(34, 60, 32, 0.40, gap=0.02)
    X, f, w = dev_inputs(s)
    part = V.Partition(s.offsets, "cuda")
    full, pairs = V.farfield_fmm_nearmasked(X, f, w, part, s.mu, 16, 3)
    again, _ = V.farfield_fmm_nearmasked(X, f, w, part, s.mu, 16, 3)
    assert torch.equal(full, again)
    lib = L.lib()
    P, M = s.n_points, len(s.offsets) - 1
    ws = torch.empty(lib.vesnet_fmm_nearmasked_workspace_bytes(P, M, 3, 16), dtype=torch.uint8, device="cuda")
    out = torch.empty((2, P), dtype=torch.float64, device="cuda")
    small = torch.empty((3, 2), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    L.check(lib.vesnet_farfield_fmm_nearmasked(X.data_ptr(), f.data_ptr(), w.data_ptr(), part.device.data_ptr(), M, P,
                                               float(s.mu), 16, 3, out.data_ptr(), small.data_ptr(), 3,
                                               count.data_ptr(), ws.data_ptr(), ws.numel(),
                                               torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(count.item()) == pairs.shape[0] > 3
    assert torch.equal(out, full)


def test_fmm_nearmasked_spacing_above_leaf_width_is_reported():
    """At depth 8 over 60 vesicles the leaves (about 0.06 wide) are narrower than the spacing (0.2): the
    count is -2 and the binding raises."""
    import torch
    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    s = S.rsa_suspension(34, 60, 32, 0.40, gap=0.02)
    X, f, w = dev_inputs(s)
    with pytest.raises(L.VesnetError, match="leaf width"):
        V.farfield_fmm_nearmasked(X, f, w, s.offsets, s.mu, 8, 8)
    torch.cuda.synchronize()


def test_fmm_nearmasked_ragged_and_empty():
    """The ragged partition (empty vesicles, single points with h_v = 2 pi, leaves of more than 64 points):
    at depths 0-2 (leaves at least 10 wide) the pairs and the field match the oracles; at depth 3 (leaves
    5.1 wide) the spacing is reported.  No points at all: count 0."""
    import torch
    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    from tests.gpu_util import near_margin
    s = _ragged()
    assert near_margin(s) > 1e-5
    X, f, w = dev_inputs(s)
    for depth in (0, 1, 2):
        ref, pairs_ref = _fmm_masked_ref(s, 24, depth)
        out, pairs = V.farfield_fmm_nearmasked(X, f, w, s.offsets, s.mu, 24, depth)
        torch.cuda.synchronize()
        got = {tuple(p) for p in pairs.cpu().numpy().tolist()}
        err, _ = rel_err(out.cpu().numpy(), ref)
        say(f"fmm nearmasked ragged depth={depth}: err vs oracle {err:.2e}, {len(got)} near pairs")
        assert got == {tuple(p) for p in pairs_ref.tolist()} and len(got) == pairs.shape[0] > 1000
        assert err <= 1e-12
    with pytest.raises(L.VesnetError, match="leaf width"):
        V.farfield_fmm_nearmasked(X, f, w, s.offsets, s.mu, 24, 3)
    torch.cuda.synchronize()
    lib = L.lib()
    off = torch.zeros(3, dtype=torch.int32, device="cuda")  # two empty vesicles
    count = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    nothing = torch.empty((2, 0), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(1, lib.vesnet_fmm_nearmasked_workspace_bytes(0, 2, 2, 8)), dtype=torch.uint8, device="cuda")
    L.check(lib.vesnet_farfield_fmm_nearmasked(nothing.data_ptr(), nothing.data_ptr(), nothing.data_ptr(),
                                               off.data_ptr(), 2, 0, 1.0, 8, 2, nothing.data_ptr(), None, 0,
                                               count.data_ptr(), ws.data_ptr(), ws.numel(),
                                               torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert int(count.item()) == 0
