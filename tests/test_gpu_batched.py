"""GPU tests of the batched persistent form, its HIP graph, and the autotuner."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import suspension as S
from tests.gpu_util import rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import paper_2606_25569_amd as V
    return V


def _small_batch():
    members = [S.rsa_suspension(900 + k, m, n, phi) for k, (m, n, phi) in
               enumerate([(10, 32, 0.2), (37, 64, 0.3), (5, 128, 0.25), (80, 32, 0.35), (1, 64, 0.2), (23, 128, 0.3)])]
    mus = [1.0, 0.5, 2.0, 1.3, 1.0, 0.8]
    return S.batch_of(members, mus)


def _dev(b):
    import torch
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    return t(b.X), t(b.f), t(b.w)


def _per_suspension_oracle(b, frac=None, seed=0):
    refs = []
    for k, m in enumerate(b.members):
        sel = None if frac is None or m.n_points < 20000 else S.sample_targets(m.n_points, frac, seed + k)
        refs.append((sel, O.farfield_suspension(m.X, m.f, m.w, m.offsets, b.mu[k], select=sel)))
    return refs


def _check_against(b, out, refs, bar):
    base = 0
    worst = 0.0
    for k, m in enumerate(b.members):
        o = out[:, base:base + m.n_points]
        sel, ref = refs[k]
        if m.n_vesicles > 1:
            err, _ = rel_err(o if sel is None else o[:, sel], ref)
            worst = max(worst, err)
        else:
            assert np.all(o == 0.0)
        base += m.n_points
    assert worst <= bar, worst
    return worst


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32c", 1e-5)])
@pytest.mark.parametrize("staging", [1, 2])
def test_small_batch_matches_oracle_and_single_calls(V, prec, bar, staging):
    """The direct persistent form (pair_form 1): the oracle per suspension, and single calls of the
    same launch shape bit for bit."""
    import torch
    b = _small_batch()
    X, f, w = _dev(b)
    bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision=prec,
                          config={"targets_per_thread": 2, "block_threads": 128, "blocks_per_cu": 2,
                                  "source_staging": staging, "pair_form": 1})
    out = bp.run().cpu().numpy()
    worst = _check_against(b, out, _per_suspension_oracle(b), bar)
    say(f"small batch {prec}: worst rel err {worst:.3e}")
    # identical launch shape, one call per suspension: same summation order, same bits
    base = 0
    for k, m in enumerate(b.members):
        sl = slice(base, base + m.n_points)
        o1 = V.farfield_forward(X[:, sl].contiguous(), X[:, sl].contiguous(), f[:, sl].contiguous(),
                                w[sl].contiguous(), m.offsets, b.mu[k], precision=prec,
                                config={"targets_per_thread": 2, "block_threads": 128, "source_splits": 1,
                                        "source_staging": staging, "pair_form": 1})
        np.testing.assert_array_equal(o1.cpu().numpy(), out[:, sl])
        base += m.n_points
    torch.cuda.synchronize()


def test_graph_replays_match_eager(V):
    """Replay the captured graph several times with eager work in between; each
    replay must reproduce the eager result bit for bit."""
    import torch
    b = _small_batch()
    X, f, w = _dev(b)
    bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c")
    eager = bp.run().clone()
    bp.capture()
    for r in range(4):
        bp.out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()  # unrelated eager work
        out = bp.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(out, eager), f"replay {r} differs"
    bp.close()


def _single_symmetric(V, X, f, w, b, T):
    """One symmetric call per suspension (pair_form 2, T targets per thread), concatenated."""
    outs = []
    base = 0
    for k, m in enumerate(b.members):
        sl = slice(base, base + m.n_points)
        base += m.n_points
        Xs = X[:, sl].contiguous()
        outs.append(V.farfield_forward(Xs, Xs, f[:, sl].contiguous(), w[sl].contiguous(), m.offsets, float(b.mu[k]),
                                       "fp32c", config={"pair_form": 2, "targets_per_thread": T}).cpu().numpy())
    return np.concatenate(outs, axis=1)


def _member(seed, sizes, spacing=4.0):
    """Ellipses of the given point counts (0 allowed) on a jittered grid, forces k <= 4 plus a small net
    force, mu = 1."""
    rng = np.random.default_rng(seed)
    m = len(sizes)
    side = max(1, int(np.ceil(np.sqrt(m))))
    centers = np.array([[spacing * (k % side) + rng.uniform(-0.3, 0.3), spacing * (k // side) + rng.uniform(-0.3, 0.3)]
                        for k in range(m)], dtype=np.float64).reshape(m, 2)
    axes = np.tile(S.ellipse_axes(0.7), (m, 1))
    angles = rng.uniform(0, 2 * np.pi, m)
    return S._assemble(rng, centers, axes, angles, np.array(sizes, dtype=np.int64), "k4", 0.05, 1.0, spacing * side)


def _ragged_batch():
    """Ragged vesicles (0 .. 130 points), a suspension without vesicles, vesicles larger than a block of
    one and of two targets per thread (700 and 650 points > 512), a single vesicle, a suspension with one
    vesicle of points among empty ones, and 1,100 two-vesicle suspensions of 1 .. 19 points each, so that
    the plan's scans run over more than one pass of 1,024 suspensions."""
    rng = np.random.default_rng(4242)
    members = [_member(950, [1, 3, 17, 0, 33, 64, 100, 130, 5, 47, 63, 65, 129, 2, 31, 96]), _member(951, []),
               _member(952, [700, 0, 650], spacing=5.0), _member(953, [40]), _member(954, [0, 12, 0])]
    for k in range(1100):
        members.append(_member(2000 + k, [int(x) for x in rng.integers(1, 20, size=2)]))
    return members


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_symmetric_batch_equals_single_symmetric_calls(V, T):
    """The batched symmetric form (the default for one compensated point array) on a small batch: the
    oracle per suspension, and one symmetric call per suspension of the same T bit for bit (fixed-point
    accumulation makes both independent of the order of the atomics)."""
    b = _small_batch()
    X, f, w = _dev(b)
    for bpc in (0, 1):
        cfg = {"pair_form": 2, "targets_per_thread": T, "blocks_per_cu": bpc}
        bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c",
                              config=cfg)
        out = bp.run().cpu().numpy()
        worst = _check_against(b, out, _per_suspension_oracle(b), 1e-5)
        say(f"symmetric batch T={T} bpc={bpc}: worst rel err {worst:.3e}")
        np.testing.assert_array_equal(out, _single_symmetric(V, X, f, w, b, T))


def test_symmetric_batch_ragged(V):
    """Empty suspensions and vesicles, one vesicle per suspension, a vesicle larger than a block, more
    suspensions than one pass of the plan: against the oracle per suspension (zeros where a suspension
    has fewer than two vesicles with points)."""
    members = _ragged_batch()
    mus = [0.5 + 0.01 * (k % 50) for k in range(len(members))]
    b = S.batch_of(members, mus)
    X, f, w = _dev(b)
    for T in (1, 2, 3):
        bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c",
                              config={"pair_form": 2, "targets_per_thread": T})
        out = bp.run().cpu().numpy()
        assert np.all(np.isfinite(out))
        base = 0
        worst = 0.0
        for k, m in enumerate(b.members):
            o = out[:, base:base + m.n_points]
            base += m.n_points
            nonempty = int(np.sum(np.diff(m.offsets) > 0))
            if nonempty < 2:
                assert np.all(o == 0.0), k
                continue
            ref = O.farfield_suspension(m.X, m.f, m.w, m.offsets, b.mu[k])
            worst = max(worst, rel_err(o, ref)[0])
        say(f"ragged symmetric batch T={T}: {b.n_suspensions} suspensions, worst rel err {worst:.3e}")
        assert worst <= 1e-5


def test_config3_batched_vs_loop(V):
    """64 suspensions (M log-uniform in [10, 1500], N in {32, 64, 128}): the persistent launch (the
    batched symmetric form, the default) against the oracle on a 1% target sample of each suspension
    above 20,000 points; equal bit for bit to the one-launch-per-suspension loop of the same form; every
    replay of its HIP graph equal to the eager result; and the autotuner's chosen shape within the bar."""
    import torch
    b = S.load_config(3)
    say(f"cfg3: S={b.n_suspensions} P={b.n_points} pairs={b.cross_pairs():.3e}")
    X, f, w = _dev(b)
    bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c")
    eager = bp.run().clone()
    out = eager.cpu().numpy()
    refs = _per_suspension_oracle(b, frac=0.01, seed=3000)
    worst = _check_against(b, out, refs, 1e-5)
    say(f"cfg3 batched fp32c worst rel err {worst:.3e}")
    # the default batched form takes three targets per thread at this size (the single call's default for
    # the total point count)
    np.testing.assert_array_equal(out, _single_symmetric(V, X, f, w, b, 3))
    say("cfg3 batched equals the per-suspension loop bit for bit")
    bp.capture()
    for r in range(3):
        bp.out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()
        got = bp.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(got, eager), f"replay {r} differs"
    bp.close()
    best, ms = V.autotune(None, None, None, None, None, batched=bp, repeats=1, store=False)
    say(f"cfg3 autotuned {best.as_dict()} {ms:.3f} ms")
    bp.config = best
    tuned = bp.run().cpu().numpy()
    assert _check_against(b, tuned, refs, 1e-5) <= 1e-5
    torch.cuda.synchronize()


def test_autotune_returns_valid_shape(V):
    import torch
    s = S.make_config(0)
    X = torch.tensor(s.X, device="cuda")
    f = torch.tensor(s.f, device="cuda")
    w = torch.tensor(s.w, device="cuda")
    best, ms = V.autotune(X, X, f, w, s.offsets, 1.0, "fp32c", repeats=2, store=False)
    d = best.as_dict()
    if d["pair_form"] == 2:  # the symmetric form: targets per thread only
        assert d["targets_per_thread"] in (1, 2, 3, 4, 8) and ms > 0
    else:
        assert d["targets_per_thread"] in (1, 2, 4) and d["block_threads"] in (64, 128, 256) and ms > 0
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    out = V.farfield_forward(X, X, f, w, s.offsets, 1.0, "fp32c", config=best).cpu().numpy()
    assert rel_err(out, ref)[0] <= 1e-5
