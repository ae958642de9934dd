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
    import torch
    b = _small_batch()
    X, f, w = _dev(b)
    bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision=prec,
                          config={"targets_per_thread": 2, "block_threads": 128, "blocks_per_cu": 2,
                                  "source_staging": staging})
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
                                        "source_staging": staging})
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


def test_config3_batched_vs_loop(V):
    """64 suspensions (M log-uniform in [10, 1500], N in {32, 64, 128}): the
    persistent launch equals the per-suspension results and the oracle."""
    import torch
    b = S.load_config(3)
    say(f"cfg3: S={b.n_suspensions} P={b.n_points} pairs={b.cross_pairs():.3e}")
    X, f, w = _dev(b)
    bp = V.BatchedProblem(X, X, f, w, b.vesicle_offsets, b.suspension_offsets, b.mu, precision="fp32c")
    out = bp.run().cpu().numpy()
    refs = _per_suspension_oracle(b, frac=0.01, seed=3000)
    worst = _check_against(b, out, refs, 1e-5)
    say(f"cfg3 batched fp32c worst rel err {worst:.3e}")
    torch.cuda.synchronize()


def test_autotune_returns_valid_shape(V):
    import torch
    s = S.make_config(0)
    X = torch.tensor(s.X, device="cuda")
    f = torch.tensor(s.f, device="cuda")
    w = torch.tensor(s.w, device="cuda")
    best, ms = V.autotune(X, X, f, w, s.offsets, 1.0, "fp32c", repeats=2, store=False)
    d = best.as_dict()
    assert d["targets_per_thread"] in (1, 2, 4) and d["block_threads"] in (64, 128, 256) and ms > 0
    ref = O.farfield_suspension(s.X, s.f, s.w, s.offsets, 1.0)
    out = V.farfield_forward(X, X, f, w, s.offsets, 1.0, "fp32c", config=best).cpu().numpy()
    assert rel_err(out, ref)[0] <= 1e-5
