"""GPU parity of the near-field layers and the Gaussian RBF interpolation (Section 3.3,
Algorithm 4 CreateNearLayers / interpolateInNearField) against the oracle."""
import numpy as np
import pytest

from oracle import nearfield_rbf as NR
from oracle import oracle as O
from synth import suspension as S
from tests.gpu_util import dev_inputs, near_margin, rel_err, say

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


def _curves(sizes, seed, clockwise=()):
    """Smooth random closed curves (perturbed ellipses) of the given point counts, far apart;
    the ones listed in clockwise run the other way round.  w = |X_alpha| 2 pi / N exactly."""
    rng = np.random.default_rng(seed)
    X, w, off = [], [], [0]
    for k, n in enumerate(sizes):
        t = 2 * np.pi * np.arange(n) / n
        if k in clockwise:
            t = -t
        a, b = rng.uniform(0.8, 1.4), rng.uniform(0.4, 0.8)
        p3, p5 = rng.uniform(0, 6, 2)
        r = 1.0 + 0.05 * np.cos(3 * t + p3) + 0.03 * np.sin(5 * t + p5)
        dr = -0.15 * np.sin(3 * t + p3) + 0.15 * np.cos(5 * t + p5)
        x = np.stack([a * r * np.cos(t), b * r * np.sin(t)])
        xt = np.stack([a * (dr * np.cos(t) - r * np.sin(t)), b * (dr * np.sin(t) + r * np.cos(t))])
        phi = rng.uniform(0, 2 * np.pi)
        R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
        X.append(R @ x + np.array([[5.0 * k], [3.0 * (k % 2)]]))
        w.append(np.hypot(*xt) * 2 * np.pi / max(n, 1))
        off.append(off[-1] + n)
    return np.concatenate(X, axis=1), np.concatenate(w), np.asarray(off, np.int32)


def _layer_tol(x, w, n):
    """Rounding of the points (eps |X|) plus the spectral tangent's rounding, up to
    16 eps |X| N log2 N / |X_alpha| (one direct circulant sum against an FFT), times h."""
    h = w.sum() / n
    J = w.min() * n / (2 * np.pi)
    return 4 * EPS * np.abs(x).max() + h * 16 * EPS * np.abs(x).max() * n * np.log2(n) / J


def test_layers_parity_across_sizes():
    import torch
    import paper_2606_25569_amd as V
    sizes = [0, 3, 7, 32, 33, 64, 130, 256, 1024]
    X, w, off = _curves(sizes, 21, clockwise=(2, 5))
    ref, _ = NR.near_layers(X, w, off)
    got = V.near_layers(torch.tensor(X, device="cuda"), torch.tensor(w, device="cuda"), off).cpu().numpy()
    for v, n in enumerate(sizes):
        if n == 0:
            continue
        a, b = off[v], off[v + 1]
        tol = _layer_tol(X[:, a:b], w[a:b], n)
        err = np.abs(got[:, 5 * a:5 * b] - ref[:, 5 * a:5 * b]).max()
        say(f"layers N={n}: err {err:.3e} (tol {tol:.1e})")
        assert err <= tol


def test_layers_degenerate_vesicles_are_nan():
    import torch
    import paper_2606_25569_amd as V
    sizes = [1, 2, 5, 1025]
    X, w, off = _curves(sizes, 22)
    got = V.near_layers(torch.tensor(X, device="cuda"), torch.tensor(w, device="cuda"), off).cpu().numpy()
    assert np.isnan(got[:, 0:15]).all()          # 1 and 2 points: no tangent
    assert np.isfinite(got[:, 15:40]).all()      # 5 points
    assert np.isnan(got[:, 40:]).all()           # above 1024 points


def _fit_case(sizes, seed, width, max_points=None):
    import torch
    import paper_2606_25569_amd as V
    X, w, off = _curves(sizes, seed)
    layers, h = NR.near_layers(X, w, off)
    U = S.smooth_field(seed + 1, layers)
    L, Ud, wd = (torch.tensor(a, device="cuda") for a in (layers, U, w))
    coeffs = V.rbf_fit(L, Ud, wd, off, width, max_points)
    return X, w, off, layers, h, U, L, wd, coeffs


def _near_queries(layers, h, off, per, seed):
    """per points in the near zone of every non-empty vesicle (layer nodes moved by up to h/2)."""
    rng = np.random.default_rng(seed)
    Q, pairs = [], []
    for v in range(len(off) - 1):
        a, b = off[v], off[v + 1]
        if b == a:
            continue
        idx = rng.integers(5 * a, 5 * b, per)
        Q.append(layers[:, idx] + rng.uniform(-0.5, 0.5, (2, per)) * h[v])
        pairs += [(len(pairs) + k, v) for k in range(per)]
    return np.concatenate(Q, axis=1), np.asarray(pairs, np.int32)


@pytest.mark.parametrize("width", [0.75, 1.0])
def test_rbf_fit_and_eval_parity(width):
    """Interpolated values at near-zone points agree with the oracle's to the conditioning of each
    vesicle's matrix (10 eps cond(K) max|u|, as the library-interpolator pin), and the GPU
    coefficients solve K c = u with a backward error of a stable Cholesky solve."""
    import torch
    import paper_2606_25569_amd as V
    sizes = [3, 7, 0, 32, 33, 64, 100, 128, 200]
    X, w, off, layers, h, U, L, wd, coeffs = _fit_case(sizes, 31, width)
    c_gpu = coeffs.cpu().numpy()
    c_ref = NR.rbf_fit(layers, U, w, off, width)
    Q, pairs = _near_queries(layers, h, off, 24, 32)
    out = torch.zeros((2, Q.shape[1]), dtype=torch.float64, device="cuda")
    V.rbf_eval_near(L, coeffs, wd, off, torch.tensor(Q, device="cuda"), torch.tensor(pairs, device="cuda"), out,
                    width)
    got = out.cpu().numpy()
    ref = NR.rbf_eval_near(layers, c_ref, w, off, width, Q, pairs)
    for v, n in enumerate(sizes):
        if n == 0:
            continue
        a, b = 5 * off[v], 5 * off[v + 1]
        K = NR.kernel_matrix(layers[:, a:b], width * h[v])
        kappa = np.linalg.cond(K)
        sel = pairs[:, 1] == v
        err = np.abs(got[:, sel] - ref[:, sel]).max()
        tol = 10 * EPS * kappa * np.abs(U[:, a:b]).max()
        resid = np.abs(c_gpu[:, a:b] @ K - U[:, a:b]).max()
        bound = 4 * (b - a) * EPS * np.abs(K).sum(axis=1).max() * np.abs(c_gpu[:, a:b]).max()
        say(f"rbf width={width} N={n}: value err {err:.2e} (tol {tol:.1e}, cond {kappa:.1e}); "
            f"residual {resid:.2e} (bound {bound:.1e})")
        assert err <= tol
        assert resid <= bound


def test_rbf_vesicles_above_max_points_get_nan():
    sizes = [16, 40, 16]
    *_, coeffs = _fit_case(sizes, 41, 1.0, max_points=32)
    c = coeffs.cpu().numpy()
    assert np.isfinite(c[:, :80]).all() and np.isfinite(c[:, 280:]).all()
    assert np.isnan(c[:, 80:280]).all()


def test_rbf_eval_accumulates_and_respects_count():
    """out is added to; only the first min(count, capacity) pairs are read; pairs outside the
    problem are skipped; a target near two vesicles receives both interpolants."""
    import torch
    import paper_2606_25569_amd as V
    sizes = [24, 24]
    X, w, off, layers, h, U, L, wd, coeffs = _fit_case(sizes, 51, 1.0)
    c_ref = NR.rbf_fit(layers, U, w, off, 1.0)
    Q = np.stack([layers[:, 5], layers[:, 130], layers[:, 7]], axis=1)
    pairs = np.array([[0, 0], [0, 1], [1, 1], [2, 5], [7, 0], [2, 0]], np.int32)
    base = np.arange(6, dtype=np.float64).reshape(2, 3)
    kappa = max(np.linalg.cond(NR.kernel_matrix(layers[:, 120 * v:120 * (v + 1)], h[v])) for v in range(2))
    tol = 2 * 10 * EPS * kappa * np.abs(U).max()  # two interpolants at most per target
    Qd = torch.tensor(Q, device="cuda")
    pd = torch.tensor(pairs, device="cuda")
    for count, used in ((5, [0, 1, 2]), (99, [0, 1, 2, 5]), (0, [])):
        out = torch.tensor(base, device="cuda")
        cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
        V.rbf_eval_near(L, coeffs, wd, off, Qd, pd, out, 1.0, near_count=cnt)
        ref = base + NR.rbf_eval_near(layers, c_ref, w, off, 1.0, Q, pairs[used])
        err = np.abs(out.cpu().numpy() - ref).max()
        say(f"eval count={count}: err {err:.2e}")
        assert err <= tol
        if not used:
            np.testing.assert_array_equal(out.cpu().numpy(), base)


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32c", 1e-5)])
def test_near_corrected_single_layer(prec, bar):
    """Algorithm 4 without its networks: u = u_far (near vesicles masked) + u_near interpolated
    from given layer velocities at the near pairs, on a dense 32-point suspension, against the
    oracle's masked far field plus its interpolation."""
    import torch
    import paper_2606_25569_amd as V
    s = S.rsa_suspension(61, 150, 32, 0.35, gap=0.02)
    assert near_margin(s) > 1e-5
    far_ref, pairs_ref = O.nearmasked_suspension(s.X, s.f, s.w, s.offsets, s.mu)
    layers, h = NR.near_layers(s.X, s.w, s.offsets)
    U = 0.05 * S.smooth_field(62, layers)
    c_ref = NR.rbf_fit(layers, U, s.w, s.offsets, 1.0)
    near_ref = NR.rbf_eval_near(layers, c_ref, s.w, s.offsets, 1.0, s.X, pairs_ref)
    X, f, w = dev_inputs(s)
    u, pairs = V.farfield_nearmasked(X, X, f, w, s.offsets, s.mu, prec)
    assert {tuple(p) for p in pairs.cpu().numpy().tolist()} == {tuple(p) for p in pairs_ref.tolist()}
    L = V.near_layers(X, w, s.offsets)
    coeffs = V.rbf_fit(L, torch.tensor(U, device="cuda"), w, s.offsets, 1.0)
    V.rbf_eval_near(L, coeffs, w, s.offsets, X, pairs, u, 1.0)
    ref = far_ref + near_ref
    err, rms = rel_err(u.cpu().numpy(), ref)
    # interpolation part: conditioning bound of the worst vesicle, relative to max|u|
    kappa = max(np.linalg.cond(NR.kernel_matrix(layers[:, 5 * s.offsets[v]:5 * s.offsets[v + 1]], h[v]))
                for v in set(pairs_ref[:, 1].tolist()))
    tol = bar + 10 * EPS * kappa * np.abs(U).max() * 4 / np.abs(ref).max()
    say(f"near-corrected {prec}: {pairs_ref.shape[0]} near pairs, err {err:.3e} (tol {tol:.1e}), rms {rms:.2e}")
    assert pairs_ref.shape[0] > 50
    assert err <= tol


def test_rbf_full_size_sampled():
    """2000 vesicles of 32 points (the dense near-field workload): every vesicle fitted on the GPU,
    the oracle refits a seeded sample of 24 and the interpolants agree at near-zone points."""
    import torch
    import paper_2606_25569_amd as V
    s = S.rsa_suspension(71, 2000, 32, 0.30, gap=0.02)
    X, f, w = dev_inputs(s)
    L = V.near_layers(X, w, s.offsets)
    layers = L.cpu().numpy()
    U = S.smooth_field(72, layers)
    coeffs = V.rbf_fit(L, torch.tensor(U, device="cuda"), w, s.offsets, 1.0).cpu().numpy()
    rng = np.random.default_rng(73)
    worst = 0.0
    for v in rng.choice(2000, 24, replace=False):
        a, b = 5 * s.offsets[v], 5 * s.offsets[v + 1]
        h = s.w[s.offsets[v]:s.offsets[v + 1]].mean()
        nodes = layers[:, a:b]
        c_ref = NR.vesicle_fit(nodes, U[:, a:b], h)
        Q = nodes[:, rng.integers(0, b - a, 16)] + rng.uniform(-0.5, 0.5, (2, 16)) * h
        err = np.abs(NR.vesicle_eval(nodes, coeffs[:, a:b], Q, h) - NR.vesicle_eval(nodes, c_ref, Q, h)).max()
        tol = 10 * EPS * np.linalg.cond(NR.kernel_matrix(nodes, h)) * np.abs(U[:, a:b]).max()
        worst = max(worst, err / tol)
        assert err <= tol, (v, err, tol)
    say(f"rbf 2000x32 sampled: worst err/tol {worst:.2e}")


def test_near_field_chain_graph_replay():
    """Layers, fit and interpolation launch kernels only: captured in one HIP graph, every replay
    (with eager work in between) equals the eager chain bit for bit."""
    import torch
    import paper_2606_25569_amd as V
    from paper_2606_25569_amd import _lib as L
    from paper_2606_25569_amd.farfield import _ptr
    s = S.rsa_suspension(81, 60, 32, 0.35, gap=0.02)
    X, f, w = dev_inputs(s)
    part = V.Partition(s.offsets, "cuda")
    P, M = s.n_points, s.n_vesicles
    u, pairs = V.farfield_nearmasked(X, X, f, w, part, s.mu, "fp64")
    assert pairs.shape[0] > 0
    pairs = pairs.contiguous()
    layers = V.near_layers(X, w, part)
    vel = torch.tensor(S.smooth_field(82, layers.cpu().numpy()), device="cuda")
    lib = L.lib()
    rws = torch.empty(lib.vesnet_rbf_workspace_bytes(32, M), dtype=torch.uint8, device="cuda")
    lay = torch.empty_like(layers)
    coeffs = torch.empty_like(layers)
    out = torch.empty_like(u)
    cnt = torch.tensor([pairs.shape[0]], dtype=torch.int32, device="cuda")

    def chain(stream):
        sp = stream.cuda_stream
        out.copy_(u)
        L.check(lib.vesnet_near_layers(_ptr(X), _ptr(w), _ptr(part.device), M, P, _ptr(lay), sp))
        L.check(lib.vesnet_rbf_fit(_ptr(lay), _ptr(vel), _ptr(w), _ptr(part.device), M, P, 32, 1.0, _ptr(coeffs),
                                   _ptr(rws), rws.numel(), sp))
        L.check(lib.vesnet_rbf_eval_near(_ptr(lay), _ptr(coeffs), _ptr(w), _ptr(part.device), M, P, 1.0, _ptr(X), P,
                                         _ptr(pairs), _ptr(cnt), pairs.shape[0], _ptr(out), sp))

    chain(torch.cuda.current_stream())
    torch.cuda.synchronize()
    eager = out.clone()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        chain(st)
        with torch.cuda.graph(g, stream=st):
            chain(st)
    torch.cuda.current_stream().wait_stream(st)
    # a target near several vesicles adds their interpolants in atomic order: compare to rounding
    scale = float(eager.abs().max())
    for k in range(3):
        out.fill_(float(k) + 3.0)
        V.farfield_forward(X, X, f, w, part, s.mu, "fp64")  # unrelated eager work in between
        g.replay()
        torch.cuda.synchronize()
        err = float((out - eager).abs().max()) / scale
        assert err <= 1e-14, (k, err)
    say("near-field chain: 3 graph replays equal the eager chain")


def test_rbf_fit_small_workspace_is_bit_identical():
    """With fewer slots than vesicles each wavefront factors several vesicles in turn, reusing its slot
    and LDS: one and three slots give the coefficients of the full workspace bit for bit."""
    import torch
    from paper_2606_25569_amd import _lib as L
    sizes = [3, 7, 0, 32, 33, 64, 100, 128, 200]
    X, w, off, layers, h, U, Ld, wd, full = _fit_case(sizes, 41, 1.0)
    lib = L.lib()
    M, P = len(sizes), int(off[-1])
    part = torch.tensor(off, dtype=torch.int32, device="cuda")
    Ud = torch.tensor(U, device="cuda")
    slot = lib.vesnet_rbf_workspace_bytes(200, 1)
    for slots in (1, 3):
        ws = torch.empty(slot * slots, dtype=torch.uint8, device="cuda")
        got = torch.full_like(full, float("nan"))
        L.check(lib.vesnet_rbf_fit(Ld.data_ptr(), Ud.data_ptr(), wd.data_ptr(), part.data_ptr(), M, P, 200, 1.0,
                                   got.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert torch.equal(got, full), slots
    say("rbf fit: 1 and 3 slots equal the full workspace bit for bit")
