"""PyTorch front end of the far-field Stokeslet library.

Torch provides device memory and the current HIP stream; every operation on
the path runs in the gfx950 kernels behind libvesnet.so (include/vesnet.h).

Tensors: points, force densities and outputs are float64 (2, P) contiguous
(planar: row 0 = x, row 1 = y); arc weights float64 (P,); vesicle offsets
int32 (M+1,) on the device.  The sum computed is eq. (single_layer) with the
Stokeslet of eq. (Stokeslet) read as -ln|r| I + r r^T/|r|^2, trapezoid rule
(Section 2.2.1), own vesicle excluded (U_far of eq. (membrane_velocity)).
"""
from __future__ import annotations

import ctypes
import json
import os
import tempfile

import numpy as np
import torch

from . import _lib as L

_P = ctypes.c_void_p


def _ptr(t):
    return _P(t.data_ptr()) if t is not None else _P(0)


def _stream():
    return _P(torch.cuda.current_stream().cuda_stream)


def _check_vec(name, t, P):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.shape != (2, P) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape (2, {P}), got {tuple(t.shape)}")


def _check_w(t, P):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("arc_weights must be a float64 CUDA tensor")
    if t.shape != (P,) or not t.is_contiguous():
        raise ValueError(f"arc_weights must be contiguous with shape ({P},)")


class Partition:
    """Vesicle partition: host copy (validated once) and device int32 offsets."""

    def __init__(self, offsets, device=None):
        host = np.ascontiguousarray(np.asarray(offsets.cpu() if isinstance(offsets, torch.Tensor) else offsets,
                                               dtype=np.int32))
        if host.ndim != 1 or host.size < 1:
            raise ValueError("offsets must be a 1-D array of length M+1 >= 1")
        self.host = host
        self.n_vesicles = int(host.size - 1)
        self.n_points = int(host[-1])
        L.check(L.lib().vesnet_check_offsets(host.ctypes.data_as(_P), self.n_vesicles, self.n_points))
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = torch.from_numpy(host).to(dev)

    def sizes(self):
        return np.diff(self.host.astype(np.int64))


def as_partition(offsets) -> Partition:
    return offsets if isinstance(offsets, Partition) else Partition(offsets)


def default_config(P, M, precision):
    cfg = L.TileConfig()
    L.check(L.lib().vesnet_default_tile_config(P, M, L.precision_code(precision), ctypes.byref(cfg)))
    return cfg


def _cfg_arg(config):
    if config is None:
        return None
    if isinstance(config, dict):
        config = L.TileConfig.from_dict(config)
    return ctypes.byref(config)


def _cfg_struct(config):
    if config is None:
        return None
    return L.TileConfig.from_dict(config) if isinstance(config, dict) else config


def workspace_bytes(P, M, precision, config=None):
    return int(L.lib().vesnet_farfield_workspace_bytes(P, M, L.precision_code(precision), _cfg_arg(config)))


def _workspace(nbytes, device):
    return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


# ----------------------------------------------------------------------------- forward

def farfield_forward(targets, sources, force_density, arc_weights, partition, mu, precision="fp32c", config=None,
                     out=None, workspace=None):
    """Forward sum without autograd; returns out (2, P) float64."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    for n, t in (("targets", targets), ("sources", sources), ("force_density", force_density)):
        _check_vec(n, t, P)
    _check_w(arc_weights, P)
    prec = L.precision_code(precision)
    if out is None:
        out = torch.empty((2, P), dtype=torch.float64, device=targets.device)
    need = workspace_bytes(P, M, prec, config)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, targets.device)
    L.check(L.lib().vesnet_farfield_stokeslet(
        _ptr(targets), _ptr(sources), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P, float(mu),
        _ptr(out), prec, _cfg_arg(config), _ptr(workspace), workspace.numel(), _stream()))
    return out


def farfield_nearmasked(targets, sources, force_density, arc_weights, partition, mu, precision="fp32c",
                        config=None, capacity=None):
    """Far field with near-field vesicles masked out, and the near pairs.

    A vesicle v is near target i when min_j |x_i - y_j| <= sum_j w_j / N_v (its mean
    arclength spacing).  Returns (out (2, P), pairs (n, 2) int32 device tensor of
    (target, vesicle), unordered).  The list is re-run with a larger capacity when
    the first pass overflows (one host synchronisation)."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    for n, t in (("targets", targets), ("sources", sources), ("force_density", force_density)):
        _check_vec(n, t, P)
    _check_w(arc_weights, P)
    prec = L.precision_code(precision)
    dev = targets.device
    out = torch.empty((2, P), dtype=torch.float64, device=dev)
    cap = int(capacity) if capacity is not None else max(1024, 4 * P)
    ws = _workspace(workspace_bytes(P, M, prec, config), dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    while True:
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        L.check(L.lib().vesnet_farfield_stokeslet_nearmasked(
            _ptr(targets), _ptr(sources), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P,
            float(mu), _ptr(out), _ptr(pairs), cap, _ptr(count), prec, _cfg_arg(config), _ptr(ws), ws.numel(),
            _stream()))
        n = int(count.item())
        if n <= cap:
            return out, pairs[:n]
        cap = n


def elastic_force(X, partition, kappa_b=1.0, sigma=None):
    """Membrane force density f = -kappa_b X_ssss + (sigma X_s)_s and trapezoid weights
    w = |X_alpha| 2 pi / N (spectral derivatives, float64): returns (f (2, P), w (P,))."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("X", X, P)
    if sigma is not None:
        _check_w(sigma, P)
    f = torch.empty((2, P), dtype=torch.float64, device=X.device)
    w = torch.empty((P,), dtype=torch.float64, device=X.device)
    L.check(L.lib().vesnet_elastic_force(_ptr(X), _ptr(sigma), float(kappa_b), _ptr(part.device), M, P, _ptr(f),
                                         _ptr(w), _stream()))
    return f, w


def farfield_treecode(X, force_density, arc_weights, partition, mu, order=30, depth=None, out=None,
                      workspace=None):
    """Treecode far field of the points X on themselves (own vesicle excluded): expansions of
    the given order over a uniform quadtree (default depth: leaves of about 64 points)."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("X", X, P)
    _check_vec("force_density", force_density, P)
    _check_w(arc_weights, P)
    lib = L.lib()
    depth = int(lib.vesnet_treecode_default_depth(P)) if depth is None else int(depth)
    if out is None:
        out = torch.empty((2, P), dtype=torch.float64, device=X.device)
    if workspace is None:
        workspace = _workspace(lib.vesnet_treecode_workspace_bytes(P, depth, int(order)), X.device)
    L.check(lib.vesnet_farfield_treecode(_ptr(X), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P,
                                         float(mu), int(order), depth, _ptr(out), _ptr(workspace), workspace.numel(),
                                         _stream()))
    return out


def farfield_fmm(X, force_density, arc_weights, partition, mu, order=30, depth=None, out=None, workspace=None):
    """Fast multipole far field of the points X on themselves (own vesicle excluded), on the
    treecode's tree: local expansions of the given order (default depth: vesnet_fmm_default_depth)."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("X", X, P)
    _check_vec("force_density", force_density, P)
    _check_w(arc_weights, P)
    lib = L.lib()
    depth = int(lib.vesnet_fmm_default_depth(P, int(order))) if depth is None else int(depth)
    if out is None:
        out = torch.empty((2, P), dtype=torch.float64, device=X.device)
    if workspace is None:
        workspace = _workspace(lib.vesnet_fmm_workspace_bytes(P, depth, int(order)), X.device)
    L.check(lib.vesnet_farfield_fmm(_ptr(X), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P,
                                    float(mu), int(order), depth, _ptr(out), _ptr(workspace), workspace.numel(),
                                    _stream()))
    return out


def farfield_fmm_nearmasked(X, force_density, arc_weights, partition, mu, order=30, depth=None, capacity=None):
    """Fast multipole far field with the near-field masking of Algorithm 4, and the near pairs.

    Returns (out (2, P), pairs (n, 2) int32 device tensor of (target, vesicle), unordered).  The
    list is re-run with a larger capacity when the first pass overflows (one host
    synchronisation).  Raises when the masking could not be completed (a target with more than 16
    near vesicles, or a spacing h_v above the leaf width: pass a smaller depth)."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("X", X, P)
    _check_vec("force_density", force_density, P)
    _check_w(arc_weights, P)
    lib = L.lib()
    depth = int(lib.vesnet_fmm_default_depth(P, int(order))) if depth is None else int(depth)
    dev = X.device
    out = torch.empty((2, P), dtype=torch.float64, device=dev)
    cap = int(capacity) if capacity is not None else max(1024, 4 * P)
    ws = _workspace(lib.vesnet_fmm_nearmasked_workspace_bytes(P, M, depth, int(order)), dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    while True:
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        L.check(lib.vesnet_farfield_fmm_nearmasked(_ptr(X), _ptr(force_density), _ptr(arc_weights), _ptr(part.device),
                                                   M, P, float(mu), int(order), depth, _ptr(out), _ptr(pairs), cap,
                                                   _ptr(count), _ptr(ws), ws.numel(), _stream()))
        n = int(count.item())
        if n == -1:
            raise L.VesnetError(L.ERR_UNSUPPORTED, "a target has more than 16 near vesicles")
        if n == -2:
            raise L.VesnetError(L.ERR_UNSUPPORTED, f"a vesicle's arclength spacing exceeds the leaf width at depth {depth}")
        if n <= cap:
            return out, pairs[:n]
        cap = n


def near_layers(X, arc_weights, partition):
    """CreateNearLayers (Section 3.3): the five layers of every vesicle, membrane points moved along
    the outward normal by (-h, -h/2, 0, h/2, h) h_v; returns (2, 5P) with vesicle v's 5 N_v nodes at
    5 offsets[v] + l N_v + k."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("X", X, P)
    _check_w(arc_weights, P)
    layers = torch.empty((2, 5 * P), dtype=torch.float64, device=X.device)
    L.check(L.lib().vesnet_near_layers(_ptr(X), _ptr(arc_weights), _ptr(part.device), M, P, _ptr(layers), _stream()))
    return layers


def _check_layers(name, t, P):
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (2, 5 * P):
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape (2, {5 * P})")


def rbf_fit(layers, layer_velocity, arc_weights, partition, width=1.0, max_points=None):
    """Gaussian RBF coefficients of every vesicle's layer velocities (batched Cholesky, float64).
    The Gaussian of vesicle v is exp(-r^2 / (width h_v)^2); returns (2, 5P)."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_layers("layers", layers, P)
    _check_layers("layer_velocity", layer_velocity, P)
    _check_w(arc_weights, P)
    nmax = int(part.sizes().max()) if max_points is None and M > 0 else int(max_points or 1)
    coeffs = torch.empty_like(layer_velocity)
    if P == 0:
        return coeffs
    ws = _workspace(L.lib().vesnet_rbf_workspace_bytes(nmax, M), layers.device)
    L.check(L.lib().vesnet_rbf_fit(_ptr(layers), _ptr(layer_velocity), _ptr(arc_weights), _ptr(part.device), M, P,
                                   nmax, float(width), _ptr(coeffs), _ptr(ws), ws.numel(), _stream()))
    return coeffs


def rbf_eval_near(layers, coeffs, arc_weights, partition, targets, near_pairs, out, width=1.0, near_count=None):
    """interpolateInNearField (Algorithm 4): out[:, i] += s_v(targets[:, i]) for every near pair
    (i, v) in near_pairs (int32 (capacity, 2)).  near_count, a device int32 tensor of one element,
    limits the pairs read; by default all rows of near_pairs are used."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_layers("layers", layers, P)
    _check_layers("coeffs", coeffs, P)
    _check_w(arc_weights, P)
    nt = targets.shape[1]
    _check_vec("targets", targets, nt)
    _check_vec("out", out, nt)
    if near_pairs.dtype != torch.int32 or not near_pairs.is_contiguous():
        raise ValueError("near_pairs must be a contiguous int32 tensor")
    cap = near_pairs.numel() // 2
    if near_count is None:
        near_count = torch.full((1,), cap, dtype=torch.int32, device=out.device)
    L.check(L.lib().vesnet_rbf_eval_near(_ptr(layers), _ptr(coeffs), _ptr(arc_weights), _ptr(part.device), M, P,
                                         float(width), _ptr(targets), nt, _ptr(near_pairs), _ptr(near_count), cap,
                                         _ptr(out), _stream()))
    return out


def farfield_backward(targets, sources, force_density, arc_weights, partition, mu, grad_out, precision="fp32c",
                      need=(True, True, True, True)):
    """Reverse mode: returns (grad_targets, grad_sources, grad_force, grad_weights), None where not needed."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("grad_out", grad_out, P)
    prec = L.precision_code(precision)
    dev = targets.device
    gt = torch.empty((2, P), dtype=torch.float64, device=dev) if need[0] else None
    gs = torch.empty((2, P), dtype=torch.float64, device=dev) if need[1] else None
    gf = torch.empty((2, P), dtype=torch.float64, device=dev) if need[2] else None
    gw = torch.empty((P,), dtype=torch.float64, device=dev) if need[3] else None
    ws = _workspace(L.lib().vesnet_backward_workspace_bytes(P, M, prec), dev)
    L.check(L.lib().vesnet_farfield_stokeslet_backward(
        _ptr(targets), _ptr(sources), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P, float(mu),
        _ptr(grad_out), _ptr(gt), _ptr(gs), _ptr(gf), _ptr(gw), prec, _ptr(ws), ws.numel(), _stream()))
    return gt, gs, gf, gw


def farfield_backward_points(points, force_density, arc_weights, partition, mu, grad_out, precision="fp32c",
                             need=(True, True, True)):
    """Reverse mode for one point array used as targets and sources: returns (grad_points,
    grad_force, grad_weights), None where not needed.  grad_points holds both roles of each point."""
    part = as_partition(partition)
    P, M = part.n_points, part.n_vesicles
    _check_vec("grad_out", grad_out, P)
    prec = L.precision_code(precision)
    dev = points.device
    gx = torch.empty((2, P), dtype=torch.float64, device=dev) if need[0] else None
    gf = torch.empty((2, P), dtype=torch.float64, device=dev) if need[1] else None
    gw = torch.empty((P,), dtype=torch.float64, device=dev) if need[2] else None
    ws = _workspace(L.lib().vesnet_backward_points_workspace_bytes(P, M, prec), dev)
    L.check(L.lib().vesnet_farfield_stokeslet_backward_points(
        _ptr(points), _ptr(force_density), _ptr(arc_weights), _ptr(part.device), M, P, float(mu), _ptr(grad_out),
        _ptr(gx), _ptr(gf), _ptr(gw), prec, _ptr(ws), ws.numel(), _stream()))
    return gx, gf, gw


class _FarField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, targets, sources, force_density, arc_weights, part, mu, precision, config, same=False):
        out = farfield_forward(targets, sources, force_density, arc_weights, part, mu, precision, config)
        ctx.save_for_backward(targets, sources, force_density, arc_weights)
        ctx.part, ctx.mu = part, mu
        ctx.precision = L.precision_code(precision)
        ctx.same = same
        return out

    @staticmethod
    def backward(ctx, grad_out):
        targets, sources, f, w = ctx.saved_tensors
        need = ctx.needs_input_grad[:4]
        if not any(need):
            return (None,) * 9
        if ctx.precision == L.FP32_NAIVE:
            raise L.VesnetError(L.ERR_UNSUPPORTED, "the naive float32 control has no backward; use 'fp32c' or 'fp64'")
        g = grad_out.contiguous()
        if ctx.same and need[0] and need[1]:
            # one tensor in both roles: its gradient is the sum of the two, computed in one pass
            gx, gf, gw = farfield_backward_points(targets, f, w, ctx.part, ctx.mu, g, ctx.precision,
                                                  (True, need[2], need[3]))
            return gx, None, gf, gw, None, None, None, None, None
        gt, gs, gf, gw = farfield_backward(targets, sources, f, w, ctx.part, ctx.mu, g, ctx.precision, need)
        return gt, gs, gf, gw, None, None, None, None, None


def farfield_stokeslet(targets, sources, force_density, arc_weights, vesicle_offsets, mu=1.0, precision="fp32c",
                       config=None):
    """u_far at every target: (2, P) float64, differentiable in targets, sources,
    force_density and arc_weights (the backward runs the hand-written adjoint
    kernels; the naive float32 form has no backward)."""
    part = as_partition(vesicle_offsets)
    return _FarField.apply(targets, sources, force_density, arc_weights, part, float(mu), precision, config,
                           targets is sources)


# ----------------------------------------------------------------------------- batched

class BatchedProblem:
    """S independent suspensions concatenated; owns device tables and the workspace."""

    def __init__(self, targets, sources, force_density, arc_weights, vesicle_offsets, suspension_offsets, mu,
                 precision="fp32c", config=None):
        part = as_partition(vesicle_offsets)
        P, M = part.n_points, part.n_vesicles
        for n, t in (("targets", targets), ("sources", sources), ("force_density", force_density)):
            _check_vec(n, t, P)
        _check_w(arc_weights, P)
        soff = np.ascontiguousarray(np.asarray(suspension_offsets, dtype=np.int32))
        S = int(soff.size - 1)
        if S < 1 or soff[0] != 0 or soff[-1] != M or np.any(np.diff(soff) < 0):
            raise ValueError("suspension_offsets must run from 0 to n_vesicles, non-decreasing")
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (S,)))
        if not np.all(np.isfinite(mu) & (mu > 0)):
            raise ValueError("every mu must be finite and > 0")
        dev = targets.device
        self.targets, self.sources, self.f, self.w = targets, sources, force_density, arc_weights
        self.part = part
        self.sus_off = torch.from_numpy(soff).to(dev)
        self.mu = torch.from_numpy(mu.copy()).to(dev)
        self.S, self.P, self.M = S, P, M
        self.prec = L.precision_code(precision)
        self.config = _cfg_struct(config)
        self.out = torch.empty((2, P), dtype=torch.float64, device=dev)
        self.ws = _workspace(L.lib().vesnet_batched_workspace_bytes(P, M, S, self.prec), dev)
        self._graph = None

    def _args(self):
        return (_ptr(self.targets), _ptr(self.sources), _ptr(self.f), _ptr(self.w), _ptr(self.part.device), self.M,
                self.P, _ptr(self.sus_off), self.S, _ptr(self.mu), _ptr(self.out), self.prec,
                ctypes.byref(self.config) if self.config is not None else None, _ptr(self.ws), self.ws.numel())

    def run(self):
        """One persistent launch on the current stream; returns out (2, P)."""
        L.check(L.lib().vesnet_farfield_stokeslet_batched(*self._args(), _stream()))
        return self.out

    def capture(self):
        """Capture the batched call into a HIP graph (once)."""
        if self._graph is None:
            h = _P()
            L.check(L.lib().vesnet_graph_create_batched(*self._args(), ctypes.byref(h)))
            self._graph = h
        return self

    def replay(self):
        if self._graph is None:
            self.capture()
        L.check(L.lib().vesnet_graph_launch(self._graph, _stream()))
        return self.out

    def close(self):
        if self._graph is not None:
            L.lib().vesnet_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- autotuning

def _tune_cache_path():
    return os.environ.get("VESNET_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "vesnet_tune.json"))


def _bucket(x):
    return int(2 ** round(np.log2(max(1, x))))


def tune_key(P, M, precision, batched):
    prop = torch.cuda.get_device_properties(torch.cuda.current_device())
    n_mean = P / max(1, M)
    return f"{prop.name}|{getattr(prop, 'gcnArchName', '')}|p{L.precision_code(precision)}|b{int(bool(batched))}|" \
           f"N{_bucket(n_mean)}|P{_bucket(P)}"


def load_tuned(P, M, precision, batched=False):
    path = _tune_cache_path()
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(tune_key(P, M, precision, batched))
    return L.TileConfig.from_dict(e["config"]) if e else None


def _store_tuned(key, cfg, ms):
    path = _tune_cache_path()
    d = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                d = json.load(fh)
        except (OSError, ValueError):
            d = {}
    d[key] = {"config": cfg.as_dict(), "ms": ms}
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(targets, sources, force_density, arc_weights, vesicle_offsets, mu=1.0, precision="fp32c", repeats=3,
             batched: BatchedProblem | None = None, store=True):
    """Time every launch shape (host-synchronous) and cache the fastest in a JSON file.

    For the batched form pass a BatchedProblem (its tensors are used)."""
    lib = L.lib()
    best = L.TileConfig()
    ms = ctypes.c_float()
    if batched is not None:
        b = batched
        L.check(lib.vesnet_autotune(_ptr(b.targets), _ptr(b.sources), _ptr(b.f), _ptr(b.w), _ptr(b.part.device), b.M,
                                    b.P, 1, _ptr(b.sus_off), b.S, _ptr(b.mu), 1.0, _ptr(b.out), b.prec, repeats,
                                    _ptr(b.ws), b.ws.numel(), _stream(), ctypes.byref(best), ctypes.byref(ms)))
        key = tune_key(b.P, b.M, b.prec, True)
    else:
        part = as_partition(vesicle_offsets)
        P, M = part.n_points, part.n_vesicles
        for n, t in (("targets", targets), ("sources", sources), ("force_density", force_density)):
            _check_vec(n, t, P)
        _check_w(arc_weights, P)
        prec = L.precision_code(precision)
        big = L.TileConfig(1, 64, 16, 1)
        ws = _workspace(L.lib().vesnet_farfield_workspace_bytes(P, M, prec, ctypes.byref(big)), targets.device)
        out = torch.empty((2, P), dtype=torch.float64, device=targets.device)
        L.check(lib.vesnet_autotune(_ptr(targets), _ptr(sources), _ptr(force_density), _ptr(arc_weights),
                                    _ptr(part.device), M, P, 0, None, 0, None, float(mu), _ptr(out), prec, repeats,
                                    _ptr(ws), ws.numel(), _stream(), ctypes.byref(best), ctypes.byref(ms)))
        key = tune_key(P, M, prec, False)
    if store:
        _store_tuned(key, best, float(ms.value))
    return best, float(ms.value)
