"""Shared helpers for the GPU parity tests (inputs to device, error norms)."""
import sys

import numpy as np


def rel_err(a, ref):
    """Component-wise max-norm error relative to max |ref| (and the RMS ratio)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = float(np.max(np.abs(ref)))
    d = a - ref
    return float(np.max(np.abs(d)) / scale), float(np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(ref * ref)))


def dev_inputs(s, device="cuda"):
    import torch
    X = torch.tensor(s.X, dtype=torch.float64, device=device)
    f = torch.tensor(s.f, dtype=torch.float64, device=device)
    w = torch.tensor(s.w, dtype=torch.float64, device=device)
    return X, f, w


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def near_margin(s):
    """Smallest |d_iv - h_v| / h_v over all (target, other vesicle) of a suspension: near-field
    decisions closer than float32 rounding may legitimately differ between the GPU and the
    oracle, so test inputs must stay clear of it."""
    from oracle import oracle as O
    vid = O.vesicle_ids(s.offsets)
    worst = np.inf
    for v in range(s.n_vesicles):
        a, b = s.offsets[v], s.offsets[v + 1]
        if b == a:
            continue
        h = s.w[a:b].sum() / (b - a)
        d = np.sqrt(((s.X[:, :, None] - s.X[:, None, a:b]) ** 2).sum(axis=0)).min(axis=1)
        m = np.abs(d - h)[vid != v] / h
        worst = min(worst, float(m.min()))
    return worst
