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
