"""GPU test of vesnet_farfield_stokeslet_noalloc (the entry point whose workspace is the library's
own device array) against vesnet_farfield_stokeslet, through the C-ABI: two calls in a row, the
second on a smaller problem, in every precision.  Bars: float64 <= 1e-12, float32 forms <= 1e-5
(max-norm difference relative to max |u|), the oracle's bars."""
import ctypes

import numpy as np
import pytest

from synth import suspension as S
from tests.gpu_util import dev_inputs, rel_err, say

pytestmark = pytest.mark.gpu

BARS = {"fp64": 1e-12, "fp32c": 1e-5, "fp32": 1e-5}


def _noalloc(V, X, T, f, w, part, mu, prec, cfg=None):
    import torch
    lib = V._lib.lib()
    P, M = part.n_points, part.n_vesicles
    out = torch.full((2, P), float("nan"), dtype=torch.float64, device="cuda")
    p = V.farfield._ptr
    c = ctypes.byref(V.TileConfig.from_dict(cfg)) if cfg else None
    V._lib.check(lib.vesnet_farfield_stokeslet_noalloc(p(T), p(X), p(f), p(w), p(part.device), M, P, float(mu),
                                                        p(out), V._lib.precision_code(prec), c,
                                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_workspace_entry_two_calls():
    import torch
    import paper_2606_25569_amd as V
    for s in (S.load_config(4), S.make_config(0)):   # 512 x 64, then the smaller 16 x 32
        X, f, w = dev_inputs(s)
        part = V.Partition(s.offsets, X.device)
        for prec in ("fp32c", "fp64", "fp32"):
            ref = V.farfield_forward(X, X, f, w, part, s.mu, precision=prec)
            torch.cuda.synchronize()
            ref = ref.cpu().numpy()
            got = _noalloc(V, X, X, f, w, part, s.mu, prec)
            err, _ = rel_err(got, ref)
            say(f"noalloc P={s.n_points} {prec}: {err:.3e}")
            assert np.isfinite(got).all() and err <= BARS[prec], (prec, err)
        # separate target array (the direct form) and the forced symmetric form
        T = X + 1e-3
        ref = V.farfield_forward(T, X, f, w, part, s.mu, precision="fp32c").cpu().numpy()
        err, _ = rel_err(_noalloc(V, X, T, f, w, part, s.mu, "fp32c"), ref)
        say(f"noalloc P={s.n_points} separate targets: {err:.3e}")
        assert err <= BARS["fp32c"]
        for prec in ("fp32c", "fp64"):  # the symmetric forms add fixed-point integers: equal bit for bit
            cfg = {"pair_form": 2, "targets_per_thread": 1}
            ref = V.farfield_forward(X, X, f, w, part, s.mu, precision=prec, config=cfg).cpu().numpy()
            got = _noalloc(V, X, X, f, w, part, s.mu, prec, cfg)
            say(f"noalloc P={s.n_points} symmetric {prec}: bitwise {np.array_equal(got, ref)}")
            assert np.array_equal(got, ref)
