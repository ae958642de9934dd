"""CPU tests of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments on the host before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2606_25569_amd import _lib
    return _lib


def _declared():
    txt = open(os.path.join(ROOT, "include", "vesnet.h")).read()
    return sorted(set(re.findall(r"VESNET_API\s+[\w\s\*]+?\b(vesnet_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    names = _declared()
    assert len(names) == 33, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_only_c_symbols_exported(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True, check=True).stdout
    funcs = [ln.split()[-1] for ln in out.splitlines() if " T " in ln]
    assert funcs and all(f.startswith("vesnet_") for f in funcs), funcs


def test_version(L):
    assert b"gfx950" in L.lib().vesnet_version()


def _offs(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def test_check_offsets(L):
    lib = L.lib()
    a, p = _offs([0, 3, 3, 7])
    assert lib.vesnet_check_offsets(p, 3, 7) == 0
    for bad, M, P in (([1, 3, 7], 2, 7), ([0, 5, 3], 2, 3), ([0, 3, 6], 2, 7)):
        a, p = _offs(bad)
        assert lib.vesnet_check_offsets(p, M, P) == L.ERR_INVALID_ARGUMENT
        assert lib.vesnet_last_error()
    assert lib.vesnet_check_offsets(None, 1, 1) == L.ERR_INVALID_ARGUMENT
    assert lib.vesnet_check_offsets(p, -1, 3) == L.ERR_INVALID_ARGUMENT
    a, p = _offs([0])
    assert lib.vesnet_check_offsets(p, 0, 0) == 0
    assert lib.vesnet_check_offsets(p, 0, 5) == L.ERR_INVALID_ARGUMENT


def test_default_config_and_workspace_sizes(L):
    lib = L.lib()
    cfg = L.TileConfig()
    assert lib.vesnet_default_tile_config(256000, 2000, 1, ctypes.byref(cfg)) == 0
    d = cfg.as_dict()
    assert d["targets_per_thread"] in (1, 2, 4) and d["block_threads"] in (64, 128, 256) and d["source_splits"] >= 1
    n1 = lib.vesnet_farfield_workspace_bytes(256000, 2000, 1, ctypes.byref(L.TileConfig(2, 256, 1, 1)))
    n4 = lib.vesnet_farfield_workspace_bytes(256000, 2000, 1, ctypes.byref(L.TileConfig(2, 256, 4, 1)))
    n64 = lib.vesnet_farfield_workspace_bytes(256000, 2000, 0, ctypes.byref(L.TileConfig(2, 256, 1, 1)))
    direct = L.TileConfig(2, 256, 1, 1)
    direct.pair_form = 1
    n1d = lib.vesnet_farfield_workspace_bytes(256000, 2000, 1, ctypes.byref(direct))
    sym4 = L.TileConfig(2, 256, 4, 1)
    sym4.pair_form = 2
    ns4 = lib.vesnet_farfield_workspace_bytes(256000, 2000, 1, ctypes.byref(sym4))
    assert n1d >= 256000 * (16 + 16 + 4) + 2000 * 56   # records, float64 forces, ids; vesicle tables
    assert n4 - n1 >= 2 * 4 * 256000 * 8                # split partials of the direct form
    assert n1 - n1d >= 256000 * 16 + 16000 * 32         # symmetric form: fixed-point sums, cycle table
    assert ns4 < n4                                     # the symmetric form needs no split partials
    assert n64 >= 256000 * (32 + 4) + 2000 * 40
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 7, None) == 0          # bad precision
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 1, ctypes.byref(L.TileConfig(3, 256, 1, 1))) == 0
    assert lib.vesnet_backward_workspace_bytes(10, 2, 2) == 0                # naive has no backward
    assert lib.vesnet_batched_workspace_bytes(100, 10, 3, 1) > 0


FAKE = 0x10000  # never dereferenced: every call below fails validation first


def _p(x):
    return ctypes.c_void_p(x)


def _fwd(L, **kw):
    a = dict(targets=FAKE, sources=FAKE + 0x100000, f=FAKE + 0x200000, w=FAKE + 0x300000, off=FAKE + 0x400000,
             M=2, P=10, mu=1.0, out=FAKE + 0x500000, prec=1, cfg=None, ws=FAKE + 0x600000, wsb=1 << 30)
    a.update(kw)
    return L.lib().vesnet_farfield_stokeslet(_p(a["targets"]), _p(a["sources"]), _p(a["f"]), _p(a["w"]), _p(a["off"]),
                                             a["M"], a["P"], a["mu"], _p(a["out"]), a["prec"], a["cfg"], _p(a["ws"]),
                                             a["wsb"], None)


@pytest.mark.parametrize("kw,code", [
    ({"targets": 0}, -1), ({"sources": 0}, -1), ({"f": 0}, -1), ({"w": 0}, -1), ({"off": 0}, -1), ({"out": 0}, -1),
    ({"mu": 0.0}, -1), ({"mu": -1.0}, -1), ({"mu": float("nan")}, -1), ({"mu": float("inf")}, -1),
    ({"prec": 9}, -1), ({"P": -1}, -1), ({"M": -2}, -1), ({"M": 0}, -1), ({"P": (1 << 30) + 1}, -1),
    ({"ws": 0}, -3), ({"wsb": 16}, -3),
    ({"out": FAKE}, -1), ({"out": FAKE + 0x100000 + 8}, -1), ({"out": FAKE + 0x600000 + 64}, -1),
])
def test_forward_rejects_bad_arguments(L, kw, code):
    assert _fwd(L, **kw) == code
    assert len(L.lib().vesnet_last_error()) > 0


def test_bad_tile_configs_rejected(L):
    for cfg in (L.TileConfig(3, 256, 1, 1), L.TileConfig(1, 96, 1, 1), L.TileConfig(1, 64, 65, 1),
                L.TileConfig(1, 64, -1, 1), L.TileConfig(1, 64, 1, 17), L.TileConfig(1, 64, 1, 1, 3)):
        assert _fwd(L, cfg=ctypes.byref(cfg)) == -1


def test_empty_problem_is_a_no_op(L):
    assert _fwd(L, P=0, M=0, targets=0, sources=0, f=0, w=0, off=0, out=0, ws=0, wsb=0) == 0


def test_backward_rejects(L):
    lib = L.lib()
    args = [_p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000), _p(FAKE + 0x400000), 2, 10, 1.0,
            _p(FAKE + 0x500000)]
    ws = [_p(FAKE + 0x600000), 1 << 30, None]
    # naive precision unsupported
    assert lib.vesnet_farfield_stokeslet_backward(*args, _p(FAKE + 0x700000), None, None, None, 2, *ws) == -2
    # outputs overlapping each other
    assert lib.vesnet_farfield_stokeslet_backward(*args, _p(FAKE + 0x700000), _p(FAKE + 0x700000 + 8), None, None, 1,
                                                  *ws) == -1
    # output overlapping grad_out
    assert lib.vesnet_farfield_stokeslet_backward(*args, _p(FAKE + 0x500000), None, None, None, 1, *ws) == -1
    # missing grad_out
    a2 = list(args)
    a2[8] = None
    assert lib.vesnet_farfield_stokeslet_backward(*a2, _p(FAKE + 0x700000), None, None, None, 1, *ws) == -1
    # workspace too small
    assert lib.vesnet_farfield_stokeslet_backward(*args, _p(FAKE + 0x700000), None, None, None, 1, _p(FAKE + 0x600000),
                                                  8, None) == -3


def test_backward_points_rejects(L):
    lib = L.lib()
    # points, force_density, arc_weights, offsets, M, P, mu, grad_out
    args = [_p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000), 2, 10, 1.0, _p(FAKE + 0x500000)]
    ws = [_p(FAKE + 0x600000), 1 << 30, None]
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, _p(FAKE + 0x700000), None, None, 2, *ws) == -2
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, _p(FAKE + 0x700000), _p(FAKE + 0x700000 + 8), None, 1,
                                                         *ws) == -1
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, _p(FAKE + 0x500000), None, None, 1, *ws) == -1
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, None, None, _p(FAKE + 0x200000), 1, *ws) == -1
    a2 = list(args)
    a2[7] = None
    assert lib.vesnet_farfield_stokeslet_backward_points(*a2, _p(FAKE + 0x700000), None, None, 1, *ws) == -1
    a2 = list(args)
    a2[6] = -1.0
    assert lib.vesnet_farfield_stokeslet_backward_points(*a2, _p(FAKE + 0x700000), None, None, 1, *ws) == -1
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, _p(FAKE + 0x700000), None, None, 1,
                                                         _p(FAKE + 0x600000), 8, None) == -3
    # nothing requested, and the empty problem: no-ops
    assert lib.vesnet_farfield_stokeslet_backward_points(*args, None, None, None, 1, *ws) == 0
    assert lib.vesnet_farfield_stokeslet_backward_points(None, None, None, None, 0, 0, 1.0, None, None, None, None, 1,
                                                         None, 0, None) == 0
    # workspace sizes: the symmetric forms (fp32c and fp64) need less than the gathers plus their sum
    # buffer, and at least two prepared regions, the cycle table, the [2][P] sums and a [2][P] buffer
    for P, M in ((512, 16), (256000, 2000)):
        b32 = lib.vesnet_backward_points_workspace_bytes(P, M, 1)
        b64 = lib.vesnet_backward_points_workspace_bytes(P, M, 0)
        assert 0 < b32 and 0 < b64
        assert b32 < lib.vesnet_backward_workspace_bytes(P, M, 1) + 16 * P
        assert b64 < lib.vesnet_backward_workspace_bytes(P, M, 0) + 16 * P
        assert b64 >= 2 * P * (32 + 16 + 4) + 16 * P + 16 * P
    assert lib.vesnet_backward_points_workspace_bytes(512, 16, 2) == 0


def test_batched_rejects(L):
    lib = L.lib()
    base = [_p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000), _p(FAKE + 0x400000), 2, 10]
    tail = [_p(FAKE + 0x500000), 1, None, _p(FAKE + 0x600000), 1 << 30, None]
    assert lib.vesnet_farfield_stokeslet_batched(*base, None, 1, _p(FAKE + 0x800000), *tail) == -1   # no sus offsets
    assert lib.vesnet_farfield_stokeslet_batched(*base, _p(FAKE + 0x900000), 0, _p(FAKE + 0x800000), *tail) == -1
    assert lib.vesnet_farfield_stokeslet_batched(*base, _p(FAKE + 0x900000), 1, None, *tail) == -1   # no mu
    g = ctypes.c_void_p()
    assert lib.vesnet_graph_create_batched(*base, None, 1, _p(FAKE + 0x800000), *tail[:5], ctypes.byref(g)) == -1
    assert lib.vesnet_graph_launch(None, None) == -1
    assert lib.vesnet_graph_destroy(None) == 0


def test_nearmasked_rejects(L):
    lib = L.lib()
    base = [_p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000), _p(FAKE + 0x400000), 2, 10, 1.0,
            _p(FAKE + 0x500000)]
    ws = [1, None, _p(FAKE + 0x600000), 1 << 30, None]
    assert lib.vesnet_farfield_stokeslet_nearmasked(*base, _p(FAKE + 0x700000), 4, None, *ws) == -1      # no count
    assert lib.vesnet_farfield_stokeslet_nearmasked(*base, None, 4, _p(FAKE + 0x800000), *ws) == -1      # no list
    assert lib.vesnet_farfield_stokeslet_nearmasked(*base, _p(FAKE + 0x700000), -1, _p(FAKE + 0x800000), *ws) == -1
    assert lib.vesnet_farfield_stokeslet_nearmasked(*base, _p(FAKE + 0x500000), 4, _p(FAKE + 0x800000), *ws) == -1


def test_elastic_force_rejects(L):
    lib = L.lib()
    X, off, f, w = _p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000)
    assert lib.vesnet_elastic_force(X, None, float("nan"), off, 2, 10, f, w, None) == -1
    assert lib.vesnet_elastic_force(None, None, 1.0, off, 2, 10, f, w, None) == -1
    assert lib.vesnet_elastic_force(X, None, 1.0, off, 2, 10, None, w, None) == -1
    assert lib.vesnet_elastic_force(X, None, 1.0, off, 2, 10, X, w, None) == -1          # f overlaps X
    assert lib.vesnet_elastic_force(X, None, 1.0, off, 2, 10, f, _p(FAKE + 0x200000 + 8), None) == -1
    assert lib.vesnet_elastic_force(None, None, 1.0, None, 0, 0, None, None, None) == 0


def test_near_layers_and_rbf_reject(L):
    lib = L.lib()
    X, off, w, lay = _p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000)
    vel, co, ws, tg = _p(FAKE + 0x400000), _p(FAKE + 0x500000), _p(FAKE + 0x600000), _p(FAKE + 0x8000000)
    pairs, cnt, out = _p(FAKE + 0x9000000), _p(FAKE + 0x9100000), _p(FAKE + 0x9200000)
    # layers: NULLs, overlap with X (10P doubles from X's start)
    assert lib.vesnet_near_layers(None, w, off, 2, 10, lay, None) == -1
    assert lib.vesnet_near_layers(X, w, off, 2, 10, None, None) == -1
    assert lib.vesnet_near_layers(X, w, off, 2, 10, _p(FAKE + 8), None) == -1
    assert lib.vesnet_near_layers(None, None, None, 0, 0, None, None) == 0
    # workspace query: out-of-range max_points or vesicle count gives 0
    assert lib.vesnet_rbf_workspace_bytes(0, 4) == 0
    assert lib.vesnet_rbf_workspace_bytes(201, 4) == 0
    assert lib.vesnet_rbf_workspace_bytes(32, 0) == 0
    slot = lib.vesnet_rbf_workspace_bytes(32, 1)
    assert slot > 0 and lib.vesnet_rbf_workspace_bytes(32, 4) == 4 * slot
    assert lib.vesnet_rbf_workspace_bytes(32, 100000) == 2048 * slot          # 2048 slots of 160 KB
    big = lib.vesnet_rbf_workspace_bytes(200, 1)
    assert lib.vesnet_rbf_workspace_bytes(200, 100000) == (2 ** 30 // big) * big  # capped at 1 GiB
    fit = lambda **k: lib.vesnet_rbf_fit(k.get("lay", lay), vel, w, off, 2, 10, k.get("nmax", 32),
                                         k.get("width", 1.0), k.get("co", co), k.get("ws", ws),
                                         k.get("wsb", slot), None)
    assert fit(width=0.0) == -1
    assert fit(width=float("inf")) == -1
    assert fit(nmax=201) == -2
    assert fit(lay=None) == -1
    assert fit(wsb=slot - 1) == -3
    assert fit(ws=None) == -3
    assert fit(co=_p(FAKE + 0x400000 + 8)) == -1   # coeffs overlap the velocities
    assert fit(ws=_p(FAKE + 0x500000 + 64)) == -1  # workspace overlaps coeffs
    ev = lambda **k: lib.vesnet_rbf_eval_near(lay, co, w, off, 2, 10, k.get("width", 1.0), tg, k.get("nt", 10),
                                              pairs, cnt, k.get("cap", 16), k.get("out", out), None)
    assert ev(width=-1.0) == -1
    assert ev(cap=-1) == -1
    assert ev(nt=-3) == -1
    assert ev(out=None) == -1
    assert ev(out=_p(FAKE + 0x8000000 + 8)) == -1  # out overlaps the targets
    assert ev(cap=0) == 0 and ev(nt=0) == 0


@pytest.mark.parametrize("method", ["treecode", "fmm"])
def test_tree_methods_reject(L, method):
    """Treecode and fast multipole entry points: workspace queries give 0 out of range, and the
    calls refuse bad orders, depths, viscosities, NULLs, short workspaces and overlaps."""
    lib = L.lib()
    wsq = getattr(lib, f"vesnet_{method}_workspace_bytes")
    run = getattr(lib, f"vesnet_farfield_{method}")
    assert lib.vesnet_treecode_default_depth(0) == 0
    assert lib.vesnet_treecode_default_depth(64) == 0
    assert lib.vesnet_treecode_default_depth(65) == 1
    assert lib.vesnet_treecode_default_depth(256000) == 6
    assert lib.vesnet_fmm_default_depth(256000, 30) == 6 and lib.vesnet_fmm_default_depth(256000, 40) == 6
    assert lib.vesnet_fmm_default_depth(512000, 30) == 7 and lib.vesnet_fmm_default_depth(512000, 40) == 6
    assert lib.vesnet_fmm_default_depth(0, 30) == 0 and lib.vesnet_fmm_default_depth(10 ** 9, 8) == 10
    assert wsq(100, 3, 0) == 0 and wsq(100, 3, 49) == 0 and wsq(100, -1, 8) == 0 and wsq(100, 11, 8) == 0
    assert wsq(-1, 3, 8) == 0
    need = wsq(100, 3, 8)
    assert need > 0
    if method == "fmm":  # the treecode's workspace plus the local expansions and the binomial table
        assert need > lib.vesnet_treecode_workspace_bytes(100, 3, 8)
    X, f, w, off = _p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000)
    out, ws = _p(FAKE + 0x400000), _p(FAKE + 0x1000000)
    call = lambda **k: run(k.get("X", X), f, w, off, 2, 100, k.get("mu", 1.0), k.get("order", 8), k.get("depth", 3),
                           k.get("out", out), k.get("ws", ws), k.get("wsb", need), None)
    assert call(order=0) == -2 and call(order=49) == -2
    assert call(depth=-1) == -2 and call(depth=11) == -2
    assert call(mu=0.0) == -1 and call(mu=float("nan")) == -1
    assert call(X=None) == -1 and call(out=None) == -1
    assert call(wsb=need - 1) == -3 and call(ws=None) == -3
    assert call(out=_p(FAKE + 8)) == -1                      # out overlaps the points
    assert call(ws=_p(FAKE + 0x400000 + 64)) == -1           # workspace overlaps out
    assert run(None, None, None, None, 0, 0, 1.0, 8, 3, None, None, 0, None) == 0  # empty: no-op


def test_fmm_nearmasked_rejects(L):
    lib = L.lib()
    wsq = lib.vesnet_fmm_nearmasked_workspace_bytes
    assert wsq(100, 4, 3, 0) == 0 and wsq(100, 4, 11, 8) == 0 and wsq(-1, 4, 3, 8) == 0
    need = wsq(100, 4, 3, 8)
    assert need > lib.vesnet_fmm_workspace_bytes(100, 3, 8)  # plus h_v^2 and a status word
    X, f, w, off = _p(FAKE), _p(FAKE + 0x100000), _p(FAKE + 0x200000), _p(FAKE + 0x300000)
    out, ws = _p(FAKE + 0x400000), _p(FAKE + 0x1000000)
    pairs, cnt = _p(FAKE + 0x2000000), _p(FAKE + 0x2100000)
    call = lambda **k: lib.vesnet_farfield_fmm_nearmasked(X, f, w, off, 4, 100, 1.0, k.get("order", 8), 3,
                                                          k.get("out", out), k.get("pairs", pairs), k.get("cap", 16),
                                                          k.get("cnt", cnt), ws, k.get("wsb", need), None)
    assert call(order=49) == -2
    assert call(cnt=None) == -1
    assert call(cap=-1) == -1
    assert call(pairs=None) == -1
    assert call(wsb=need - 1) == -3
    assert call(pairs=_p(FAKE + 0x400000 + 16)) == -1  # the list overlaps out
    assert call(cnt=_p(FAKE + 0x2000000 + 8)) == -1    # the count overlaps the list


def test_product_package_has_no_cpu_fallback():
    """The package imports the library eagerly and never imports the oracle."""
    import ast
    pkg = os.path.join(ROOT, "paper_2606_25569_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, fn)).read())
            for node in ast.walk(tree):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                    assert not any(m.split(".")[0] == "oracle" for m in mods), (fn, mods)


def test_naive_precision_has_no_backward(L):
    """The autograd function refuses to differentiate the naive float32 control (it would otherwise
    have to substitute another precision's adjoint); the error is raised before any device call."""
    import torch
    from paper_2606_25569_amd import farfield as F

    class Ctx:
        pass

    ctx = Ctx()
    t = torch.zeros((2, 4), dtype=torch.float64)
    ctx.saved_tensors = (t, t, t, torch.zeros(4, dtype=torch.float64))
    ctx.needs_input_grad = (True, True, True, True, False, False, False, False)
    ctx.part, ctx.mu, ctx.precision = None, 1.0, L.FP32_NAIVE
    with pytest.raises(L.VesnetError) as e:
        F._FarField.backward(ctx, t)
    assert e.value.status == L.ERR_UNSUPPORTED


def test_symmetric_form_rejects(L):
    """pair_form 2 (one evaluation per unordered pair) needs targets == sources and the compensated or
    float64 precision (float64: one to four targets per thread); bad pair_form values are refused."""
    lib = L.lib()
    cfg = L.TileConfig()
    cfg.pair_form = 2
    assert _fwd(L, cfg=ctypes.byref(cfg)) == L.ERR_INVALID_ARGUMENT          # targets != sources
    assert _fwd(L, cfg=ctypes.byref(cfg), prec=2, sources=FAKE) == L.ERR_UNSUPPORTED
    cfg.targets_per_thread = 8                                                # compensated only
    assert _fwd(L, cfg=ctypes.byref(cfg), prec=0, sources=FAKE) == L.ERR_INVALID_ARGUMENT
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 0, ctypes.byref(cfg)) == 0
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 1, ctypes.byref(cfg)) > 0
    for t in (3, 4):
        cfg.targets_per_thread = t
        assert lib.vesnet_farfield_workspace_bytes(10, 2, 0, ctypes.byref(cfg)) > 0
        assert lib.vesnet_farfield_workspace_bytes(10, 2, 1, ctypes.byref(cfg)) > 0
    for bad in (5, 6, 7, 9, -1):
        cfg.targets_per_thread = bad
        assert lib.vesnet_farfield_workspace_bytes(10, 2, 1, ctypes.byref(cfg)) == 0
    cfg.targets_per_thread = 2
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 0, ctypes.byref(cfg)) > 0
    cfg.targets_per_thread = 0
    cfg.pair_form = 3
    assert _fwd(L, cfg=ctypes.byref(cfg)) == L.ERR_INVALID_ARGUMENT
    assert lib.vesnet_farfield_workspace_bytes(10, 2, 1, ctypes.byref(cfg)) == 0


def test_noalloc_rejects_before_any_device_call(L):
    """The no-allocation entry point refuses problems whose workspace exceeds its fixed scratch
    array, and bad arguments, on the host (these calls never reach a device)."""
    lib = L.lib()
    P, M = 4_000_000, 10
    args = [_p(FAKE), _p(FAKE), _p(FAKE + 0x2000000 * 8), _p(FAKE + 0x4000000 * 8), _p(FAKE + 0x6000000 * 8), M, P,
            1.0, _p(FAKE + 0x8000000 * 8), 1, None, None]
    assert lib.vesnet_farfield_stokeslet_noalloc(*args) == L.ERR_WORKSPACE
    assert b"scratch" in lib.vesnet_last_error()
    args[7] = 0.0
    assert lib.vesnet_farfield_stokeslet_noalloc(*args) == L.ERR_INVALID_ARGUMENT
    assert lib.vesnet_farfield_stokeslet_noalloc(None, None, None, None, None, 0, 0, 1.0, None, 1, None, None) == 0
