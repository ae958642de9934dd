"""ctypes front end of the plain FP64 CPU oracle (vesnet_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

The sum it evaluates is eq. (single_layer) with the Stokeslet of
eq. (Stokeslet) (read with -ln|r| I), trapezoid rule of Section 2.2.1, each
target excluding the points of its own vesicle (eq. (membrane_velocity),
Algorithm 4 DirectSingleLayerIntegral).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vesnet_oracle.c")
_LIB = os.path.join(_HERE, "libvesnet_oracle.so")
# A test may point this at a deliberately broken copy to check that the pins catch it.
_LIB_OVERRIDE = os.environ.get("VESNET_ORACLE_LIB")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build()
            lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        lib.vo_num_threads.restype = ctypes.c_int
        lib.vo_farfield_at.argtypes = [I, P, P, P, P, I, P, P, P, P, P, P, D, P, P]
        lib.vo_farfield_at.restype = ctypes.c_int
        lib.vo_grad_targets_at.argtypes = [I, P, P, P, P, I, P, P, P, P, P, P, D, P, P, P, P]
        lib.vo_grad_targets_at.restype = ctypes.c_int
        lib.vo_grad_sources_at.argtypes = [I, P, I, P, P, P, P, P, P, P, P, P, D, P, P, P, P, P, P, P, P, P]
        lib.vo_grad_sources_at.restype = ctypes.c_int
        lib.vo_farfield_nearmasked_at.argtypes = [I, P, P, P, P, I, P, P, P, ctypes.c_int32, P, P, P, D, P, P, P, I]
        lib.vo_farfield_nearmasked_at.restype = ctypes.c_long
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().vo_num_threads())


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def vesicle_ids(offsets, n_points=None) -> np.ndarray:
    """Vesicle id of every point from the CSR offsets."""
    offsets = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(offsets)
    return np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)


def farfield(targets, sources, f, w, mu, target_excl, source_ves, select=None):
    """u at targets[:, select] (all targets if select is None); returns (2, n_sel) float64.

    target_excl[i] is the vesicle id whose sources target i skips (-1 for none);
    source_ves[j] is the vesicle id of source j.
    """
    lib = _load()
    tx, ty = _c(targets[0], np.float64), _c(targets[1], np.float64)
    sx, sy = _c(sources[0], np.float64), _c(sources[1], np.float64)
    fx, fy = _c(f[0], np.float64), _c(f[1], np.float64)
    w = _c(w, np.float64)
    te = _c(target_excl, np.int32)
    sv = _c(source_ves, np.int32)
    sel = _c(np.arange(tx.shape[0]) if select is None else select, np.int64)
    ux = np.empty(sel.shape[0])
    uy = np.empty(sel.shape[0])
    rc = lib.vo_farfield_at(sel.shape[0], _ptr(sel), _ptr(tx), _ptr(ty), _ptr(te), sx.shape[0], _ptr(sx), _ptr(sy),
                            _ptr(sv), _ptr(fx), _ptr(fy), _ptr(w), float(mu), _ptr(ux), _ptr(uy))
    if rc != 0:
        raise ValueError("oracle: coincident points in different vesicles (r = 0)")
    return np.stack([ux, uy])


def farfield_suspension(X, f, w, offsets, mu, select=None, targets=None):
    """Own-vesicle-excluded far field of a suspension; targets default to the points X."""
    vid = vesicle_ids(offsets)
    T = X if targets is None else targets
    return farfield(T, X, f, w, mu, vid, vid, select)


def farfield_nearmasked(targets, sources, f, w, mu, target_excl, source_ves, n_ves, select=None):
    """Near-field masked far field at targets[:, select] and the near pairs.

    Returns (u (2, n_sel), pairs (n_pairs, 2) int64 of (selected position, vesicle id))."""
    lib = _load()
    tx, ty = _c(targets[0], np.float64), _c(targets[1], np.float64)
    sx, sy = _c(sources[0], np.float64), _c(sources[1], np.float64)
    fx, fy = _c(f[0], np.float64), _c(f[1], np.float64)
    w = _c(w, np.float64)
    te, sv = _c(target_excl, np.int32), _c(source_ves, np.int32)
    sel = _c(np.arange(tx.shape[0]) if select is None else select, np.int64)
    ux, uy = np.empty(sel.shape[0]), np.empty(sel.shape[0])
    cap = 16 * sel.shape[0] + 16
    while True:
        pairs = np.empty((cap, 2), dtype=np.int64)
        n = lib.vo_farfield_nearmasked_at(sel.shape[0], _ptr(sel), _ptr(tx), _ptr(ty), _ptr(te), sx.shape[0], _ptr(sx),
                                          _ptr(sy), _ptr(sv), int(n_ves), _ptr(fx), _ptr(fy), _ptr(w), float(mu),
                                          _ptr(ux), _ptr(uy), _ptr(pairs), cap)
        if n == -2:
            raise ValueError("oracle: coincident points in different vesicles (r = 0)")
        if n < 0:
            raise ValueError(f"oracle: near-masked sum failed ({n})")
        if n <= cap:
            return np.stack([ux, uy]), pairs[:n].copy()
        cap = int(n)


def nearmasked_suspension(X, f, w, offsets, mu, select=None, targets=None):
    vid = vesicle_ids(offsets)
    T = X if targets is None else targets
    return farfield_nearmasked(T, X, f, w, mu, vid, vid, len(offsets) - 1, select)


def grad_targets(targets, sources, f, w, mu, target_excl, source_ves, g, select=None):
    lib = _load()
    tx, ty = _c(targets[0], np.float64), _c(targets[1], np.float64)
    sx, sy = _c(sources[0], np.float64), _c(sources[1], np.float64)
    fx, fy = _c(f[0], np.float64), _c(f[1], np.float64)
    w = _c(w, np.float64)
    gx, gy = _c(g[0], np.float64), _c(g[1], np.float64)
    te, sv = _c(target_excl, np.int32), _c(source_ves, np.int32)
    sel = _c(np.arange(tx.shape[0]) if select is None else select, np.int64)
    ox, oy = np.empty(sel.shape[0]), np.empty(sel.shape[0])
    rc = lib.vo_grad_targets_at(sel.shape[0], _ptr(sel), _ptr(tx), _ptr(ty), _ptr(te), sx.shape[0], _ptr(sx),
                                _ptr(sy), _ptr(sv), _ptr(fx), _ptr(fy), _ptr(w), float(mu), _ptr(gx), _ptr(gy),
                                _ptr(ox), _ptr(oy))
    if rc != 0:
        raise ValueError("oracle: coincident points in different vesicles (r = 0)")
    return np.stack([ox, oy])


def grad_sources(targets, sources, f, w, mu, target_excl, source_ves, g, select=None):
    """Returns dict with grad_sources (2,n), v (2,n), grad_f (2,n), grad_w (n,) at the selected sources."""
    lib = _load()
    tx, ty = _c(targets[0], np.float64), _c(targets[1], np.float64)
    sx, sy = _c(sources[0], np.float64), _c(sources[1], np.float64)
    fx, fy = _c(f[0], np.float64), _c(f[1], np.float64)
    w = _c(w, np.float64)
    gx, gy = _c(g[0], np.float64), _c(g[1], np.float64)
    te, sv = _c(target_excl, np.int32), _c(source_ves, np.int32)
    sel = _c(np.arange(sx.shape[0]) if select is None else select, np.int64)
    n = sel.shape[0]
    out = [np.empty(n) for _ in range(7)]
    rc = lib.vo_grad_sources_at(n, _ptr(sel), tx.shape[0], _ptr(tx), _ptr(ty), _ptr(te), _ptr(sx), _ptr(sy),
                                _ptr(sv), _ptr(fx), _ptr(fy), _ptr(w), float(mu), _ptr(gx), _ptr(gy),
                                *[_ptr(o) for o in out])
    if rc != 0:
        raise ValueError("oracle: coincident points in different vesicles (r = 0)")
    return {"grad_sources": np.stack(out[0:2]), "v": np.stack(out[2:4]),
            "grad_f": np.stack(out[4:6]), "grad_w": out[6]}


def grad_suspension(X, f, w, offsets, mu, g, select=None):
    """dL/dX (targets and sources both X, both roles), dL/df, dL/dw at the selected points."""
    vid = vesicle_ids(offsets)
    gt = grad_targets(X, X, f, w, mu, vid, vid, g, select)
    gs = grad_sources(X, X, f, w, mu, vid, vid, g, select)
    return {"grad_X": gt + gs["grad_sources"], "grad_targets": gt, **gs}
