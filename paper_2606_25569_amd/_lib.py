"""ctypes loader and signatures for libvesnet.so (include/vesnet.h).

Argument marshalling only: every step of the far-field path runs in the HIP
kernels behind the C-ABI.  There is no fallback: if the library is missing or
fails to load, importing the product API raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VESNET_LIB", os.path.join(_HERE, "libvesnet.so"))

OK, ERR_INVALID_ARGUMENT, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = 0, -1, -2, -3, -4
FP64, FP32_COMPENSATED, FP32_NAIVE = 0, 1, 2

PRECISIONS = {"fp64": FP64, "fp32c": FP32_COMPENSATED, "fp32": FP32_NAIVE,
              FP64: FP64, FP32_COMPENSATED: FP32_COMPENSATED, FP32_NAIVE: FP32_NAIVE}

EXPORTED = (
    "vesnet_version", "vesnet_last_error", "vesnet_check_offsets", "vesnet_default_tile_config",
    "vesnet_farfield_workspace_bytes", "vesnet_farfield_prepare", "vesnet_farfield_evaluate",
    "vesnet_farfield_stokeslet", "vesnet_batched_workspace_bytes", "vesnet_farfield_stokeslet_batched",
    "vesnet_graph_create_batched", "vesnet_graph_launch", "vesnet_graph_destroy",
    "vesnet_backward_workspace_bytes", "vesnet_farfield_stokeslet_backward", "vesnet_backward_points_workspace_bytes",
    "vesnet_farfield_stokeslet_backward_points", "vesnet_autotune",
    "vesnet_farfield_stokeslet_nearmasked", "vesnet_elastic_force", "vesnet_near_layers",
    "vesnet_rbf_workspace_bytes", "vesnet_rbf_fit", "vesnet_rbf_eval_near", "vesnet_treecode_default_depth",
    "vesnet_treecode_workspace_bytes", "vesnet_farfield_treecode", "vesnet_fmm_default_depth", "vesnet_fmm_workspace_bytes",
    "vesnet_farfield_fmm", "vesnet_fmm_nearmasked_workspace_bytes", "vesnet_farfield_fmm_nearmasked",
    "vesnet_farfield_stokeslet_noalloc",
)

NOALLOC_SCRATCH_BYTES = 64 << 20  # VESNET_NOALLOC_SCRATCH_BYTES of include/vesnet.h


class VesnetError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vesnet status {status}: {message}")
        self.status = status


class TileConfig(ctypes.Structure):
    _fields_ = [("targets_per_thread", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("source_splits", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("source_staging", ctypes.c_int32), ("accumulate", ctypes.c_int32), ("pair_form", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(int(d.get("targets_per_thread", 0)), int(d.get("block_threads", 0)),
                   int(d.get("source_splits", 0)), int(d.get("blocks_per_cu", 0)), int(d.get("source_staging", 0)),
                   int(d.get("accumulate", 0)), int(d.get("pair_form", 0)))


_lib = None


def lib():
    """The loaded library (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"libvesnet.so not found at {LIB_PATH}: build it first (python __graft_entry__.py build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, SZ, D, INT = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double, ctypes.c_int
    CFG = ctypes.POINTER(TileConfig)
    sig = {
        "vesnet_version": ([], ctypes.c_char_p),
        "vesnet_last_error": ([], ctypes.c_char_p),
        "vesnet_check_offsets": ([P, I32, I32], INT),
        "vesnet_default_tile_config": ([I32, I32, INT, CFG], INT),
        "vesnet_farfield_workspace_bytes": ([I32, I32, INT, CFG], SZ),
        "vesnet_farfield_prepare": ([P, P, P, P, I32, I32, INT, P, SZ, P], INT),
        "vesnet_farfield_evaluate": ([P, P, I32, I32, D, P, INT, CFG, P, SZ, P], INT),
        "vesnet_farfield_stokeslet": ([P, P, P, P, P, I32, I32, D, P, INT, CFG, P, SZ, P], INT),
        "vesnet_farfield_stokeslet_noalloc": ([P, P, P, P, P, I32, I32, D, P, INT, CFG, P], INT),
        "vesnet_batched_workspace_bytes": ([I32, I32, I32, INT], SZ),
        "vesnet_farfield_stokeslet_batched": ([P, P, P, P, P, I32, I32, P, I32, P, P, INT, CFG, P, SZ, P], INT),
        "vesnet_graph_create_batched": ([P, P, P, P, P, I32, I32, P, I32, P, P, INT, CFG, P, SZ,
                                         ctypes.POINTER(P)], INT),
        "vesnet_graph_launch": ([P, P], INT),
        "vesnet_graph_destroy": ([P], INT),
        "vesnet_backward_workspace_bytes": ([I32, I32, INT], SZ),
        "vesnet_farfield_stokeslet_backward": ([P, P, P, P, P, I32, I32, D, P, P, P, P, P, INT, P, SZ, P], INT),
        "vesnet_backward_points_workspace_bytes": ([I32, I32, INT], SZ),
        "vesnet_farfield_stokeslet_backward_points": ([P, P, P, P, I32, I32, D, P, P, P, P, INT, P, SZ, P], INT),
        "vesnet_farfield_stokeslet_nearmasked": ([P, P, P, P, P, I32, I32, D, P, P, I32, P, INT, CFG, P, SZ, P], INT),
        "vesnet_elastic_force": ([P, P, D, P, I32, I32, P, P, P], INT),
        "vesnet_near_layers": ([P, P, P, I32, I32, P, P], INT),
        "vesnet_rbf_workspace_bytes": ([I32, I32], SZ),
        "vesnet_rbf_fit": ([P, P, P, P, I32, I32, I32, D, P, P, SZ, P], INT),
        "vesnet_rbf_eval_near": ([P, P, P, P, I32, I32, D, P, I32, P, P, I32, P, P], INT),
        "vesnet_treecode_default_depth": ([I32], I32),
        "vesnet_treecode_workspace_bytes": ([I32, I32, I32], SZ),
        "vesnet_farfield_treecode": ([P, P, P, P, I32, I32, D, I32, I32, P, P, SZ, P], INT),
        "vesnet_fmm_default_depth": ([I32, I32], I32),
        "vesnet_fmm_workspace_bytes": ([I32, I32, I32], SZ),
        "vesnet_farfield_fmm": ([P, P, P, P, I32, I32, D, I32, I32, P, P, SZ, P], INT),
        "vesnet_fmm_nearmasked_workspace_bytes": ([I32, I32, I32, I32], SZ),
        "vesnet_farfield_fmm_nearmasked": ([P, P, P, P, I32, I32, D, I32, I32, P, P, I32, P, P, SZ, P], INT),
        "vesnet_autotune": ([P, P, P, P, P, I32, I32, INT, P, I32, P, D, P, INT, INT, P, SZ, P, CFG,
                             ctypes.POINTER(ctypes.c_float)], INT),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status: int):
    if status != OK:
        raise VesnetError(status, lib().vesnet_last_error().decode(errors="replace"))


def precision_code(precision) -> int:
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"unknown precision {precision!r}; use 'fp64', 'fp32c' or 'fp32'") from None
