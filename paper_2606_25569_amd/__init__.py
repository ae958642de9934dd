"""MI355X-native far-field Stokeslet sum (the far-field N-body hot path of the
VesNet vesicle solver): C-ABI library libvesnet.so with gfx950 HIP kernels,
and a thin PyTorch binding.  Importing fails loudly if the library is not built."""
from . import _lib
from ._lib import FP32_COMPENSATED, FP32_NAIVE, FP64, TileConfig, VesnetError

_lib.lib()  # load now: no CPU fallback exists

from .farfield import (BatchedProblem, Partition, autotune, default_config, elastic_force,  # noqa: E402
                       farfield_backward, farfield_backward_points, farfield_fmm, farfield_fmm_nearmasked, farfield_forward,
                       farfield_nearmasked, farfield_stokeslet,
                       farfield_treecode, load_tuned, near_layers, rbf_eval_near, rbf_fit, workspace_bytes)

__all__ = ["BatchedProblem", "Partition", "TileConfig", "VesnetError", "autotune", "default_config", "elastic_force",
           "farfield_backward", "farfield_backward_points", "farfield_fmm", "farfield_fmm_nearmasked", "farfield_forward", "farfield_nearmasked",
           "farfield_stokeslet",
           "farfield_treecode",
           "load_tuned",
           "near_layers", "rbf_eval_near", "rbf_fit", "workspace_bytes",
           "FP64", "FP32_COMPENSATED", "FP32_NAIVE"]
