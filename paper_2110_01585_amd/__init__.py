"""MI355X-native EP for TV-prior image restoration (arXiv 2110.01585).

The compute path is libeptv.so (hand-written HIP for gfx950, C ABI in
include/ep_tv.h); this package holds its build script and a thin ctypes
binding.  Importing the package does not load the library; the first call
does, and fails loudly if it has not been built.
"""
from .api import (Context, EPTVError, ProblemSpec, ep_tv_denoise_noalloc, ep_tv_tilted_moments,
                  ep_tv_tilted_moments_prior, ep_tv_version, ep_tv_workspace_bytes,
                  spec_from_synthetic)
from . import _native as native
from .net import Net, load_weights, save_weights

__all__ = ["Context", "EPTVError", "ProblemSpec", "ep_tv_denoise_noalloc", "ep_tv_tilted_moments",
           "ep_tv_tilted_moments_prior",
           "ep_tv_version", "ep_tv_workspace_bytes",
           "spec_from_synthetic", "native", "Net", "load_weights", "save_weights"]
