"""MI355X (gfx950) rasterized Steered Mixture of Experts: HIP kernels behind a C ABI.

``_capi`` binds ``libsmoe.so`` (declared in ``include/smoe.h``); ``core`` manages
device memory around it; ``autograd`` exposes the render as a torch.autograd.Function.
Importing the package requires the built library: there is no CPU fallback.
"""
from . import _capi  # noqa: F401  (fails loudly when libsmoe.so is missing)
from .core import (AdamConfig, Bins, FitState, Segments, bin, bin_batched,  # noqa: F401
                   fuse_windows, make_grid, materialize, num_params, psnr, render,
                   render_backward, render_batched, render_noalloc, tiles)

__version__ = "0.1.0"
