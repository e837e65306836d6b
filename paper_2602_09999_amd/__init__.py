"""MI355X (gfx950) training step of 3D Gaussian Splatting after Faster-GS.

The compute path is libfastergs.so (hand-written HIP kernels behind the C ABI
in include/fastergs.h); this package only marshals arguments.  Importing it
does not load the library; the first call does, and raises if it is missing.
"""
from .binding import (  # noqa: F401
    PARAM_NAMES, Rasterizer, adam_step, default_settings, l1_loss_backward, make_camera,
    rasterize_backward, rasterize_forward, workspace_layout, workspace_size,
)
from .autograd import FusedAdam, RasterizeGaussians, rasterize, train_step  # noqa: F401

__all__ = [
    "PARAM_NAMES", "Rasterizer", "adam_step", "default_settings", "l1_loss_backward", "make_camera",
    "rasterize_backward", "rasterize_forward", "workspace_layout", "workspace_size", "FusedAdam",
    "RasterizeGaussians", "rasterize", "train_step",
]
