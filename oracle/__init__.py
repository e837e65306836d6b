"""CPU reference ("oracle") for one training step of the differentiable 3DGS rasterizer.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
definition the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call it; the product path (``paper_2602_09999_amd``) never does, and
this package imports nothing from it.

Contents
--------
render64   FP64 preprocess (Eq. 1-2, activations, SH colour, culling),
           per-pixel brute-force front-to-back compositing (Eq. 3-4, alpha
           cap, 1/255 skip, early stop), gradients by torch autograd in FP64,
           L1 loss gradient.
keys32     FP32 emulation of the (tile, depth) instance keys: opacity-aware
           rectangle, exact per-tile test, canonical (tile, depth, id) order
           and tile ranges, with borderline bands.
adam64     Adam in FP64 with the paper's hyperparameters.
cond4d64   conditional 4D Gaussians (Sec. 3.4): 4D rotation from a left and a
           right quaternion, conditional mean and covariance at a time, the
           marginal factor of the opacity.
zorder32   Morton (z-order) permutation of the means: FP32 quantisation,
           bit interleave, stable order.
fp32err    float32 error model of the threshold decisions (Monte Carlo
           arithmetic over the per-Gaussian formulas): the width of the
           borderline bands the comparison protocol exempts.

Pins (tests/test_oracle_*.py) tie each function to closed forms, invariants,
finite differences, library special cases and brute force; see those tests.
"""
from .render64 import (  # noqa: F401
    Settings, DEFAULT_SETTINGS, sh_basis64, quat_to_rotation64, preprocess64,
    composite64, rect_candidates64, render64, l1_loss_grad64, camera_center64,
)
from .adam64 import adam64  # noqa: F401
from .keys32 import keys_ref, keys_ref_banded, depth_key32, tile_lists_for, record32, tile_rect  # noqa: F401
from . import zorder32  # noqa: F401
from . import fp32err  # noqa: F401
from . import cond4d64  # noqa: F401
