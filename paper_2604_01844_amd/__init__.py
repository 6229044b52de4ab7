"""MI355X (gfx950) implementation of the FaCT-GS hot path (arXiv 2604.01844):
the differentiable cone-beam X-ray rasterizer and the Gaussian voxelizer,
forward and backward, in hand-written HIP behind the C ABI of
include/factgs.h (libfactgs.so). This package is the thin Python binding.
"""
from .ops import (  # noqa: F401
    Geometry, Grid, Workspace, ProjectViews, Voxelize, project_views, project_views_backward,
    voxelize, voxelize_backward, l1_loss_grad, ssim_loss_grad, ssim3d_loss_grad, tv_loss_grad, adam_step, psnr, phantom_project, phantom_voxelize,
    binning_dump, project_views_support, voxelize_support, timing_events, fdk, gradient_init, reduce_max, KAPPA, NEAR,
    workspace_bytes,
)
from ._abi import lib, LIB_PATH, FgsError  # noqa: F401
from .mlp import InitMLP, canonical_targets  # noqa: F401,E402
from . import ops, recon  # noqa: F401,E402
