"""ctypes binding of libfactgs.so (include/factgs.h): argument marshalling only.

Every computation runs in the HIP library. PyTorch supplies device memory
and the current HIP stream. There is no CPU fallback: if the library is not
built, or a tensor is not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfactgs.so")

FGS_OK = 0
FGS_E_INVALID = -1
FGS_E_CAPACITY = -2
FGS_E_HIP = -3
FGS_E_UNSUPPORTED = -4
FGS_CONE = 0
FGS_PARALLEL = 1
FGS_MODEL_SPLAT = 0
FGS_MODEL_RAY_EXACT = 1
FGS_OP_PROJECT_FWD, FGS_OP_PROJECT_BWD, FGS_OP_VOXELIZE_FWD, FGS_OP_VOXELIZE_BWD = 0, 1, 2, 3

_vp = ctypes.c_void_p


class fgs_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", _vp), ("log_scale", _vp), ("quat", _vp),
                ("density", _vp)]


class fgs_gaussian_grads(ctypes.Structure):
    _fields_ = [("mean", _vp), ("log_scale", _vp), ("quat", _vp), ("density", _vp)]


class fgs_geom(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n_views", ctypes.c_int32), ("angles", _vp),
                ("sod", ctypes.c_float), ("sdd", ctypes.c_float), ("det_w", ctypes.c_int32),
                ("det_h", ctypes.c_int32), ("pitch_u", ctypes.c_float), ("pitch_v", ctypes.c_float),
                ("off_u", ctypes.c_float), ("off_v", ctypes.c_float)]


class fgs_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3),
                ("dims", ctypes.c_int32 * 3)]


class fgs_opts(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_float), ("near_plane", ctypes.c_float),
                ("recompute", ctypes.c_int32), ("accumulate", ctypes.c_int32), ("ablate", ctypes.c_int32),
                ("model", ctypes.c_int32), ("events", _vp), ("density_aabb_tau", ctypes.c_float)]


class fgs_workspace(ctypes.Structure):
    _fields_ = [("ptr", _vp), ("bytes", ctypes.c_uint64), ("needed", ctypes.c_uint64),
                ("n_pairs", ctypes.c_uint64), ("n_records", ctypes.c_uint64),
                ("n_tiles", ctypes.c_uint64), ("kind", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("key_capacity", ctypes.c_uint64), ("overflow", _vp), ("record_bits", ctypes.c_int32),
                ("n_gauss", ctypes.c_uint64)]


class fgs_adc_params(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("split_scale", ctypes.c_float),
                ("prune_density", ctypes.c_float), ("prune_scale", ctypes.c_float),
                ("split_shrink", ctypes.c_float), ("reserved", ctypes.c_int32), ("n_max", ctypes.c_int64)]


class fgs_phantom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("centre", _vp), ("semi", _vp), ("quat", _vp), ("amp", _vp)]


class fgs_mlp(ctypes.Structure):
    _fields_ = [("k_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("w1", _vp), ("w1t", _vp), ("w2", _vp), ("w2t", _vp), ("w3", _vp), ("w3t", _vp),
                ("b1", _vp), ("b2", _vp), ("b3", _vp)]


class fgs_mlp_acts(ctypes.Structure):
    _fields_ = [("z1", _vp), ("z2", _vp), ("z3", _vp), ("h1", _vp), ("h1t", _vp), ("h2", _vp), ("h2t", _vp)]


class fgs_mlp_grads(ctypes.Structure):
    _fields_ = [("dw1", _vp), ("db1", _vp), ("dw2", _vp), ("db2", _vp), ("dw3", _vp), ("db3", _vp)]


class fgs_step_params(ctypes.Structure):
    _fields_ = [("ssim_weight", ctypes.c_float), ("ssim_c1", ctypes.c_float), ("ssim_c2", ctypes.c_float),
                ("tv_weight", ctypes.c_float), ("lr", ctypes.c_float * 4), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("step", ctypes.c_int32)]


class fgs_step_buffers(ctypes.Structure):
    _fields_ = [("img", _vp), ("grad_img", _vp), ("crop_vol", _vp), ("crop_grad", _vp), ("loss", _vp),
                ("params", _vp)]


P = ctypes.POINTER
# (name, argtypes) of every symbol declared in include/factgs.h
SIGNATURES = {
    "fgs_project_views_fwd": [P(fgs_gaussians), P(fgs_geom), ctypes.c_int32, ctypes.c_int32,
                              P(fgs_opts), _vp, P(fgs_workspace), _vp],
    "fgs_project_views_fwd_noalloc": [P(fgs_gaussians), P(fgs_geom), ctypes.c_int32, ctypes.c_int32,
                                      P(fgs_opts), _vp, _vp],
    "fgs_recon_step": [P(fgs_gaussian_grads), P(fgs_gaussian_grads), P(fgs_gaussian_grads), P(fgs_gaussian_grads),
                       ctypes.c_int64, P(fgs_geom), ctypes.c_int32, _vp, P(fgs_grid), P(fgs_opts), P(fgs_step_params),
                       P(fgs_step_buffers), P(fgs_workspace), P(fgs_workspace), P(fgs_workspace), _vp],
    "fgs_step_graph_capture": [P(fgs_gaussian_grads), P(fgs_gaussian_grads), P(fgs_gaussian_grads),
                               P(fgs_gaussian_grads), ctypes.c_int64, P(fgs_geom), ctypes.c_int32, _vp, P(fgs_grid),
                               P(fgs_opts), P(fgs_step_params), P(fgs_step_buffers), P(fgs_workspace),
                               P(fgs_workspace), P(fgs_workspace), P(_vp)],
    "fgs_step_graph_launch": [_vp, P(fgs_step_params), P(fgs_grid), _vp],
    "fgs_step_graph_destroy": [_vp],
    "fgs_project_views_bwd": [P(fgs_gaussians), P(fgs_geom), ctypes.c_int32, ctypes.c_int32,
                              P(fgs_opts), _vp, P(fgs_gaussian_grads), P(fgs_workspace), _vp],
    "fgs_voxelize_fwd": [P(fgs_gaussians), P(fgs_grid), P(fgs_opts), _vp, P(fgs_workspace), _vp],
    "fgs_voxelize_bwd": [P(fgs_gaussians), P(fgs_grid), P(fgs_opts), _vp, P(fgs_gaussian_grads),
                         P(fgs_workspace), _vp],
    "fgs_l1_loss_grad": [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, P(fgs_workspace), _vp],
    "fgs_adam_step": [_vp, _vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                      ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp],
    "fgs_project_views_support": [P(fgs_gaussians), P(fgs_geom), ctypes.c_int32, ctypes.c_int32,
                                  P(fgs_opts), _vp, P(fgs_workspace), _vp],
    "fgs_voxelize_support": [P(fgs_gaussians), P(fgs_grid), P(fgs_opts), _vp, P(fgs_workspace), _vp],
    "fgs_psnr": [_vp, _vp, ctypes.c_int64, ctypes.c_float, _vp, P(fgs_workspace), _vp],
    "fgs_phantom_project": [P(fgs_phantom), P(fgs_geom), ctypes.c_int32, ctypes.c_int32, _vp, _vp],
    "fgs_phantom_voxelize": [P(fgs_phantom), P(fgs_grid), _vp, _vp],
    "fgs_binning_layout": [P(fgs_workspace), P(ctypes.c_uint64), P(ctypes.c_uint64)],
    "fgs_workspace_query": [ctypes.c_int32, P(fgs_gaussians), P(fgs_geom), P(fgs_grid), ctypes.c_int32, P(fgs_opts),
                            P(ctypes.c_uint64), P(ctypes.c_uint64)],
    "fgs_fdk": [_vp, P(fgs_geom), ctypes.c_int32, ctypes.c_int32, P(fgs_grid), _vp, P(fgs_workspace), _vp],
    "fgs_gradient_init": [_vp, P(fgs_grid), ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int64, _vp,
                          P(fgs_gaussian_grads), P(fgs_workspace), _vp],
    "fgs_intensity_init": [_vp, P(fgs_grid), ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int64, _vp,
                           P(fgs_gaussian_grads), P(fgs_workspace), _vp],
    "fgs_gather_patches": [_vp, P(fgs_grid), ctypes.c_float, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_int32, _vp, _vp, _vp],
    "fgs_reduce_max": [_vp, ctypes.c_int64, _vp, P(fgs_workspace), _vp],
    "fgs_adc_accumulate": [_vp, ctypes.c_int64, _vp, _vp],
    "fgs_adc_densify": [P(fgs_gaussians), P(fgs_gaussian_grads), P(fgs_gaussian_grads), _vp, _vp, P(fgs_adc_params),
                        P(fgs_gaussian_grads), P(fgs_gaussian_grads), P(fgs_gaussian_grads), P(ctypes.c_int64),
                        P(fgs_workspace), _vp],
    "fgs_copy": [_vp, _vp, ctypes.c_int64, _vp],
    "fgs_probe": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, P(ctypes.c_double), _vp],
    "fgs_tv_loss_grad": [_vp, P(ctypes.c_int32), ctypes.c_float, _vp, _vp, P(fgs_workspace), _vp],
    "fgs_ssim3d_loss_grad": [_vp, _vp, P(ctypes.c_int32), ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp, _vp,
                             ctypes.c_int32, P(fgs_workspace), _vp],
    "fgs_ssim_loss_grad": [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _vp, _vp, ctypes.c_int32, P(fgs_workspace), _vp],
    "fgs_mlp_pack": [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp],
    "fgs_mlp_fwd": [P(fgs_mlp), _vp, ctypes.c_int32, P(fgs_mlp_acts), _vp],
    "fgs_mlp_heads": [_vp, ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, P(fgs_workspace), _vp],
    "fgs_mlp_bwd": [P(fgs_mlp), _vp, ctypes.c_int32, P(fgs_mlp_acts), _vp, _vp, P(fgs_mlp_grads),
                    P(fgs_workspace), _vp],
    "fgs_canonical_targets": [P(fgs_gaussians), _vp, _vp],
    "fgs_last_error": [],
    "fgs_version": [],
}

_lib = None


class FgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfactgs error {code}: {msg}")
        self.code = code


def lib():
    """Load libfactgs.so (built in-tree by paper_2604_01844_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2604_01844_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name in ("fgs_last_error", "fgs_version") else ctypes.c_int
        _lib = L
    return _lib


def check(code: int):
    if code != FGS_OK:
        raise FgsError(code, lib().fgs_last_error().decode())


def ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libfactgs takes GPU tensors only")
    if not t.is_contiguous():
        raise ValueError("libfactgs takes contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def stream_ptr(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
