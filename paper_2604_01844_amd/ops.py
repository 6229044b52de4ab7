"""Python entry points over libfactgs: the rasterizer (``project_views``), the
voxelizer (``voxelize``), their backward calls, losses, Adam, PSNR and the
phantom generator, plus ``torch.autograd.Function`` wrappers whose backward
is the library's hand-written backward.

Argument marshalling only: tensors must already be contiguous float32 on the
GPU; every step runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _abi as A

KAPPA = 3.0
NEAR = 1e-2


# ------------------------------------------------------------------ descriptors

@dataclass
class Geometry:
    """Circular-orbit flat-detector geometry (cone or parallel beam).
    ``angles`` is a float32 GPU tensor of view angles in radians."""
    angles: torch.Tensor
    det_w: int
    det_h: int
    pitch_u: float
    pitch_v: float
    sod: float = 1.5
    sdd: float = 2.0
    mode: str = "cone"
    off_u: float = 0.0
    off_v: float = 0.0

    @classmethod
    def from_dict(cls, d: dict, angles, device="cuda") -> "Geometry":
        ang = torch.as_tensor(angles, dtype=torch.float32).to(device).contiguous()
        return cls(angles=ang, det_w=d["det_w"], det_h=d["det_h"], pitch_u=d["pitch_u"],
                   pitch_v=d["pitch_v"], sod=d["sod"], sdd=d["sdd"], mode=d["mode"],
                   off_u=d.get("off_u", 0.0), off_v=d.get("off_v", 0.0))

    @property
    def n_views(self) -> int:
        return int(self.angles.numel())

    def struct(self) -> A.fgs_geom:
        return A.fgs_geom(A.FGS_PARALLEL if self.mode == "parallel" else A.FGS_CONE, self.n_views,
                          A.ptr(self.angles), self.sod, self.sdd, self.det_w, self.det_h,
                          self.pitch_u, self.pitch_v, self.off_u, self.off_v)


@dataclass
class Grid:
    """Voxel grid: voxel (ix, iy, iz) centre = origin + (index + 1/2) * spacing;
    volumes are [nz][ny][nx]."""
    origin: tuple
    spacing: tuple
    dims: tuple

    @classmethod
    def from_dict(cls, d: dict) -> "Grid":
        return cls(tuple(d["origin"]), tuple(d["spacing"]), tuple(int(x) for x in d["dims"]))

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def struct(self) -> A.fgs_grid:
        return A.fgs_grid((ctypes.c_float * 3)(*self.origin), (ctypes.c_float * 3)(*self.spacing),
                          (ctypes.c_int32 * 3)(*self.dims))


class Workspace:
    """Caller-owned device workspace that grows on FGS_E_CAPACITY."""

    def __init__(self, device="cuda", nbytes: int = 0):
        self.device = torch.device(device)
        self.buf = None
        self.overflow_buf = None
        self.s = A.fgs_workspace()
        if nbytes:
            self.ensure(nbytes)

    def ensure(self, nbytes: int):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(int(nbytes * 1.25) + (1 << 20), dtype=torch.uint8, device=self.device)
            self.s.kind = 0
        self.s.ptr = self.buf.data_ptr()
        self.s.bytes = self.buf.numel()

    def set_capacity(self, pairs: int):
        """Lay the lists out for at most `pairs` (tile, Gaussian) pairs and keep
        the pair count on the device (no host wait per call; key_capacity in
        include/factgs.h). A call that needs more bins nothing and is recorded
        in a device overflow word, read with overflowed()."""
        if self.overflow_buf is None:
            self.overflow_buf = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.s.key_capacity = int(pairs)
        self.s.overflow = self.overflow_buf.data_ptr()
        self.s.kind = 0

    def overflowed(self, reset: bool = True):
        """(any call overflowed since the last reset, largest pair count it
        needed); waits for the stream. With reset, clears the record."""
        if self.overflow_buf is None:
            return False, 0
        f, need = (int(x) for x in self.overflow_buf.tolist())
        if reset and f:
            self.overflow_buf.zero_()
        return bool(f), need & 0xffffffff

    def call(self, fn, *args):
        """Call fn(*args, &ws, stream), growing the workspace on FGS_E_CAPACITY."""
        for _ in range(6):
            if self.buf is None:
                self.ensure(64 << 20)
            code = fn(*args, ctypes.byref(self.s), A.stream_ptr(self.device))
            if code != A.FGS_E_CAPACITY:
                A.check(code)
                return
            self.ensure(int(self.s.needed))
        raise A.FgsError(A.FGS_E_CAPACITY, "workspace did not converge")

    @property
    def n_pairs(self) -> int:
        return int(self.s.n_pairs)


def _gauss(mean, log_scale, quat, density) -> A.fgs_gaussians:
    n = density.numel()
    for t, rows in ((mean, 3), (log_scale, 3), (quat, 4)):
        if t.dtype != torch.float32 or t.shape != (rows, n):
            raise ValueError(f"expected float32 [{rows}][{n}], got {t.dtype} {tuple(t.shape)}")
    if density.dtype != torch.float32:
        raise ValueError("density must be float32")
    return A.fgs_gaussians(n, A.ptr(mean), A.ptr(log_scale), A.ptr(quat), A.ptr(density))


def _grads_like(mean, log_scale, quat, density):
    return (torch.empty_like(mean), torch.empty_like(log_scale), torch.empty_like(quat),
            torch.empty_like(density))


# fgs_opts.ablate bits (include/factgs.h): switch one part of the
# rasterizer's design off, for measuring what it contributes
ABLATE_SQUARE_BOX, ABLATE_QUADRANT_CULL, ABLATE_PER_PIXEL_BWD = 1, 2, 4


# fgs_opts.model: the splat M of Eq. 4 (the method) or the ray-exact E of Eq. 3
MODELS = {"splat": A.FGS_MODEL_SPLAT, "exact": A.FGS_MODEL_RAY_EXACT}


def _model(model: str) -> int:
    if model not in MODELS:
        raise ValueError(f"model must be one of {sorted(MODELS)}")
    return MODELS[model]


def _opts(kappa, near, recompute=1, events=None, accumulate=0, ablate=0, model="splat", tau=0.0) -> A.fgs_opts:
    """events: optional pair of started torch.cuda.Event objects to record
    around the call's pixel/voxel kernel. tau > 0: the density-aware support
    d^2 <= min(kappa^2, 2 ln(peak / tau)) (fgs_opts.density_aabb_tau)."""
    o = A.fgs_opts(float(kappa), float(near), int(recompute), int(accumulate), int(ablate), _model(model), None,
                   float(tau))
    if events is not None:
        arr = (ctypes.c_void_p * 2)(events[0].cuda_event, events[1].cuda_event)
        o._events_keepalive = arr
        o.events = ctypes.cast(arr, ctypes.c_void_p)
    return o


def timing_events():
    """A (start, stop) pair of timing events, created on the current stream so
    the library can record them."""
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    for e in ev:
        e.record()
    return ev


# ------------------------------------------------------------------ rasterizer
#
# One library call bins all its views together; a call whose (tile, Gaussian)
# pairs would exceed 2^32 is refused with FGS_E_UNSUPPORTED. The wrappers then
# split the view range into chunks (halving until the library accepts them)
# and remember the chunk size in the workspace object. The backward of a
# chunked range rebuilds each chunk's lists and accumulates the gradients in
# the library (opts.accumulate).

def _chunk_events(events, k):
    """events: None, one (start, stop) pair, or a list of pairs (one per chunk)."""
    if events is None or isinstance(events, tuple):
        return events
    return events[k]


def _over_views(ws: Workspace, vc: int, views_per_call: int | None, run):
    """run(begin_offset, count, first, chunked, chunk_index) for each chunk of
    the range."""
    per = views_per_call or getattr(ws, "views_per_call", None) or vc
    while True:
        try:
            for k, b in enumerate(range(0, vc, per)):
                run(b, min(per, vc - b), b == 0, per < vc, k)
            return
        except A.FgsError as e:
            if e.code != A.FGS_E_UNSUPPORTED or per == 1 or views_per_call:
                raise
            per = (per + 1) // 2
            ws.views_per_call = per


def project_views(mean, log_scale, quat, density, geom: Geometry, view_begin: int = 0,
                  view_count: int | None = None, *, kappa: float = KAPPA, near: float = NEAR,
                  ws: Workspace | None = None, out: torch.Tensor | None = None, events=None,
                  views_per_call: int | None = None, ablate: int = 0, model: str = "splat",
                  tau: float = 0.0) -> torch.Tensor:
    """Rasterize views [view_begin, view_begin + view_count): [V][H][W] float32.
    model="exact": the ray-exact line integrals instead of the splat.
    tau > 0: the density-aware support (splat model)."""
    L = A.lib()
    vc = geom.n_views - view_begin if view_count is None else view_count
    ws = ws or Workspace(mean.device)
    if out is None:
        out = torch.empty((vc, geom.det_h, geom.det_w), dtype=torch.float32, device=mean.device)
    g = _gauss(mean, log_scale, quat, density)
    gm = geom.struct()

    def run(b, c, first, chunked, k):
        o = _opts(kappa, near, events=_chunk_events(events, k), ablate=ablate, model=model, tau=tau)
        ws.call(L.fgs_project_views_fwd, ctypes.byref(g), ctypes.byref(gm), view_begin + b, c, ctypes.byref(o),
                A.ptr(out[b]))
    _over_views(ws, vc, views_per_call, run)
    return out


def project_views_backward(mean, log_scale, quat, density, geom: Geometry, grad_img, view_begin: int = 0,
                           view_count: int | None = None, *, kappa: float = KAPPA, near: float = NEAR,
                           recompute: bool = True, ws: Workspace | None = None, out=None, events=None,
                           views_per_call: int | None = None, ablate: int = 0, model: str = "splat",
                           tau: float = 0.0):
    """dL/d(mean, log_scale, quat, density) given dL/dimg. Lists left by the
    forward are reused only when the range ran as one call (with the same
    model)."""
    L = A.lib()
    vc = geom.n_views - view_begin if view_count is None else view_count
    ws = ws or Workspace(mean.device)
    grads = out if out is not None else _grads_like(mean, log_scale, quat, density)
    g = _gauss(mean, log_scale, quat, density)
    gr = A.fgs_gaussian_grads(*(A.ptr(t) for t in grads))
    gm = geom.struct()
    gi = grad_img.contiguous()

    def run(b, c, first, chunked, k):
        o = _opts(kappa, near, 1 if (recompute or chunked) else 0, _chunk_events(events, k),
                  accumulate=0 if first else 1, ablate=ablate, model=model, tau=tau)
        ws.call(L.fgs_project_views_bwd, ctypes.byref(g), ctypes.byref(gm), view_begin + b, c, ctypes.byref(o),
                A.ptr(gi[b]), ctypes.byref(gr))
    _over_views(ws, vc, views_per_call, run)
    return grads


# ------------------------------------------------------------------ voxelizer

def voxelize(mean, log_scale, quat, density, grid: Grid, *, kappa: float = KAPPA,
             ws: Workspace | None = None, out: torch.Tensor | None = None, events=None,
             tau: float = 0.0) -> torch.Tensor:
    L = A.lib()
    ws = ws or Workspace(mean.device)
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=mean.device)
    g = _gauss(mean, log_scale, quat, density)
    gd = grid.struct()
    o = _opts(kappa, NEAR, events=events, tau=tau)
    ws.call(L.fgs_voxelize_fwd, ctypes.byref(g), ctypes.byref(gd), ctypes.byref(o), A.ptr(out))
    return out


def voxelize_backward(mean, log_scale, quat, density, grid: Grid, grad_vol, *, kappa: float = KAPPA,
                      recompute: bool = True, ws: Workspace | None = None, out=None, events=None,
                      accumulate: bool = False, tau: float = 0.0):
    """dL/d(mean, log_scale, quat, density) given dL/dvol; with accumulate the
    gradients are added to `out` instead of overwriting it."""
    L = A.lib()
    ws = ws or Workspace(mean.device)
    grads = out if out is not None else _grads_like(mean, log_scale, quat, density)
    g = _gauss(mean, log_scale, quat, density)
    gr = A.fgs_gaussian_grads(*(A.ptr(t) for t in grads))
    gd = grid.struct()
    o = _opts(kappa, NEAR, 1 if recompute else 0, events, accumulate=1 if accumulate else 0, tau=tau)
    ws.call(L.fgs_voxelize_bwd, ctypes.byref(g), ctypes.byref(gd), ctypes.byref(o),
            A.ptr(grad_vol.contiguous()), ctypes.byref(gr))
    return grads


def project_views_support(mean, log_scale, quat, density, geom: Geometry, view_begin: int = 0,
                          view_count: int | None = None, *, kappa: float = KAPPA, near: float = NEAR,
                          ws: Workspace | None = None, model: str = "splat", tau: float = 0.0) -> int:
    """Number of (pixel, Gaussian) pairs in the support (the rasterizer's work)."""
    L = A.lib()
    vc = geom.n_views - view_begin if view_count is None else view_count
    ws = ws or Workspace(mean.device)
    out = torch.zeros(1, dtype=torch.int64, device=mean.device)
    g = _gauss(mean, log_scale, quat, density)
    gm = geom.struct()
    o = _opts(kappa, near, model=model, tau=tau)
    total = [0]

    def run(b, c, first, chunked, k):
        if first:
            total[0] = 0
        ws.call(L.fgs_project_views_support, ctypes.byref(g), ctypes.byref(gm), view_begin + b, c,
                ctypes.byref(o), A.ptr(out))
        total[0] += int(out.item())
    _over_views(ws, vc, None, run)
    return total[0]


def voxelize_support(mean, log_scale, quat, density, grid: Grid, *, kappa: float = KAPPA,
                     ws: Workspace | None = None, tau: float = 0.0) -> int:
    """Number of (voxel, Gaussian) pairs in the support (the voxelizer's work)."""
    L = A.lib()
    ws = ws or Workspace(mean.device)
    out = torch.zeros(1, dtype=torch.int64, device=mean.device)
    g = _gauss(mean, log_scale, quat, density)
    gd = grid.struct()
    o = _opts(kappa, NEAR, tau=tau)
    ws.call(L.fgs_voxelize_support, ctypes.byref(g), ctypes.byref(gd), ctypes.byref(o), A.ptr(out))
    return int(out.item())


def workspace_bytes(op: str, n: int, n_pairs: int, *, geom: Geometry | None = None, view_count: int = 1,
                    grid: Grid | None = None, model: str = "splat") -> int:
    """Upper bound on the workspace bytes of one call binning n_pairs (tile,
    Gaussian) pairs (fgs_workspace_query). op: "project_fwd", "project_bwd",
    "voxelize_fwd" or "voxelize_bwd"."""
    ops_ = {"project_fwd": A.FGS_OP_PROJECT_FWD, "project_bwd": A.FGS_OP_PROJECT_BWD,
            "voxelize_fwd": A.FGS_OP_VOXELIZE_FWD, "voxelize_bwd": A.FGS_OP_VOXELIZE_BWD}
    g = A.fgs_gaussians(int(n), None, None, None, None)
    gm = geom.struct() if geom is not None else None
    gd = grid.struct() if grid is not None else None
    o = _opts(KAPPA, NEAR, model=model)
    fixed, per = ctypes.c_uint64(), ctypes.c_uint64()
    A.check(A.lib().fgs_workspace_query(ops_[op], ctypes.byref(g), ctypes.byref(gm) if gm is not None else None,
                                        ctypes.byref(gd) if gd is not None else None, int(view_count),
                                        ctypes.byref(o), ctypes.byref(fixed), ctypes.byref(per)))
    return int(fixed.value) + int(n_pairs) * int(per.value)


# ------------------------------------------------------------------ loss / optimiser

def l1_loss_grad(img, gt, *, n_views: int | None = None, ws: Workspace | None = None, want_grad=True):
    """Eq. 5 L1 term: (sum over views of mean |img - gt|, sign(img - gt)/P)."""
    L = A.lib()
    ws = ws or Workspace(img.device, 1 << 16)
    nv = img.shape[0] if n_views is None else n_views
    per = img.numel() // nv
    loss = torch.empty(1, dtype=torch.float32, device=img.device)
    grad = torch.empty_like(img) if want_grad else None
    ws.call(L.fgs_l1_loss_grad, A.ptr(img), A.ptr(gt), per, nv, A.ptr(loss), A.ptr(grad))
    return loss, grad


SSIM_C1, SSIM_C2 = 0.01 ** 2, 0.03 ** 2


def ssim_loss_grad(img, gt, *, scale: float = 1.0, c1: float = SSIM_C1, c2: float = SSIM_C2,
                   ws: Workspace | None = None, grad=None, accumulate: bool = False, want_grad=True):
    """SSIM term of Eq. 5 over img, gt [V][H][W]: (loss device scalar
    scale * (1 - mean SSIM), gradient or None). With accumulate the gradient
    is added to `grad`."""
    ws = ws or Workspace(img.device)
    V, H, W = img.shape
    loss = torch.empty(1, device=img.device)
    if want_grad and grad is None:
        grad = torch.empty_like(img)
    ws.call(A.lib().fgs_ssim_loss_grad, A.ptr(img.contiguous()), A.ptr(gt.contiguous()), W, H, V, float(c1),
            float(c2), float(scale), A.ptr(loss), A.ptr(grad if want_grad else None), 1 if accumulate else 0)
    return loss, (grad if want_grad else None)


def ssim3d_loss_grad(vol, gt, *, scale: float = 1.0, c1: float = SSIM_C1, c2: float = SSIM_C2,
                     ws: Workspace | None = None, grad=None, accumulate: bool = False, want_grad=True):
    """3D SSIM term of Eq. 6 over vol, gt [nz][ny][nx]: (loss device scalar,
    gradient or None); with accumulate the gradient is added to `grad`."""
    ws = ws or Workspace(vol.device)
    nz, ny, nx = vol.shape
    dims = (ctypes.c_int32 * 3)(nx, ny, nz)
    loss = torch.empty(1, device=vol.device)
    if want_grad and grad is None:
        grad = torch.empty_like(vol)
    ws.call(A.lib().fgs_ssim3d_loss_grad, A.ptr(vol.contiguous()), A.ptr(gt.contiguous()), dims, float(c1),
            float(c2), float(scale), A.ptr(loss), A.ptr(grad if want_grad else None), 1 if accumulate else 0)
    return loss, (grad if want_grad else None)


def tv_loss_grad(vol, *, scale: float = 1.0, ws: Workspace | None = None, want_grad=True, grad=None):
    """3D total variation of vol [nz][ny][nx] (TV term of Eq. 5) times scale:
    (loss device scalar, gradient or None)."""
    ws = ws or Workspace(vol.device, 1 << 16)
    nz, ny, nx = vol.shape
    dims = (ctypes.c_int32 * 3)(nx, ny, nz)
    loss = torch.empty(1, device=vol.device)
    if want_grad and grad is None:
        grad = torch.empty_like(vol)
    ws.call(A.lib().fgs_tv_loss_grad, A.ptr(vol.contiguous()), dims, float(scale), A.ptr(loss),
            A.ptr(grad if want_grad else None))
    return loss, (grad if want_grad else None)


def psnr(vol, ref, peak: float, ws: Workspace | None = None):
    L = A.lib()
    ws = ws or Workspace(vol.device, 1 << 16)
    out = torch.empty(1, dtype=torch.float32, device=vol.device)
    ws.call(L.fgs_psnr, A.ptr(vol), A.ptr(ref), vol.numel(), float(peak), A.ptr(out))
    return out


def adam_step(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-15,
              clamp_min_zero=False, grad2=None):
    """Adam on param with gradient grad (+ grad2 when given), in place."""
    L = A.lib()
    A.check(L.fgs_adam_step(A.ptr(param), A.ptr(grad), A.ptr(grad2), A.ptr(m), A.ptr(v), param.numel(), int(step),
                            float(lr), float(beta1), float(beta2), float(eps), int(clamp_min_zero),
                            A.stream_ptr(param.device)))


# ------------------------------------------------------------------ phantom

def _phantom(ph: dict) -> tuple:
    keep = [ph[k].contiguous() for k in ("centre", "semi", "quat", "amp")]
    for t in keep:
        if t.dtype != torch.float64:
            raise ValueError("phantom parameters are float64")
    return keep, A.fgs_phantom(keep[3].numel(), *(A.ptr(t) for t in keep))


def phantom_project(ph: dict, geom: Geometry, view_begin=0, view_count=None, out=None):
    L = A.lib()
    vc = geom.n_views - view_begin if view_count is None else view_count
    keep, s = _phantom(ph)
    dev = keep[0].device
    if out is None:
        out = torch.empty((vc, geom.det_h, geom.det_w), dtype=torch.float32, device=dev)
    gm = geom.struct()
    A.check(L.fgs_phantom_project(ctypes.byref(s), ctypes.byref(gm), view_begin, vc, A.ptr(out),
                                  A.stream_ptr(dev)))
    return out


def phantom_voxelize(ph: dict, grid: Grid, out=None):
    L = A.lib()
    keep, s = _phantom(ph)
    dev = keep[0].device
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    gd = grid.struct()
    A.check(L.fgs_phantom_voxelize(ctypes.byref(s), ctypes.byref(gd), A.ptr(out), A.stream_ptr(dev)))
    return out


# ------------------------------------------------------------------ initialisation (Sec. 3.1)

def fdk(img, geom: Geometry, grid: Grid, view_begin: int = 0, view_count: int | None = None,
        ws: Workspace | None = None, out=None):
    """FDK reconstruction of cone-beam projections img[V][H][W] on `grid`."""
    L = A.lib()
    vc = geom.n_views - view_begin if view_count is None else view_count
    ws = ws or Workspace(img.device)
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float32, device=img.device)
    gm = geom.struct()
    gd = grid.struct()
    ws.call(L.fgs_fdk, A.ptr(img.contiguous()), ctypes.byref(gm), view_begin, vc, ctypes.byref(gd), A.ptr(out))
    return out


def gradient_init(vol, grid: Grid, uniforms, *, background_fraction: float = 0.05, density_scale: float = 0.15,
                  min_scale: float = 1e-4, ws: Workspace | None = None, weighting: str = "gradient"):
    """FDK-gradient sampling initialisation: returns (mean, log_scale, quat,
    density) of n = uniforms.shape[1] Gaussians; uniforms is a float64 GPU
    tensor [4][n] of U[0, 1) variates. weighting="intensity" samples by the
    thresholded value instead of its gradient magnitude (fgs_intensity_init)."""
    L = A.lib()
    fn = {"gradient": L.fgs_gradient_init, "intensity": L.fgs_intensity_init}.get(weighting)
    if fn is None:
        raise ValueError("weighting must be 'gradient' or 'intensity'")
    if uniforms.dtype != torch.float64 or uniforms.dim() != 2 or uniforms.shape[0] != 4:
        raise ValueError("uniforms must be float64 [4][n]")
    n = uniforms.shape[1]
    dev = vol.device
    outs = (torch.empty((3, n), device=dev), torch.empty((3, n), device=dev), torch.empty((4, n), device=dev),
            torch.empty(n, device=dev))
    o = A.fgs_gaussian_grads(*(A.ptr(t) for t in outs))
    ws = ws or Workspace(dev)
    gd = grid.struct()
    ws.call(fn, A.ptr(vol.contiguous()), ctypes.byref(gd), float(background_fraction),
            float(density_scale), float(min_scale), n, A.ptr(uniforms.contiguous()), ctypes.byref(o))
    return outs


def reduce_max(x, ws: Workspace | None = None, out=None):
    """Device scalar max(x) (FP32), computed by the library."""
    ws = ws or Workspace(x.device, 1 << 16)
    out = torch.empty(1, device=x.device) if out is None else out
    ws.call(A.lib().fgs_reduce_max, A.ptr(x.contiguous()), x.numel(), A.ptr(out))
    return out


# ------------------------------------------------------------------ adaptive density control

def adc_accumulate(grad_mean, stat):
    """stat[2][n] += (|dL/dmean|, [|dL/dmean| > 0]) per Gaussian (in place)."""
    n = stat.shape[1]
    if stat.shape != (2, n) or grad_mean.shape != (3, n) or stat.dtype != torch.float32:
        raise ValueError("expected grad_mean [3][n] and stat float32 [2][n]")
    A.check(A.lib().fgs_adc_accumulate(A.ptr(grad_mean.contiguous()), n, A.ptr(stat),
                                       A.stream_ptr(stat.device)))


def adc_densify(params, m, v, stat, normals, *, grad_threshold: float, split_scale: float,
                prune_density: float, prune_scale: float, split_shrink: float = 1.6, n_max: int,
                ws: Workspace | None = None):
    """One densification step (fgs_adc_densify). params, m, v: lists of the
    four SoA tensors; stat [2][n]; normals float32 [6][n] standard normal
    variates. Returns (params, m, v) at the new count."""
    n = params[3].numel()
    dev = params[3].device
    if normals.shape != (6, n) or normals.dtype != torch.float32:
        raise ValueError("normals must be float32 [6][n]")
    rows = (3, 3, 4, 1)
    bufs = [[torch.empty(r * n_max, device=dev) for r in rows] for _ in range(3)]
    outs = [A.fgs_gaussian_grads(*(A.ptr(t) for t in b)) for b in bufs]
    g = _gauss(*params)
    gm = A.fgs_gaussian_grads(*(A.ptr(t) for t in m))
    gv = A.fgs_gaussian_grads(*(A.ptr(t) for t in v))
    prm = A.fgs_adc_params(float(grad_threshold), float(split_scale), float(prune_density), float(prune_scale),
                           float(split_shrink), 0, int(n_max))
    n_out = ctypes.c_int64(0)
    ws = ws or Workspace(dev)
    ws.call(A.lib().fgs_adc_densify, ctypes.byref(g), ctypes.byref(gm), ctypes.byref(gv), A.ptr(stat.contiguous()),
            A.ptr(normals.contiguous()), ctypes.byref(prm), ctypes.byref(outs[0]), ctypes.byref(outs[1]),
            ctypes.byref(outs[2]), ctypes.byref(n_out))
    k = int(n_out.value)

    def shaped(b):
        return [b[0][:3 * k].view(3, k), b[1][:3 * k].view(3, k), b[2][:4 * k].view(4, k), b[3][:k]]
    return shaped(bufs[0]), shaped(bufs[1]), shaped(bufs[2])


# ------------------------------------------------------------------ introspection

def binning_dump(ws: Workspace) -> dict:
    """Views of the binning arrays the last forward call left in ``ws``
    (rasterizer: per-tile [begin, end) ranges; voxelizer: tile starts)."""
    L = A.lib()
    off = (ctypes.c_uint64 * 9)()
    cnt = (ctypes.c_uint64 * 3)()
    A.check(L.fgs_binning_layout(ctypes.byref(ws.s), off, cnt))
    R, K, T = (int(c) for c in cnt)
    buf = ws.buf
    vox = ws.s.kind == 2

    def view(i, dtype, count, width=1):
        nbytes = torch.tensor([], dtype=dtype).element_size() * count * width
        t = buf[int(off[i]):int(off[i]) + nbytes].view(dtype)
        return t.view(count, width) if width > 1 else t

    sorted_keys, sorted_vals = view(6, torch.int32, K), view(7, torch.int32, K)
    rb = int(ws.s.record_bits) if not vox else 0
    if rb:
        # one-word lists: word = tile << record_bits | record; the key is
        # (record / n_gauss) << tile_bits | tile, the value the record
        w = sorted_keys.to(torch.int64) & 0xffffffff
        rec = w & ((1 << rb) - 1)
        sorted_keys = (((rec // int(ws.s.n_gauss)) << int(ws.s.tile_bits)) | (w >> rb)).to(torch.int32)
        sorted_vals = rec.to(torch.int32)
    return dict(
        centre=view(0, torch.float32, R, 4 if vox else 2),
        radii=view(1, torch.float32, R, 4 if vox else 2),
        rect=view(2, torch.int16, R, 8 if vox else 4),
        offset=view(3, torch.int32, R + 1),
        sorted_keys=sorted_keys,
        sorted_vals=sorted_vals,
        **({"tile_start": view(8, torch.int32, T + 1)} if vox else
           {"tile_ranges": view(8, torch.int32, T, 2), "tile_bits": int(ws.s.tile_bits)}),
        n_records=R, n_pairs=K, n_tiles=T)


# ------------------------------------------------------------------ autograd

class ProjectViews(torch.autograd.Function):
    """Differentiable rasterizer; the backward is libfactgs' hand-written one."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, density, geom: Geometry, view_begin: int, view_count: int,
                kappa: float = KAPPA, ws: Workspace | None = None, recompute: bool = True, model: str = "splat"):
        ws = ws or Workspace(mean.device)
        img = project_views(mean, log_scale, quat, density, geom, view_begin, view_count, kappa=kappa, ws=ws,
                            model=model)
        ctx.save_for_backward(mean, log_scale, quat, density)
        ctx.geom, ctx.vb, ctx.vc, ctx.kappa, ctx.ws, ctx.recompute = geom, view_begin, view_count, kappa, ws, recompute
        ctx.model = model
        return img

    @staticmethod
    def backward(ctx, grad_img):
        mean, log_scale, quat, density = ctx.saved_tensors
        g = project_views_backward(mean, log_scale, quat, density, ctx.geom, grad_img.contiguous(), ctx.vb,
                                   ctx.vc, kappa=ctx.kappa, recompute=ctx.recompute, ws=ctx.ws, model=ctx.model)
        return (*g, None, None, None, None, None, None, None)


class Voxelize(torch.autograd.Function):
    """Differentiable voxelizer; the backward is libfactgs' hand-written one."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, density, grid: Grid, kappa: float = KAPPA,
                ws: Workspace | None = None, recompute: bool = True):
        ws = ws or Workspace(mean.device)
        vol = voxelize(mean, log_scale, quat, density, grid, kappa=kappa, ws=ws)
        ctx.save_for_backward(mean, log_scale, quat, density)
        ctx.grid, ctx.kappa, ctx.ws, ctx.recompute = grid, kappa, ws, recompute
        return vol

    @staticmethod
    def backward(ctx, grad_vol):
        mean, log_scale, quat, density = ctx.saved_tensors
        g = voxelize_backward(mean, log_scale, quat, density, ctx.grid, grad_vol.contiguous(), kappa=ctx.kappa,
                              recompute=ctx.recompute, ws=ctx.ws)
        return (*g, None, None, None, None)
