"""Optimisation loops over the library's kernels: CT reconstruction from
projections (Sec. 3.4) and fitting Gaussians to a volume (Sec. 3.6).

Both are thin drivers. Every numerical step runs in libfactgs:
- the rasterizer or voxelizer forward and backward;
- the L1 loss and its gradient;
- Adam;
- PSNR;
- FDK and the gradient-sampling initialisation.

Python only orders the calls, draws the view order and keeps the clock.

Reconstruction follows the paper's loop with the loss of Eq. 5:
- one view per optimizer step, views in a fresh random order each epoch;
- L1 plus, with ssim_weight > 0, ssim_weight * (1 - SSIM) on the view;
- with a CropTV, each step also voxelizes a randomly placed 32^3 crop of
  the reconstruction grid and adds the gradient of tv_weight * TV(crop);
- a paper "iteration" is one pass over all views (its Table 1 times grow
  linearly with the number of views at a fixed iteration count).

The paper prints no weights; the defaults used in this package's
experiments are stated where they are set.

Fitting follows Sec. 3.6 with the L1 term of Eq. 6:
- initialise by gradient sampling on the target volume;
- each step voxelizes the whole grid, takes L1 against the target,
  backpropagates and applies Adam.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from . import ops


@dataclass
class AdamConfig:
    """Per-group learning rates (the paper gives none; these are tuned on the
    synthetic scans)."""
    lr_mean: float = 2e-4
    lr_log_scale: float = 5e-3
    lr_quat: float = 1e-3
    lr_density: float = 5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def lrs(self):
        return (self.lr_mean, self.lr_log_scale, self.lr_quat, self.lr_density)


# Learning rates for fitting Gaussians to a volume (Sec. 3.6): tuned on
# 128^3 / 50k and 256^3 / 200k phantom fits (about 49 dB after 200 steps).
FIT_ADAM = AdamConfig(lr_mean=1e-3, lr_log_scale=2e-2, lr_quat=5e-3, lr_density=2e-2)


@dataclass
class ADCConfig:
    """Adaptive density control during reconstruction (Sec. 3.4; the count is
    capped at `cap` times the initial one, Suppl. C). The paper gives no
    schedule or thresholds; these are this library's choices."""
    every: int = 75              # optimiser steps between densifications
    start: int = 150             # no densification before this step
    stop: int = 3750             # nor after this one
    grad_threshold: float = 2e-4 # mean |dL/dmean| over the steps a Gaussian was seen
    split_scale: float = 0.02    # largest standard deviation above which candidates split
    prune_density: float = 1e-3
    prune_scale: float = 0.25
    split_shrink: float = 1.6
    cap: float = 1.1
    seed: int = 0


class GaussianModel:
    """Gaussian parameters (float32 SoA on the GPU) with their Adam state."""

    def __init__(self, mean, log_scale, quat, density):
        self.params = [t.contiguous() for t in (mean, log_scale, quat, density)]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.grads = [torch.empty_like(p) for p in self.params]
        self.grads2 = [torch.empty_like(p) for p in self.params]
        self.step = 0

    @property
    def n(self) -> int:
        return self.params[3].numel()

    def replace(self, params, m, v):
        """Take new parameters and moments (e.g. after densification); the
        step count is kept, gradient buffers follow the new size."""
        self.params, self.m, self.v = list(params), list(m), list(v)
        self.grads = [torch.empty_like(p) for p in self.params]
        self.grads2 = [torch.empty_like(p) for p in self.params]

    def adam(self, cfg: AdamConfig, second: bool = False):
        """One Adam step with the gradient in `grads` (+ `grads2`)."""
        self.step += 1
        for k, (p, lr) in enumerate(zip(self.params, cfg.lrs())):
            ops.adam_step(p, self.grads[k], self.m[k], self.v[k], self.step, lr, cfg.beta1, cfg.beta2, cfg.eps,
                          clamp_min_zero=(k == 3), grad2=self.grads2[k] if second else None)

    def state_dict(self) -> dict:
        names = ("mean", "log_scale", "quat", "density")
        out = {n: p.detach().cpu().numpy() for n, p in zip(names, self.params)}
        out.update({f"m_{n}": t.cpu().numpy() for n, t in zip(names, self.m)})
        out.update({f"v_{n}": t.cpu().numpy() for n, t in zip(names, self.v)})
        out["step"] = np.array(self.step)
        return out

    @classmethod
    def from_state_dict(cls, d: dict, device="cuda") -> "GaussianModel":
        names = ("mean", "log_scale", "quat", "density")
        g = cls(*(torch.from_numpy(np.asarray(d[n], dtype=np.float32)).to(device) for n in names))
        for k, n in enumerate(names):
            g.m[k].copy_(torch.from_numpy(np.asarray(d[f"m_{n}"], dtype=np.float32)))
            g.v[k].copy_(torch.from_numpy(np.asarray(d[f"v_{n}"], dtype=np.float32)))
        g.step = int(d["step"])
        return g


@dataclass
class History:
    epochs: list = field(default_factory=list)
    seconds: list = field(default_factory=list)   # optimisation clock (evaluation excluded)
    psnr: list = field(default_factory=list)
    loss: list = field(default_factory=list)
    overflows: int = 0                            # step-capacity overflows seen (ViewStep)

    def seconds_to(self, target: float):
        for s, p in zip(self.seconds, self.psnr):
            if p >= target:
                return s
        return None


def init_from_volume(vol, grid: ops.Grid, n: int, uniforms, *, background_fraction=0.05,
                     density_scale=0.15, weighting="gradient") -> GaussianModel:
    """Gradient-sampling initialisation (Sec. 3.1) from a volume on the GPU;
    uniforms is a float64 [4][>= n] array or device tensor of U[0, 1) draws.
    weighting="intensity" gives the intensity-sampling baseline."""
    if isinstance(uniforms, torch.Tensor):
        u = uniforms[:, :n].to(vol.device, torch.float64).contiguous()
    else:
        u = torch.from_numpy(np.ascontiguousarray(uniforms[:, :n], dtype=np.float64)).to(vol.device)
    mean, ls, q, d = ops.gradient_init(vol, grid, u, background_fraction=background_fraction,
                                       density_scale=density_scale, min_scale=0.25 * min(grid.spacing),
                                       weighting=weighting)
    return GaussianModel(mean, ls, q, d)


class CropTV:
    """The per-step TV prior of Eq. 5: a crop of `size`^3 voxels of `grid`,
    placed uniformly at random, voxelized, and weight * TV(crop) added to the
    step's gradient through the voxelizer backward."""

    def __init__(self, grid: ops.Grid, weight: float, size: int = 32, device="cuda"):
        self.grid, self.weight, self.size = grid, float(weight), size
        self.ws = ops.Workspace(device)
        self.ws_l = ops.Workspace(device, 1 << 16)
        self.vol = torch.empty((size, size, size), device=device)
        self.grad = torch.empty_like(self.vol)

    def crop(self, rng) -> ops.Grid:
        off = [int(rng.integers(0, d - self.size + 1)) for d in self.grid.dims]
        origin = tuple(float(np.float32(o + k * h)) for o, k, h in zip(self.grid.origin, off, self.grid.spacing))
        return ops.Grid(origin, self.grid.spacing, (self.size,) * 3)

    def add_grad(self, params, grads, rng):
        """Add the gradient of weight * TV(random crop) to `grads` (the four
        parameter gradient tensors); returns the TV term (device scalar)."""
        g = self.crop(rng)
        ops.voxelize(*params, g, ws=self.ws, out=self.vol)
        loss, _ = ops.tv_loss_grad(self.vol, scale=self.weight, ws=self.ws_l, grad=self.grad)
        ops.voxelize_backward(*params, g, self.grad, recompute=False, ws=self.ws, out=grads, accumulate=True)
        return loss


class ViewStep:
    """One optimiser step of the reconstruction loop as a single library call
    (fgs_recon_step): forward of one view, L1 (+ SSIM) of Eq. 5, backward,
    the optional crop TV, Adam on all parameters.

    The rasterizer and crop workspaces run with a fixed key capacity, so no
    step waits for the GPU: the rasterizer's is `key_margin` times the pairs
    of view 0 at construction, the crop's `crop_keys`. A step whose pairs
    exceed its capacity bins nothing (a zero image, no gradient from it);
    check_overflow() (which waits for the GPU) reports that and raises the
    capacity for the steps after it.

    graphs=True: each view's step is captured once in a HIP graph
    (fgs_step_graph_capture) and replayed on later steps of that view
    (fgs_step_graph_launch), with the same result bit for bit and without the
    per-kernel launch cost. The graphs are dropped and captured again when a
    workspace is reallocated, a capacity changes or the model's tensors move
    (adaptive density control), or another gt tensor is passed for a view."""

    def __init__(self, model: GaussianModel, geom: ops.Geometry, adam: AdamConfig, *, ssim_weight: float = 0.0,
                 tv: "CropTV | None" = None, kappa: float = ops.KAPPA, near: float = ops.NEAR,
                 key_margin: float = 2.0, crop_keys: int = 1 << 18, graphs: bool = True):
        dev = model.params[0].device
        self.model, self.geom, self.adam, self.tv = model, geom, adam, tv
        self.H, self.W = geom.det_h, geom.det_w
        self.img = torch.empty((self.H, self.W), device=dev)
        self.grad_img = torch.empty_like(self.img)
        self.loss = torch.zeros(3, device=dev)
        self.params_blk = torch.zeros(8, device=dev)
        self.ws_proj = ops.Workspace(dev)
        self.ws_crop = ops.Workspace(dev)
        self.ws_loss = ops.Workspace(dev, 12 * self.H * self.W + 44 * model.n + (1 << 16))
        ops.project_views(*model.params, geom, 0, 1, kappa=kappa, near=near, ws=self.ws_proj)
        self.ws_proj.set_capacity(int(key_margin * self.ws_proj.n_pairs) + 4096)
        if tv is not None:
            self.ws_crop.set_capacity(crop_keys)
        self.opts = ops._opts(kappa, near)
        self.gm = geom.struct()
        self.sp = A.fgs_step_params(float(ssim_weight), ops.SSIM_C1, ops.SSIM_C2,
                                    float(tv.weight) if tv is not None else 0.0, (ctypes.c_float * 4)(*adam.lrs()),
                                    adam.beta1, adam.beta2, adam.eps, 0)
        self.use_graphs = graphs
        self._graphs = {}       # view -> (graph handle, gt pointer)
        self._bound = None

    def _drop_graphs(self):
        L = A.lib()
        for h, _ in self._graphs.values():
            A.check(L.fgs_step_graph_destroy(h))
        self._graphs = {}

    def __del__(self):
        try:
            if self._graphs:
                torch.cuda.synchronize()
                self._drop_graphs()
        except Exception:
            pass

    def _bind(self):
        m = self.model
        key = tuple(t.data_ptr() for t in (*m.params, *m.m, *m.v, *m.grads))
        if key != self._bound:
            self._p = A.fgs_gaussian_grads(*(A.ptr(t) for t in m.params))
            self._m = A.fgs_gaussian_grads(*(A.ptr(t) for t in m.m))
            self._v = A.fgs_gaussian_grads(*(A.ptr(t) for t in m.v))
            self._g = A.fgs_gaussian_grads(*(A.ptr(t) for t in m.grads))
            if self._bound is not None and self._graphs:
                torch.cuda.synchronize()
                self._drop_graphs()
            self._bound = key
        tv = self.tv
        self._buf = A.fgs_step_buffers(A.ptr(self.img), A.ptr(self.grad_img),
                                       A.ptr(tv.vol) if tv is not None else None,
                                       A.ptr(tv.grad) if tv is not None else None, A.ptr(self.loss),
                                       A.ptr(self.params_blk))

    def _args(self, view, gt_view, crop):
        m = self.model
        return (ctypes.byref(self._p), ctypes.byref(self._m), ctypes.byref(self._v), ctypes.byref(self._g), m.n,
                ctypes.byref(self.gm), int(view), A.ptr(gt_view), ctypes.byref(crop) if crop is not None else None,
                ctypes.byref(self.opts), ctypes.byref(self.sp), ctypes.byref(self._buf),
                ctypes.byref(self.ws_proj.s), ctypes.byref(self.ws_crop.s), ctypes.byref(self.ws_loss.s))

    def _grow(self) -> bool:
        """Grows the workspaces a call asked more of; True if any moved."""
        moved = False
        for w in (self.ws_proj, self.ws_loss, self.ws_crop):
            if w.buf is None or int(w.s.needed) > w.buf.numel():
                w.ensure(max(int(w.s.needed), 1 << 20))
                moved = True
        if moved and self._graphs:
            torch.cuda.synchronize()
            self._drop_graphs()
        return moved

    def _graph(self, view: int, gt_view, crop):
        hit = self._graphs.get(view)
        if hit is not None and hit[1] == gt_view.data_ptr():
            return hit[0]
        if hit is not None:
            torch.cuda.synchronize()
            A.check(A.lib().fgs_step_graph_destroy(hit[0]))
            del self._graphs[view]
        L = A.lib()
        for _ in range(6):
            h = ctypes.c_void_p()
            code = L.fgs_step_graph_capture(*self._args(view, gt_view, crop), ctypes.byref(h))
            if code != A.FGS_E_CAPACITY:
                A.check(code)
                self._graphs[view] = (h, gt_view.data_ptr())
                return h
            self._grow()
        raise A.FgsError(A.FGS_E_CAPACITY, "step workspaces did not converge")

    def __call__(self, view: int, gt_view, rng=None):
        """Step on view `view` against gt_view[H][W] (device, contiguous); rng
        places the crop. Returns the device loss terms [L1, SSIM, TV]."""
        self._bind()
        m = self.model
        crop = self.tv.crop(rng).struct() if self.tv is not None else None
        self.sp.step = m.step + 1
        L = A.lib()
        stream = A.stream_ptr(self.img.device)
        if self.use_graphs:
            h = self._graph(view, gt_view, crop)
            A.check(L.fgs_step_graph_launch(h, ctypes.byref(self.sp),
                                            ctypes.byref(crop) if crop is not None else None, stream))
            m.step += 1
            return self.loss
        for _ in range(6):
            code = L.fgs_recon_step(*self._args(view, gt_view, crop), stream)
            if code != A.FGS_E_CAPACITY:
                A.check(code)
                m.step += 1
                return self.loss
            self._grow()
        raise A.FgsError(A.FGS_E_CAPACITY, "step workspaces did not converge")

    def check_overflow(self) -> int:
        """Waits for the GPU. Number of workspaces whose capacity some step
        since the last check exceeded (those steps binned nothing); each such
        capacity is raised to 1.5 times the largest need seen (which drops
        the captured graphs)."""
        hit = 0
        for w in (self.ws_proj, self.ws_crop):
            f, need = w.overflowed()
            if f:
                hit += 1
                w.set_capacity(int(1.5 * need) + 4096)
        if hit and self._graphs:
            self._drop_graphs()
        return hit


def reconstruct(model: GaussianModel, proj_gt, geom: ops.Geometry, *, epochs: int, adam: AdamConfig,
                vol_gt=None, eval_grid: ops.Grid | None = None, eval_every: int = 1,
                target_psnr: float | None = None, seed: int = 0, clock_start: float | None = None,
                t_offset: float = 0.0, eval_at_start: bool = False, tv: CropTV | None = None,
                ssim_weight: float = 0.0, adc: ADCConfig | None = None, graphs: bool = True) -> History:
    """Optimise `model` against projections proj_gt[V][H][W] (GPU), one view
    per step. If vol_gt/eval_grid are given, PSNR is evaluated every
    `eval_every` epochs (and before the first step with eval_at_start),
    outside the clock, and the loop stops at target_psnr. The clock starts
    at t_offset seconds (time already spent, e.g. on the initialisation).
    graphs: each view's step is captured in a HIP graph on its first step and
    replayed after (ViewStep); the captures are inside the clock."""
    dev = proj_gt.device
    V = proj_gt.shape[0]
    ws_p, ws_l, ws_v = ops.Workspace(dev), ops.Workspace(dev, 1 << 16), ops.Workspace(dev)
    ws_s = ops.Workspace(dev)
    img = torch.empty((1, geom.det_h, geom.det_w), device=dev)
    vol = torch.empty(eval_grid.shape, device=dev) if eval_grid is not None else None
    peak = float(vol_gt.max().item()) if vol_gt is not None else 1.0
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = History()
    torch.cuda.synchronize()
    t_run = t_offset
    if vol_gt is not None and eval_at_start:
        ops.voxelize(*model.params, eval_grid, ws=ws_v, out=vol)
        hist.epochs.append(0)
        hist.seconds.append(t_run)
        hist.psnr.append(float(ops.psnr(vol, vol_gt, peak, ws=ws_l).item()))
        hist.loss.append(float("nan"))
        if target_psnr is not None and hist.psnr[-1] >= target_psnr:
            return hist
        torch.cuda.synchronize()
    dens = _Densifier(model, adc, dev) if adc is not None else None
    # without density control a step is one library call that never waits
    stepper = ViewStep(model, geom, adam, ssim_weight=ssim_weight, tv=tv, graphs=graphs) if dens is None else None
    if stepper is not None and clock_start is None:
        torch.cuda.synchronize()
    t0 = time.perf_counter() if clock_start is None else clock_start
    for ep in range(1, epochs + 1):
        for v in rng.permutation(V):
            if stepper is not None:
                loss = stepper(int(v), proj_gt[v], rng)[0:1]
                continue
            ops.project_views(*model.params, geom, int(v), 1, ws=ws_p, out=img)
            loss, g = ops.l1_loss_grad(img, proj_gt[v:v + 1], ws=ws_l)
            if ssim_weight > 0:
                ops.ssim_loss_grad(img, proj_gt[v:v + 1], scale=ssim_weight, ws=ws_s, grad=g, accumulate=True)
            ops.project_views_backward(*model.params, geom, g, int(v), 1, recompute=False, ws=ws_p,
                                       out=model.grads)
            if tv is not None:
                tv.add_grad(model.params, model.grads, rng)
            if dens is not None:
                dens.observe()
            model.adam(adam)
            if dens is not None:
                dens.maybe_densify()
        if vol_gt is not None and (ep % eval_every == 0 or ep == epochs):
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            ops.voxelize(*model.params, eval_grid, ws=ws_v, out=vol)
            p = float(ops.psnr(vol, vol_gt, peak, ws=ws_l).item())
            hist.epochs.append(ep)
            hist.seconds.append(t_run)
            hist.psnr.append(p)
            hist.loss.append(float(loss.item()))
            if stepper is not None:
                hist.overflows += stepper.check_overflow()
            if target_psnr is not None and p >= target_psnr:
                break
            torch.cuda.synchronize()
            t0 = time.perf_counter()
    return hist


class _Densifier:
    """Gradient statistics and the densification schedule of ADCConfig."""

    def __init__(self, model: GaussianModel, cfg: ADCConfig, dev):
        self.model, self.cfg, self.dev = model, cfg, dev
        self.n_max = int(cfg.cap * model.n)
        self.stat = torch.zeros((2, model.n), device=dev)
        self.rng = np.random.Generator(np.random.PCG64(cfg.seed))
        self.ws = ops.Workspace(dev)
        self.steps = 0
        self.counts = []

    def observe(self):
        ops.adc_accumulate(self.model.grads[0], self.stat)

    def maybe_densify(self):
        self.steps += 1
        c = self.cfg
        if self.steps < c.start or self.steps > c.stop or self.steps % c.every:
            return
        m = self.model
        z = torch.from_numpy(self.rng.standard_normal((6, m.n), dtype=np.float32)).to(self.dev)
        p, mo, vo = ops.adc_densify(m.params, m.m, m.v, self.stat, z, grad_threshold=c.grad_threshold,
                                    split_scale=c.split_scale, prune_density=c.prune_density,
                                    prune_scale=c.prune_scale, split_shrink=c.split_shrink, n_max=self.n_max,
                                    ws=self.ws)
        m.replace(p, mo, vo)
        self.stat = torch.zeros((2, m.n), device=self.dev)
        self.counts.append(m.n)


def fit_volume(model: GaussianModel, vol_gt, grid: ops.Grid, *, iters: int, adam: AdamConfig,
               eval_every: int = 10, ssim_weight: float = 0.0) -> History:
    """Fit `model` to vol_gt on `grid` (Sec. 3.6, Eq. 6): voxelize, L1 plus
    (with ssim_weight > 0) ssim_weight * (1 - 3D SSIM), voxelizer backward,
    Adam, each step over the whole grid."""
    dev = vol_gt.device
    ws_v, ws_l = ops.Workspace(dev), ops.Workspace(dev, 1 << 16)
    ws_s = ops.Workspace(dev)
    vol = torch.empty(grid.shape, device=dev)
    peak = float(vol_gt.max().item())
    hist = History()
    torch.cuda.synchronize()
    t_run = 0.0
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        ops.voxelize(*model.params, grid, ws=ws_v, out=vol)
        loss, g = ops.l1_loss_grad(vol, vol_gt, n_views=1, ws=ws_l)
        if ssim_weight > 0:
            ops.ssim3d_loss_grad(vol, vol_gt, scale=ssim_weight, ws=ws_s, grad=g, accumulate=True)
        ops.voxelize_backward(*model.params, grid, g, recompute=False, ws=ws_v, out=model.grads)
        model.adam(adam)
        if it % eval_every == 0 or it == iters:
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            ops.voxelize(*model.params, grid, ws=ws_v, out=vol)
            hist.epochs.append(it)
            hist.seconds.append(t_run)
            hist.psnr.append(float(ops.psnr(vol, vol_gt, peak, ws=ws_l).item()))
            hist.loss.append(float(loss.item()))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
    return hist
