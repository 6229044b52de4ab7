"""Benchmark of the FaCT-GS hot path on one MI355X.

One step = one pass of the whole hot path over the standard-scan workload
(the paper's 75-view 512^2 setting, Sec. 4.1, with 50,000 Gaussians and a
256^3 voxel grid):
  rasterizer forward over all 75 views -> L1 loss and gradient against the
  phantom's exact projections -> rasterizer backward (lists reused) ->
  voxelizer forward at 256^3 -> L1 against the phantom volume -> voxelizer
  backward -> one Adam step on all 11 N parameters (both gradients fused).

Prints ONE JSON line. `value` is view-pixels processed per second of whole
steps (75 * 512^2 per step); `voxels_per_s` the same for the 256^3 grid.
`roofline` is for the step's dominant kernel, timed with HIP events that the
library records around it on the stream it runs on; its work is the exact
number of (pixel|voxel, Gaussian) support pairs, counted on the GPU.
`cpu_baseline` times the FP64 oracle on a bounded sample of the same step
on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd view-pixels/s and voxels/s; s/iter and s-to-PSNR at 75×512² views"

# Algorithmic FP32 operations per support pair (an exponential counts as one):
#   rasterizer forward : offset 2, quadratic form 7, exp 1, weight and sum 2        = 12
#   rasterizer backward: offset 2, quadratic form 7, exp 1, g*e 1, six moments 11   = 22
#   voxelizer forward  : offset 3, quadratic form 14, exp 1, weight and sum 2       = 20
#   voxelizer backward : offset 3, quadratic form 14, exp 1, g*e 1, ten moments 19  = 38
FLOPS_PER_PAIR = {"splat_fwd": 12, "splat_bwd": 22, "vox_fwd": 20, "vox_bwd": 38}
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(gs, gd, ang, grid_d, budget_views=4, budget_slices=16, budget_gauss=2000):
    """Time the FP64 oracle on a bounded sample of one step and scale it to the
    whole step: `budget_views` of the 75 views (forward + backward over all
    Gaussians), `budget_slices` z-slices of the 256^3 voxelizer forward and
    the voxelizer backward of `budget_gauss` Gaussians."""
    import oracle
    oracle.build(force=False)
    n_views = len(ang)
    nx, ny, nz = grid_d["dims"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c = np.ones((budget_views, gd["det_h"], gd["det_w"])) / (gd["det_h"] * gd["det_w"])
    t0 = time.perf_counter()
    oracle.project(gs, gd, ang[:budget_views])
    t1 = time.perf_counter()
    oracle.project_bwd(gs, gd, ang[:budget_views], c)
    t2 = time.perf_counter()
    slab = dict(origin=grid_d["origin"], spacing=grid_d["spacing"], dims=(nx, ny, budget_slices))
    oracle.voxelize(gs, slab)
    t3 = time.perf_counter()
    n = gs["density"].shape[0]
    sel = np.random.default_rng(0).choice(n, budget_gauss, replace=False)
    gv = np.ones((nz, ny, nx)) / (nx * ny * nz)
    t4 = time.perf_counter()
    oracle.voxelize_bwd(gs, grid_d, gv, sel=sel)
    t5 = time.perf_counter()
    step_s = ((t1 - t0) + (t2 - t1)) * n_views / budget_views + (t3 - t2) * nz / budget_slices \
        + (t5 - t4) * n / budget_gauss
    sampled = (t2 - t0) + (t3 - t2) + (t5 - t4)
    return dict(value=n_views * gd["det_w"] * gd["det_h"] / step_s, unit="view-pixels/s", cores=cores,
                kind="oracle",
                sample=(f"FP64 oracle, {budget_views} of {n_views} views rasterized forward+backward over all "
                        f"{n} Gaussians, {budget_slices} of {nz} z-slices voxelized, voxelizer backward of "
                        f"{budget_gauss} of {n} Gaussians; {sampled:.1f} s measured, scaled linearly to one "
                        f"step ({step_s:.1f} s)"),
                seconds_per_step=step_s)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy a MIB-MiB float32 buffer device-to-device 3 times "
                         "(a plain copy kernel of known size, to scale HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_01844_amd as fgs
    import synth_inputs as si

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = si.CONFIGS["scan"]
    N, V, D, NV = cfg["n_gauss"], cfg["n_views"], cfg["det"], cfg["vol"]
    gs = si.gaussians(N, cfg["seed"])
    gd = si.geometry(D)
    ang = si.angles(V)
    grid_d = si.grid(NV)
    geom = fgs.Geometry.from_dict(gd, ang, dev)
    grid = fgs.Grid.from_dict(grid_d)
    ph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in si.phantom(cfg["n_ell"],
                                                                                       cfg["phantom_seed"]).items()}
    log(f"workload: {N} Gaussians, {V} views {D}x{D}, {NV}^3 voxels")
    i_gt = fgs.phantom_project(ph, geom)
    v_gt = fgs.phantom_voxelize(ph, grid)

    params = [torch.from_numpy(gs[k]).to(dev) for k in ("mean", "log_scale", "quat", "density")]
    lrs = [2e-4, 5e-3, 1e-3, 1e-2]
    moms = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    gp = [torch.empty_like(p) for p in params]
    gv = [torch.empty_like(p) for p in params]
    img = torch.empty((V, D, D), device=dev)
    vol = torch.empty(grid.shape, device=dev)
    ws_p, ws_v, ws_l = fgs.Workspace(dev), fgs.Workspace(dev), fgs.Workspace(dev, 1 << 16)
    names = ("splat_fwd", "splat_bwd", "vox_fwd", "vox_bwd")
    state = {"step": 0}

    def step(ev=None):
        e = ev or {}
        fgs.project_views(*params, geom, ws=ws_p, out=img, events=e.get("splat_fwd"))
        _, g_img = fgs.l1_loss_grad(img, i_gt, ws=ws_l)
        fgs.project_views_backward(*params, geom, g_img, recompute=False, ws=ws_p, out=gp,
                                   events=e.get("splat_bwd"))
        fgs.voxelize(*params, grid, ws=ws_v, out=vol, events=e.get("vox_fwd"))
        _, g_vol = fgs.l1_loss_grad(vol, v_gt, n_views=1, ws=ws_l)
        fgs.voxelize_backward(*params, grid, g_vol, recompute=False, ws=ws_v, out=gv, events=e.get("vox_bwd"))
        state["step"] += 1
        for k, p in enumerate(params):
            fgs.adam_step(p, gp[k], moms[k][0], moms[k][1], state["step"], lrs[k], grad2=gv[k],
                          clamp_min_zero=(k == 3))

    pairs0 = {"splat": fgs.project_views_support(*params, geom), "vox": fgs.voxelize_support(*params, grid)}
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    evs = [{n: fgs.timing_events() for n in names} for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    t_start.record()
    wall0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    t_stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_stop)
    ms_step = ms_total / args.steps
    kern_ms = {n: float(np.mean([e[n][0].elapsed_time(e[n][1]) for e in evs])) for n in names}
    pairs1 = {"splat": fgs.project_views_support(*params, geom), "vox": fgs.voxelize_support(*params, grid)}
    pairs = {k: 0.5 * (pairs0[k] + pairs1[k]) for k in pairs0}
    log(f"timed: {ms_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}); kernels {kern_ms}")

    kernels = {}
    for n in names:
        pr = pairs["splat" if n.startswith("splat") else "vox"]
        tf = pr * FLOPS_PER_PAIR[n] / (kern_ms[n] * 1e-3) / 1e12
        kernels[n] = dict(ms=round(kern_ms[n], 4), support_pairs=int(pr),
                          pairs_per_s=pr / (kern_ms[n] * 1e-3), tflops=round(tf, 3))
    dom = max(names, key=lambda n: kern_ms[n])
    roof = dict(bound="alu", achieved=round(kernels[dom]["tflops"], 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(kernels[dom]["tflops"] / PEAK_FP32_TFLOPS, 4), traffic=None, kernel=dom,
                flops_per_pair=FLOPS_PER_PAIR[dom], support_pairs=int(pairs["splat" if dom.startswith("splat")
                                                                             else "vox"]))
    out = dict(metric=METRIC, value=V * D * D / (ms_step * 1e-3), unit="view-pixels/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"standard scan: {N} Gaussians, {V} cone-beam views {D}x{D} "
                                    f"(SOD 1.5, SDD 2.0), voxelizer {NV}^3; rasterizer and voxelizer "
                                    f"fwd+bwd, L1 losses and Adam per step",
                           n_gauss=N, views=V, det=D, vol=NV),
               voxels_per_s=NV ** 3 / (ms_step * 1e-3),
               s_per_step=ms_step * 1e-3,
               kernels=kernels, roofline=roof)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(gs, gd, ang, grid_d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
