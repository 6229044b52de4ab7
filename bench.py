"""Benchmark of the FaCT-GS hot path on one MI355X.

One step = one pass of the whole hot path over one workload:
  rasterizer forward over all views -> L1 loss and gradient against the
  phantom's exact projections -> rasterizer backward -> voxelizer forward
  over the whole grid -> L1 against the phantom volume -> voxelizer backward
  -> one Adam step on all 11 N parameters (both gradients fused).

Workloads (synthetic, seeded; they stand in for the paper's datasets):
  scan  (default) 50,000 Gaussians, 75 cone-beam views of 512^2, 256^3 voxels;
        all views in one library call, the backward reuses the forward's lists.
  scale 500,000 Gaussians, 50 views of 2048^2, 512^3 voxels; 10 views per
        library call, lists rebuilt in the backward.

Prints ONE JSON line. `value` is view-pixels per second of whole steps;
`voxels_per_s` the same for the voxel grid. For the scan workload the
one-view optimisation step of the reconstruction loop (Sec. 3.4, the loss
of Eq. 5: forward for one view, L1 and SSIM with their gradients, backward,
a randomly placed 32^3 crop voxelized with the gradient of its total
variation, then Adam) is also timed over one epoch of 75 steps
(`s_per_view_step`, `s_per_epoch`). `roofline` is for the step's dominant
kernel, timed with HIP events that the library records around it on the
stream it runs on; its work is the exact number of (pixel|voxel, Gaussian)
support pairs, counted on the GPU. `cpu_baseline` times the FP64 oracle on a
bounded sample of the same step on the host cores.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
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
# FP32 vector peak this build can reach: 256 CUs x 64 FMA lanes per clock x
# 2 flops x 2.4 GHz. The published 157.3 TFLOP/s counts two-wide packed FP32
# instructions, which the library is compiled without.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
NAMES = ("splat_fwd", "splat_bwd", "vox_fwd", "vox_bwd")
WORKLOADS = {
    "scan": dict(config="scan", views_per_call=None, recompute=False,
                 label="standard scan: {N} Gaussians, {V} cone-beam views {D}x{D} (SOD 1.5, SDD 2.0), voxelizer "
                       "{NV}^3; rasterizer and voxelizer fwd+bwd, L1 losses and Adam per step"),
    "scale": dict(config="scale", views_per_call=10, recompute=True,
                  label="scaling: {N} Gaussians, {V} cone-beam views {D}x{D} (10 views per call, lists rebuilt "
                        "in the backward), voxelizer {NV}^3; fwd+bwd, L1 losses and Adam per step"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
# Weights of the SSIM and crop-TV terms of Eq. 5 in the one-view step (the
# paper prints none).
SSIM_WEIGHT = 0.25
TV_WEIGHT = 0.05


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest() -> str:
    """SHA-256 over the library's kernel sources: HBM traffic measured on an
    older build of the kernels is not reported."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2604_01844_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = source_digest()
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if line.startswith("#") or len(f) != 5:
                continue
            if f[0] == workload and f[1] == kernel and f[2] == digest:
                return dict(fetch_bytes=float(f[3]), write_bytes=float(f[4]))
    return None


def cpu_baseline(gs, gd, ang, grid_d, budget_s=12.0):
    """Time the FP64 oracle on a bounded sample of one step and scale it to the
    whole step: whole views of the rasterizer forward+backward over all
    Gaussians (about half the budget), 8-slice slabs of the voxelizer forward
    from the middle of the grid outwards, and the voxelizer backward of
    chunks of 1000 Gaussians (a quarter each)."""
    import oracle
    oracle.build(force=False)
    n_views = len(ang)
    nx, ny, nz = grid_d["dims"]
    n = gs["density"].shape[0]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c1 = np.ones((1, gd["det_h"], gd["det_w"])) / (gd["det_h"] * gd["det_w"])
    t_proj, nv = 0.0, 0
    while nv < n_views and (nv == 0 or t_proj < 0.5 * budget_s):
        t0 = time.perf_counter()
        oracle.project(gs, gd, ang[nv:nv + 1])
        oracle.project_bwd(gs, gd, ang[nv:nv + 1], c1)
        t_proj += time.perf_counter() - t0
        nv += 1
    h = grid_d["spacing"][2]
    t_vox, slabs = 0.0, 0
    order = [nz // 2 - 8 * (k // 2 + 1) if k % 2 == 0 else nz // 2 + 8 * (k // 2) for k in range(nz // 8)]
    while slabs < len(order) and (slabs == 0 or t_vox < 0.25 * budget_s):
        z0 = order[slabs]
        slab = dict(origin=(grid_d["origin"][0], grid_d["origin"][1], grid_d["origin"][2] + z0 * h),
                    spacing=grid_d["spacing"], dims=(nx, ny, 8))
        t0 = time.perf_counter()
        oracle.voxelize(gs, slab)
        t_vox += time.perf_counter() - t0
        slabs += 1
    gv = np.ones((nz, ny, nx)) / (nx * ny * nz)
    perm = np.random.default_rng(0).permutation(n)
    t_vb, done = 0.0, 0
    while done < n and (done == 0 or t_vb < 0.25 * budget_s):
        t0 = time.perf_counter()
        oracle.voxelize_bwd(gs, grid_d, gv, sel=perm[done:done + 1000])
        t_vb += time.perf_counter() - t0
        done += min(1000, n - done)
    step_s = t_proj * n_views / nv + t_vox * nz / (8 * slabs) + t_vb * n / done
    sampled = t_proj + t_vox + t_vb
    return dict(value=n_views * gd["det_w"] * gd["det_h"] / step_s, unit="view-pixels/s", cores=cores,
                kind="oracle",
                sample=(f"FP64 oracle with {cores} OpenMP threads: {nv} of {n_views} views rasterized "
                        f"forward+backward over all {n} Gaussians, {8 * slabs} of {nz} z-slices voxelized, "
                        f"voxelizer backward of {done} of {n} Gaussians; {sampled:.1f} s measured, scaled "
                        f"linearly to one step ({step_s:.1f} s)"),
                seconds_per_step=step_s)


ABLATIONS = (("design", 0, "splat"), ("square boxes", 1, "splat"), ("no quadrant culling", 2, "splat"),
             ("per-pixel atomic backward", 4, "splat"), ("all three", 7, "splat"),
             ("ray-exact model (E of Eq. 3 instead of M)", 0, "exact"))


def ablation(fgs, params, geom, i_gt, V, D, steps, log):
    """An MI355X analogue of the paper's Table 3 for the rasterizer: the
    standard scan's batched forward, L1 and backward (lists reused), with one
    part of the design switched off at a time. Prints one JSON line."""
    import torch
    dev = params[0].device
    img = torch.empty((V, D, D), device=dev)
    gp = [torch.empty_like(p) for p in params]
    ws_p, ws_l = fgs.Workspace(dev), fgs.Workspace(dev, 1 << 16)
    rows = {}
    for name, flag, model in ABLATIONS:
        def step(ev=None):
            e = ev or {}
            fgs.project_views(*params, geom, ws=ws_p, out=img, ablate=flag, model=model, events=e.get("fwd"))
            _, g = fgs.l1_loss_grad(img, i_gt, ws=ws_l)
            fgs.project_views_backward(*params, geom, g, recompute=False, ws=ws_p, out=gp, ablate=flag,
                                       model=model, events=e.get("bwd"))
        step()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            step()
        b.record()
        torch.cuda.synchronize()
        ev = {k: fgs.timing_events() for k in ("fwd", "bwd")}
        step(ev)
        torch.cuda.synchronize()
        pairs = fgs.project_views_support(*params, geom, model=model)
        rows[name] = dict(ms=a.elapsed_time(b) / steps, keys=ws_p.n_pairs, support_pairs=pairs,
                          pixel_kernel_ms={k: v[0].elapsed_time(v[1]) for k, v in ev.items()})
        log(f"ablation {name}: {rows[name]['ms']:.3f} ms per fwd+bwd over {V} views, {ws_p.n_pairs} keys, "
            f"pixel kernels {rows[name]['pixel_kernel_ms']}, {pairs} support pairs")
    print(json.dumps(dict(ablation="rasterizer fwd+L1+bwd, standard scan", steps=steps, rows=rows)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="scan")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-view-steps", action="store_true", help="skip the one-view step timing")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the benchmark, time the rasterizer with parts of its design switched off")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run the library's plain copy kernel 3 times on a MIB-MiB buffer "
                         "(known read and write bytes, to scale HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_01844_amd as fgs
    import synth_inputs as si

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = si.CONFIGS[wl["config"]]
    N, V, D, NV = cfg["n_gauss"], cfg["n_views"], cfg["det"], cfg["vol"]
    gs = si.gaussians(N, cfg["seed"])
    gd = si.geometry(D)
    ang = si.angles(V)
    grid_d = si.grid(NV)
    geom = fgs.Geometry.from_dict(gd, ang, dev)
    grid = fgs.Grid.from_dict(grid_d)
    ph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in si.phantom(cfg["n_ell"],
                                                                                       cfg["phantom_seed"]).items()}
    log(f"workload {args.workload}: {N} Gaussians, {V} views {D}x{D}, {NV}^3 voxels")
    i_gt = fgs.phantom_project(ph, geom)
    v_gt = fgs.phantom_voxelize(ph, grid)

    params = [torch.from_numpy(gs[k]).to(dev) for k in ("mean", "log_scale", "quat", "density")]
    if args.ablation:
        ablation(fgs, params, geom, i_gt, V, D, max(1, min(args.steps, 5)), log)
        return
    lrs = [2e-4, 5e-3, 1e-3, 1e-2]
    moms = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    gp = [torch.empty_like(p) for p in params]
    gv = [torch.empty_like(p) for p in params]
    img = torch.empty((V, D, D), device=dev)
    vol = torch.empty(grid.shape, device=dev)
    ws_p, ws_v, ws_l = fgs.Workspace(dev), fgs.Workspace(dev), fgs.Workspace(dev, 1 << 16)
    vpc = wl["views_per_call"]
    chunks = 1 if vpc is None else (V + vpc - 1) // vpc
    state = {"step": 0}

    def step(ev=None):
        e = ev or {}
        fgs.project_views(*params, geom, ws=ws_p, out=img, events=e.get("splat_fwd"), views_per_call=vpc)
        _, g_img = fgs.l1_loss_grad(img, i_gt, ws=ws_l)
        fgs.project_views_backward(*params, geom, g_img, recompute=wl["recompute"], ws=ws_p, out=gp,
                                   events=e.get("splat_bwd"), views_per_call=vpc)
        fgs.voxelize(*params, grid, ws=ws_v, out=vol, events=e.get("vox_fwd"))
        _, g_vol = fgs.l1_loss_grad(vol, v_gt, n_views=1, ws=ws_l)
        fgs.voxelize_backward(*params, grid, g_vol, recompute=False, ws=ws_v, out=gv, events=e.get("vox_bwd"))
        state["step"] += 1
        for k, p in enumerate(params):
            fgs.adam_step(p, gp[k], moms[k][0], moms[k][1], state["step"], lrs[k], grad2=gv[k],
                          clamp_min_zero=(k == 3))

    def events():
        e = {n: fgs.timing_events() for n in ("vox_fwd", "vox_bwd")}
        for n in ("splat_fwd", "splat_bwd"):
            e[n] = fgs.timing_events() if chunks == 1 else [fgs.timing_events() for _ in range(chunks)]
        return e

    def elapsed(pair_or_list):
        pl = [pair_or_list] if isinstance(pair_or_list, tuple) else pair_or_list
        return sum(a.elapsed_time(b) for a, b in pl)

    pairs0 = {"splat": fgs.project_views_support(*params, geom, ws=ws_p),
              "vox": fgs.voxelize_support(*params, grid, ws=ws_v)}
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")
    evs = [events() for _ in range(args.steps)]
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
    kern_ms = {n: float(np.mean([elapsed(e[n]) for e in evs])) for n in NAMES}
    # (tile, Gaussian) keys of the last binning of each workspace (for a
    # view-chunked workload: of the last chunk)
    keys = {"splat": ws_p.n_pairs, "vox": ws_v.n_pairs}
    pairs1 = {"splat": fgs.project_views_support(*params, geom, ws=ws_p),
              "vox": fgs.voxelize_support(*params, grid, ws=ws_v)}
    pairs = {k: 0.5 * (pairs0[k] + pairs1[k]) for k in pairs0}
    log(f"timed: {ms_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}); kernels {kern_ms}")

    kernels = {}
    for n in NAMES:
        pr = pairs["splat" if n.startswith("splat") else "vox"]
        tf = pr * FLOPS_PER_PAIR[n] / (kern_ms[n] * 1e-3) / 1e12
        kernels[n] = dict(ms=round(kern_ms[n], 4), launches=chunks if n.startswith("splat") else 1,
                          support_pairs=int(pr), keys_per_launch=int(keys["splat" if n.startswith("splat") else "vox"]),
                          pairs_per_s=pr / (kern_ms[n] * 1e-3), tflops=round(tf, 3))
    dom = max(NAMES, key=lambda n: kern_ms[n])
    launches = kernels[dom]["launches"]
    tr = measured_traffic(args.workload, dom)
    roof = dict(bound="alu", achieved=round(kernels[dom]["tflops"], 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(kernels[dom]["tflops"] / PEAK_FP32_TFLOPS, 4),
                traffic=None if tr is None else round(tr["fetch_bytes"] + tr["write_bytes"]),
                peak_basis="256 CUs x 64 FP32 FMA lanes/clock x 2 flops x 2.4 GHz (no packed FP32)",
                peak_published=PEAK_FP32_PUBLISHED_TFLOPS,
                frac_of_published=round(kernels[dom]["tflops"] / PEAK_FP32_PUBLISHED_TFLOPS, 4),
                kernel=dom, flops_per_pair=FLOPS_PER_PAIR[dom], support_pairs=kernels[dom]["support_pairs"],
                launches_per_step=launches, avg_launch_ms=round(kern_ms[dom] / launches, 4))
    out = dict(metric=METRIC, value=V * D * D / (ms_step * 1e-3), unit="view-pixels/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=wl["label"].format(N=N, V=V, D=D, NV=NV), n_gauss=N, views=V, det=D, vol=NV),
               voxels_per_s=NV ** 3 / (ms_step * 1e-3), s_per_step=ms_step * 1e-3,
               kernels=kernels, roofline=roof)

    if args.workload == "scan" and not args.no_view_steps:
        # the reconstruction loop's optimizer step: one view fwd, L1, bwd (lists reused), Adam
        from paper_2604_01844_amd.recon import CropTV
        img1 = torch.empty((1, D, D), device=dev)
        rng = np.random.Generator(np.random.PCG64(0))
        order = rng.permutation(V)
        tv = CropTV(grid, TV_WEIGHT, 32, dev)
        ws_s = fgs.Workspace(dev)

        def view_step(v):
            fgs.project_views(*params, geom, int(v), 1, ws=ws_p, out=img1)
            _, g1 = fgs.l1_loss_grad(img1, i_gt[v:v + 1], ws=ws_l)
            fgs.ssim_loss_grad(img1, i_gt[v:v + 1], scale=SSIM_WEIGHT, ws=ws_s, grad=g1, accumulate=True)
            fgs.project_views_backward(*params, geom, g1, int(v), 1, recompute=False, ws=ws_p, out=gp)
            tv.add_grad(params, gp, rng)
            state["step"] += 1
            for k, p in enumerate(params):
                fgs.adam_step(p, gp[k], moms[k][0], moms[k][1], state["step"], lrs[k], clamp_min_zero=(k == 3))
        for v in order[:5]:
            view_step(v)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for v in order:
            view_step(v)
        torch.cuda.synchronize()
        epoch_s = time.perf_counter() - w0
        out["s_per_view_step"] = epoch_s / V
        out["s_per_epoch"] = epoch_s
        log(f"one-view steps: {1e3 * epoch_s / V:.3f} ms/step, {epoch_s:.3f} s/epoch")
    if args.calibrate_copy:
        from paper_2604_01844_amd import _abi
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            _abi.check(_abi.lib().fgs_copy(_abi.ptr(src), _abi.ptr(dst), src.numel(), _abi.stream_ptr(dev)))
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(gs, gd, ang, grid_d)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
