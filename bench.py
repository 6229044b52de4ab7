"""Benchmark of the FaCT-GS hot path on one MI355X.

One step = one pass of the whole hot path over one workload:
  rasterizer forward over all views -> L1 loss and gradient against the
  phantom's exact projections -> rasterizer backward -> voxelizer forward
  over the whole grid -> L1 against the phantom volume -> voxelizer backward
  -> one Adam step on all 11 N parameters (both gradients fused). Each step
  starts from the same parameters (restored by a device copy at its start),
  so every timed step does the same work.

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

# FP32 flops per support pair (an exponential counts as one) in the
# evaluation scheme the kernels use, where the quadratic form is expanded
# incrementally down a pixel column (voxel row) and the moments are
# accumulated as column and row sums:
#   forward  (splat and voxel): exponent 2 FMAs (4), exp 1, weighted sum 1 FMA (2) = 7
#   backward (splat and voxel): exponent 2 FMAs (4), exp 1, three sums 3 FMAs (6)  = 11
# The plain per-pair formula costs more (splat 12 / 22, voxel 20 / 38: the
# full quadratic form and every moment product per pair); it is reported as
# flops_per_pair_formula. Counting the scheme's own flops keeps every
# kernel's rate below the chip's peak.
FLOPS_PER_PAIR = {"splat_fwd": 7, "splat_bwd": 11, "vox_fwd": 7, "vox_bwd": 11}
FLOPS_PER_PAIR_FORMULA = {"splat_fwd": 12, "splat_bwd": 22, "vox_fwd": 20, "vox_bwd": 38}
# MI355X's published FP32 vector peak (it counts two-wide packed FP32
# instructions), and the non-packed peak this build can reach: 256 CUs x 64
# FMA lanes per clock x 2 flops x 2.4 GHz. The library is compiled without
# packed FP32.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6
# The per-pixel bodies the probes measure, per kernel (the voxel kernels run
# the same bodies per voxel).
PROBE_OF = {"splat_fwd": "fwd_body", "splat_bwd": "bwd_body", "vox_fwd": "fwd_body", "vox_bwd": "bwd_body"}
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


# (name, fgs_probe kind, unit of the rate, iterations per thread): each
# launch takes a few milliseconds on MI355X.
PROBES = (("fma", 0, "flop/s", 6000), ("exp", 1, "op/s", 1800), ("fwd_body", 2, "pairs/s", 900),
          ("bwd_body", 3, "pairs/s", 300), ("lds_b128", 4, "B/s", 3500), ("mfma_bf16", 5, "flop/s", 7000))


def ceilings(dev, blocks=2048, reps=3, copy_mib=1024):
    """Measured ceilings of this GPU (include/factgs.h fgs_probe): FP32 FMA
    and v_exp_f32 rates, the splat kernels' per-pixel bodies in pairs/s (the
    voxel kernels run the same bodies per voxel), conflict-free LDS
    ds_read_b128 bandwidth, v_mfma_f32_32x32x16_bf16 flops, and the
    library's plain copy kernel in HBM bytes/s (read + write). Each is the
    median rate of `reps` timed launches after one untimed one."""
    import ctypes
    import torch
    from paper_2604_01844_amd import _abi
    L = _abi.lib()
    sink = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    out = {}
    for name, kind, unit, iters in PROBES:
        work = ctypes.c_double()
        rates = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            _abi.check(L.fgs_probe(kind, blocks, iters, _abi.ptr(sink), ctypes.byref(work), _abi.stream_ptr(dev)))
            b.record()
            torch.cuda.synchronize()
            if r:
                rates.append(work.value / (a.elapsed_time(b) * 1e-3))
        out[name] = dict(rate=float(np.median(rates)), unit=unit)
    src = torch.ones(copy_mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    rates = []
    for r in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        _abi.check(L.fgs_copy(_abi.ptr(src), _abi.ptr(dst), src.numel(), _abi.stream_ptr(dev)))
        b.record()
        torch.cuda.synchronize()
        if r:
            rates.append(2.0 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3))
    out["copy"] = dict(rate=float(np.median(rates)), unit="B/s")
    del src, dst
    return out


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(gs, gd, ang, grid_d, budget_s=12.0):
    """Time the FP64 oracle on a bounded sample of one step and scale it to the
    whole step: whole views of the rasterizer forward+backward over all
    Gaussians (about half the budget), 8-slice slabs of the voxelizer forward
    from the middle of the grid outwards, and the voxelizer backward of
    chunks of 1000 Gaussians (a quarter each), on all the host's threads;
    then a smaller sample of the same parts on one thread."""
    import oracle
    oracle.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(cores)
    out = _oracle_sample(gs, gd, ang, grid_d, budget_s, cores)
    oracle.set_threads(1)
    try:
        one = _oracle_sample(gs, gd, ang, grid_d, budget_s / 3, 1)
    finally:
        oracle.set_threads(cores)
    out["one_thread"] = dict(value=one["value"], seconds_per_step=one["seconds_per_step"], sample=one["sample"])
    out["cpu_model"] = cpu_model()
    return out


def _oracle_sample(gs, gd, ang, grid_d, budget_s, cores):
    import oracle
    n_views = len(ang)
    nx, ny, nz = grid_d["dims"]
    n = gs["density"].shape[0]
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


def view_steps(fgs, params, moms, lrs, state, geom, grid, i_gt, dev, epochs=1, graphs=True):
    """The reconstruction loop's optimizer step (Sec. 3.4, the loss of Eq. 5):
    one view forward, L1 and SSIM with their gradients, backward (lists
    reused), a randomly placed 32^3 crop voxelized with the gradient of its
    TV, Adam, with lists at a fixed capacity so no step waits for the GPU.
    graphs=True: each view's step is captured once in a HIP graph during an
    untimed epoch and replayed (one small kernel and one graph launch per
    step); graphs=False: one fgs_recon_step call per step. Then `epochs`
    timed epochs over all views in a random order; returns seconds per epoch
    and the number of capacity overflows seen (steps that binned nothing)."""
    import torch
    from paper_2604_01844_amd import recon
    V = geom.n_views
    model = recon.GaussianModel(*params)
    model.m = [mv[0] for mv in moms]
    model.v = [mv[1] for mv in moms]
    model.step = state["step"]
    adam = recon.AdamConfig(lr_mean=lrs[0], lr_log_scale=lrs[1], lr_quat=lrs[2], lr_density=lrs[3])
    rng = np.random.Generator(np.random.PCG64(0))
    order = rng.permutation(V)
    tv = recon.CropTV(grid, TV_WEIGHT, 32, dev)
    stepper = recon.ViewStep(model, geom, adam, ssim_weight=SSIM_WEIGHT, tv=tv, graphs=graphs)
    # one untimed epoch (with graphs: each view's step captured once)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for v in order:
        stepper(int(v), i_gt[v], rng)
    torch.cuda.synchronize()
    log(f"first epoch{' (with the graph captures)' if graphs else ''}: {time.perf_counter() - c0:.3f} s")
    w0 = time.perf_counter()
    for _ in range(epochs):
        for v in order:
            stepper(int(v), i_gt[v], rng)
    torch.cuda.synchronize()
    epoch_s = (time.perf_counter() - w0) / epochs
    state["step"] = model.step
    overflows = stepper.check_overflow()
    log(f"one-view steps: {1e3 * epoch_s / V:.3f} ms/step, {epoch_s:.3f} s/epoch, {overflows} capacity overflows")
    return epoch_s, overflows


def fit_steps(fgs, si, dev, steps=30, ssim_weight=0.2):
    """The volume-fitting step (Sec. 3.6): 200,000 Gaussians placed by
    gradient sampling on a seeded 256^3 phantom, then per step the whole grid
    voxelized, the loss, the voxelizer backward and Adam. Timed with the L1
    term alone and with the full loss of Eq. 6 (L1 + ssim_weight (1 - 3D
    SSIM)); milliseconds per step, medians of three runs of `steps` steps."""
    import torch
    from paper_2604_01844_amd import recon
    cfg = si.CONFIGS["fit"]
    grid = fgs.Grid.from_dict(si.grid(cfg["vol"]))
    ph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in si.phantom(cfg["n_ell"],
                                                                                       cfg["phantom_seed"]).items()}
    v_gt = fgs.phantom_voxelize(ph, grid)
    out = dict(n_gauss=cfg["n_gauss"], vol=cfg["vol"], steps=steps, ssim_weight=ssim_weight)
    for name, w in (("ms_per_step_l1", 0.0), ("ms_per_step_eq6", ssim_weight)):
        runs = []
        for _ in range(3):
            n = cfg["n_gauss"]
            model = recon.init_from_volume(v_gt, grid, n, si.uniforms(4 * n, cfg["seed"]).reshape(4, n))
            recon.fit_volume(model, v_gt, grid, iters=3, adam=recon.FIT_ADAM, eval_every=3, ssim_weight=w)
            # the loop's own clock (synchronised, evaluation excluded)
            h = recon.fit_volume(model, v_gt, grid, iters=steps, adam=recon.FIT_ADAM, eval_every=10 ** 9,
                                 ssim_weight=w)
            runs.append(h.seconds[-1] * 1e3 / steps)
        out[name] = float(np.median(runs))
    log(f"fitting step (200k Gaussians, 256^3): {out['ms_per_step_l1']:.3f} ms with L1, "
        f"{out['ms_per_step_eq6']:.3f} ms with Eq. 6")
    return out


def _timed(fn, reps=7):
    """Median milliseconds of `reps` runs of fn() after one untimed run,
    each bracketed by events on the current stream."""
    import torch
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def fig3_sweep(fgs, si, dev):
    """Kernel scaling in the manner of the paper's Fig. 3 (Sec. 3.5, kernel
    evaluation): isotropic Gaussians (sigma 0.02, no rotation, centres uniform
    in the unit cube, densities U(0.1, 1)), one view per rasterizer call.
    (a) 20,000 Gaussians on detectors of 256^2 ... 2048^2 and grids of
    64^3 ... 512^3; (b) about 10^6 pixels (1024^2) or voxels (100^3) with
    10^3 ... 10^6 Gaussians. Milliseconds per image (volume) for the forward
    and the backward, and power-law fits t = a x^b over each series."""
    import torch
    rng = np.random.Generator(np.random.PCG64(31))

    def scene(n):
        g = dict(mean=rng.uniform(-0.5, 0.5, (3, n)).astype(np.float32),
                 log_scale=np.full((3, n), np.log(0.02), np.float32),
                 quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
                 density=rng.uniform(0.1, 1.0, n).astype(np.float32))
        return [torch.from_numpy(np.ascontiguousarray(g[k])).to(dev) for k in ("mean", "log_scale", "quat", "density")]

    def raster(params, det):
        geom = fgs.Geometry.from_dict(si.geometry(det), np.zeros(1, np.float32), dev)
        ws = fgs.Workspace(dev)
        img = torch.empty((1, det, det), device=dev)
        c = torch.from_numpy(si.normals((1, det, det), 5)).to(dev)
        grads = [torch.empty_like(p) for p in params]
        fwd = _timed(lambda: fgs.project_views(*params, geom, ws=ws, out=img))
        bwd = _timed(lambda: fgs.project_views_backward(*params, geom, c, recompute=False, ws=ws, out=grads))
        return fwd, bwd

    def voxel(params, nv):
        grid = fgs.Grid.from_dict(si.grid(nv))
        ws = fgs.Workspace(dev)
        vol = torch.empty(grid.shape, device=dev)
        c = torch.from_numpy(si.normals(grid.shape, 6)).to(dev)
        grads = [torch.empty_like(p) for p in params]
        fwd = _timed(lambda: fgs.voxelize(*params, grid, ws=ws, out=vol))
        bwd = _timed(lambda: fgs.voxelize_backward(*params, grid, c, recompute=False, ws=ws, out=grads))
        return fwd, bwd

    def fit(xs, ts):
        b, la = np.polyfit(np.log(xs), np.log(ts), 1)
        return dict(a=float(np.exp(la)), b=float(b))

    rows = []
    p20 = scene(20000)
    for det in (256, 512, 1024, 2048):
        f, b = raster(p20, det)
        rows.append(dict(series="a_raster", n_gauss=20000, pixels=det * det, fwd_ms=f, bwd_ms=b))
    for nv in (64, 128, 256, 512):
        f, b = voxel(p20, nv)
        rows.append(dict(series="a_voxel", n_gauss=20000, voxels=nv ** 3, fwd_ms=f, bwd_ms=b))
    for n in (1000, 10000, 100000, 1000000):
        p = scene(n)
        f, b = raster(p, 1024)
        rows.append(dict(series="b_raster", n_gauss=n, pixels=1024 * 1024, fwd_ms=f, bwd_ms=b))
        f, b = voxel(p, 100)
        rows.append(dict(series="b_voxel", n_gauss=n, voxels=100 ** 3, fwd_ms=f, bwd_ms=b))
    fits = {}
    for series, xkey in (("a_raster", "pixels"), ("a_voxel", "voxels"), ("b_raster", "n_gauss"),
                         ("b_voxel", "n_gauss")):
        r = [x for x in rows if x["series"] == series]
        for ph in ("fwd_ms", "bwd_ms"):
            fits[f"{series}_{ph}"] = fit([x[xkey] for x in r], [x[ph] for x in r])
        log(f"fig3 {series}: " + ", ".join(f"{x[xkey]}: {x['fwd_ms']:.3f}/{x['bwd_ms']:.3f} ms" for x in r))
    return dict(rows=rows, fits=fits)


def s_to_psnr(si, dev, epochs=40, levels=(30.0, 35.0, 38.0)):
    """Seconds-to-PSNR of the reconstruction loop on the standard scan's
    phantom (40 ellipsoids, seed 101; 75 views of 512^2): FDK at 128^3,
    50,000 Gaussians by FDK-gradient sampling (Sec. 3.1), then one view per
    optimiser step with the loss of Eq. 5 (L1, SSIM and the crop's TV). The
    clock covers FDK, the initialisation and the steps; the PSNR (256^3,
    peak = max of the phantom) is evaluated after every epoch outside it."""
    import torch
    from paper_2604_01844_amd import learned_init as li, ops, recon
    sc = li.Scanner(li.ScanConfig(), dev)
    cfg = si.CONFIGS["scan"]
    ph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in si.phantom(cfg["n_ell"],
                                                                                       cfg["phantom_seed"]).items()}
    proj = ops.phantom_project(ph, sc.geom)
    vol_gt = ops.phantom_voxelize(ph, sc.eval_grid)
    r = li.run_arm(sc, "fdk_gradient", cfg["phantom_seed"], epochs=epochs, adam=recon.AdamConfig(lr_density=2e-3),
                   proj=proj, vol_gt=vol_gt)
    h = r.history
    out = dict(init="FDK-gradient sampling", loss="Eq. 5: L1 + 0.25 SSIM + 0.05 crop TV", epochs=epochs,
               init_s=r.init_s, psnr_initial=h.psnr[0], psnr_final=h.psnr[-1], seconds_total=h.seconds[-1],
               capacity_overflows=h.overflows,
               to_psnr={f"{lv:g}": dict(s=r.seconds_to(lv), epochs=r.epochs_to(lv)) for lv in levels})
    log(f"s-to-PSNR: {h.psnr[0]:.2f} dB at start, {h.psnr[-1]:.2f} dB after {epochs} epochs "
        f"({h.seconds[-1]:.2f} s); " + ", ".join(f"{k} dB at {v['s']} s" for k, v in out["to_psnr"].items()))
    return out


def scaling_subrun(steps=3, warmup=1):
    """The scaling workload (500,000 Gaussians, 50 views of 2048^2, 512^3) in
    a child process of this script, so its 40 GB of workspace is freed
    before and after; returns its JSON line."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "scale", "--steps", str(steps), "--warmup",
           str(warmup), "--no-cpu-baseline", "--no-fit", "--no-scale", "--no-psnr"]
    log("scaling workload: " + " ".join(cmd[1:]))
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    sys.stderr.write(r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"scaling workload run failed ({r.returncode})")
    line = [l for l in r.stdout.splitlines() if l.startswith("{")][-1]
    d = json.loads(line)
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "voxels_per_s", "config", "kernels", "roofline")
    return {k: d[k] for k in keep if k in d}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="scan")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-view-steps", action="store_true", help="skip the one-view step timing")
    ap.add_argument("--no-fit", action="store_true", help="skip the volume-fitting step timing")
    ap.add_argument("--no-scale", action="store_true", help="skip the scaling-workload run")
    ap.add_argument("--no-psnr", action="store_true", help="skip the seconds-to-PSNR run")
    ap.add_argument("--fig3", action="store_true",
                    help="instead of the benchmark, run the kernel scaling sweep of the paper's Fig. 3 and print "
                         "one JSON line with power-law fits")
    ap.add_argument("--view-steps-only", type=int, default=0, metavar="EPOCHS",
                    help="instead of the benchmark, time EPOCHS epochs of the one-view optimizer step (standard "
                         "scan) and print one JSON line")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the benchmark, time the rasterizer with parts of its design switched off")
    ap.add_argument("--probes", action="store_true",
                    help="instead of the benchmark, measure the ceilings (FMA, exp, the splat bodies, LDS, MFMA, "
                         "copy) and print them as one JSON line")
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
    if args.probes:
        print(json.dumps(dict(ceilings=ceilings(dev), device=torch.cuda.get_device_name(dev))), flush=True)
        return
    if args.fig3:
        print(json.dumps(dict(fig3=fig3_sweep(fgs, si, dev))), flush=True)
        return
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
    if args.view_steps_only:
        st = {"step": 0}
        epoch_s, ovf = view_steps(fgs, params, moms, lrs, st, geom, grid, i_gt, dev, epochs=args.view_steps_only)
        epoch_d, ovf_d = view_steps(fgs, params, moms, lrs, st, geom, grid, i_gt, dev, epochs=args.view_steps_only,
                                    graphs=False)
        print(json.dumps(dict(s_per_view_step=epoch_s / V, s_per_epoch=epoch_s,
                              s_per_view_step_direct=epoch_d / V, epochs=args.view_steps_only,
                              capacity_overflows=ovf + ovf_d,
                              workload=wl["label"].format(N=N, V=V, D=D, NV=NV))), flush=True)
        return
    gp = [torch.empty_like(p) for p in params]
    gv = [torch.empty_like(p) for p in params]
    img = torch.empty((V, D, D), device=dev)
    vol = torch.empty(grid.shape, device=dev)
    ws_p, ws_v, ws_l = fgs.Workspace(dev), fgs.Workspace(dev), fgs.Workspace(dev, 1 << 16)
    vpc = wl["views_per_call"]
    chunks = 1 if vpc is None else (V + vpc - 1) // vpc
    state = {"step": 0}
    # every timed step starts from the same parameters (a 2.2 MB device copy
    # inside the step), so each does the same work and the support-pair
    # count below is that of every step; Adam still updates them each step
    params0 = [p.clone() for p in params]

    def step(ev=None):
        e = ev or {}
        for p, p0 in zip(params, params0):
            p.copy_(p0)
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

    pairs = {"splat": fgs.project_views_support(*params, geom, ws=ws_p),
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
    log(f"timed: {ms_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}); kernels {kern_ms}")

    log("measuring the ceilings (probes)")
    ceil = ceilings(dev)
    kernels = {}
    for n in NAMES:
        pr = pairs["splat" if n.startswith("splat") else "vox"]
        pps = pr / (kern_ms[n] * 1e-3)
        body = ceil[PROBE_OF[n]]["rate"]
        kernels[n] = dict(ms=round(kern_ms[n], 4), launches=chunks if n.startswith("splat") else 1,
                          support_pairs=int(pr), keys_per_launch=int(keys["splat" if n.startswith("splat") else "vox"]),
                          pairs_per_s=pps, tflops=round(pps * FLOPS_PER_PAIR[n] / 1e12, 3),
                          tflops_formula=round(pps * FLOPS_PER_PAIR_FORMULA[n] / 1e12, 3),
                          frac_of_body_ceiling=round(pps / body, 4))
    dom = max(NAMES, key=lambda n: kern_ms[n])
    launches = kernels[dom]["launches"]
    tr = measured_traffic(args.workload, dom)
    tf = kernels[dom]["tflops"]
    roof = dict(bound="alu", achieved=tf, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s", frac=round(tf / PEAK_FP32_TFLOPS, 4),
                traffic=None if tr is None else round(tr["fetch_bytes"] + tr["write_bytes"]),
                peak_basis="MI355X published FP32 vector peak (counts two-wide packed FP32)",
                kernel=dom, flops_per_pair=FLOPS_PER_PAIR[dom], support_pairs=kernels[dom]["support_pairs"],
                launches_per_step=launches, avg_launch_ms=round(kern_ms[dom] / launches, 4),
                peak_nonpacked=PEAK_FP32_NONPACKED_TFLOPS, frac_nonpacked=round(tf / PEAK_FP32_NONPACKED_TFLOPS, 4),
                flops_per_pair_formula=FLOPS_PER_PAIR_FORMULA[dom],
                frac_formula=round(kernels[dom]["tflops_formula"] / PEAK_FP32_TFLOPS, 4),
                body_ceiling_pairs_per_s=ceil[PROBE_OF[dom]]["rate"],
                frac_of_body_ceiling=kernels[dom]["frac_of_body_ceiling"])
    out = dict(metric=METRIC, value=V * D * D / (ms_step * 1e-3), unit="view-pixels/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_step, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=wl["label"].format(N=N, V=V, D=D, NV=NV), n_gauss=N, views=V, det=D, vol=NV),
               voxels_per_s=NV ** 3 / (ms_step * 1e-3), s_per_step=ms_step * 1e-3,
               kernels=kernels, roofline=roof, ceilings=ceil)

    if args.workload == "scan" and not args.no_view_steps:
        epoch_s, ovf = view_steps(fgs, params, moms, lrs, state, geom, grid, i_gt, dev)
        epoch_d, ovf_d = view_steps(fgs, params, moms, lrs, state, geom, grid, i_gt, dev, graphs=False)
        out["s_per_view_step"] = epoch_s / V
        out["s_per_epoch"] = epoch_s
        out["s_per_view_step_direct"] = epoch_d / V
        out["view_step_capacity_overflows"] = ovf + ovf_d
    if args.workload == "scan" and not args.no_fit:
        out["fit_step"] = fit_steps(fgs, si, dev)
    if args.workload == "scan" and not args.no_psnr:
        out["s_to_psnr"] = s_to_psnr(si, dev)
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
    if args.workload == "scan" and not args.no_scale:
        torch.cuda.synchronize()
        out["scaling_workload"] = scaling_subrun()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
