"""Warm start from a prior volume (Sec. 3.6, the second initialisation of
the paper's pipeline): Gaussians are fitted to a prior volume of the same
object for a few voxelizer steps, then the reconstruction of the new scan
starts from them. Eq. 7's iteration ratio measures what the prior saves.

The prior here is a synthetic earlier scan: the target phantom with its
ellipsoids slightly moved, resized and re-weighted (synth_inputs).
Every numerical step runs in libfactgs.
"""
from __future__ import annotations

import time

import numpy as np
import torch

import synth_inputs as si

from . import ops, recon
from .learned_init import LEVELS, ArmResult, Scanner, ScanConfig, eq5_loop, iteration_ratio, run_arm


def prior_phantom(sc: Scanner, seed: int) -> dict:
    ph = si.perturbed_phantom(si.random_phantom(seed), seed)
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(sc.device) for k, v in ph.items()}


def warm_model(sc: Scanner, prior_vol, uniforms, *, fit_iters: int = 50,
               adam: recon.AdamConfig = recon.FIT_ADAM) -> recon.GaussianModel:
    """Gradient-sampling init on the prior volume, then fit_iters steps of
    voxelizer fitting to it (the paper's rapid fit: 50 steps)."""
    model = recon.init_from_volume(prior_vol, sc.grid, sc.cfg.n_gauss, uniforms)
    recon.fit_volume(model, prior_vol, sc.grid, iters=fit_iters, adam=adam, eval_every=fit_iters)
    model.m = [torch.zeros_like(p) for p in model.params]   # fresh optimiser state for the reconstruction
    model.v = [torch.zeros_like(p) for p in model.params]
    model.step = 0
    return model


def run_warm(sc: Scanner, seed: int, *, epochs: int, adam: recon.AdamConfig, proj, vol_gt, fit_iters: int = 50,
             target_psnr: float | None = None, **loop) -> ArmResult:
    """Reconstruct phantom `seed` from its projections starting from the fit
    to its prior; the clock covers the prior's fit."""
    u = sc.uniforms(seed)
    prior = ops.phantom_voxelize(prior_phantom(sc, seed), sc.grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model = warm_model(sc, prior, u, fit_iters=fit_iters)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    loop = {**eq5_loop(sc), **loop}
    hist = recon.reconstruct(model, proj, sc.geom, epochs=epochs, adam=adam, vol_gt=vol_gt, eval_grid=sc.eval_grid,
                             eval_every=1, target_psnr=target_psnr, seed=seed, t_offset=t_init, eval_at_start=True,
                             **loop)
    return ArmResult(t_init, hist)


def ssim3d(vol, gt) -> float:
    """Mean 3D SSIM (Eq. 6's window and constants) of vol against gt."""
    loss, _ = ops.ssim3d_loss_grad(vol, gt, want_grad=False)
    return 1.0 - float(loss.item())


def init_quality(sc: Scanner, seed: int, *, fit_iters: int = 50) -> dict:
    """The paper's initialisation comparison (Sec. 4): 3D SSIM against the
    target volume of what each strategy starts from, on the evaluation grid:
    FDK-intensity sampling, FDK-gradient sampling (both from the FDK of the
    scan's projections), the prior volume used directly, and the rapid fit to
    the prior."""
    ph = sc.phantom(seed)
    gt = ops.phantom_voxelize(ph, sc.eval_grid)
    vfdk, _ = sc.fdk(sc.project(ph))
    u = sc.uniforms(seed)
    out = {}
    for w in ("intensity", "gradient"):
        m = recon.init_from_volume(vfdk, sc.grid, sc.cfg.n_gauss, u, weighting=w)
        out[f"fdk_{w}"] = ssim3d(ops.voxelize(*m.params, sc.eval_grid), gt)
    pph = prior_phantom(sc, seed)
    out["prior_direct"] = ssim3d(ops.phantom_voxelize(pph, sc.eval_grid), gt)
    warm = warm_model(sc, ops.phantom_voxelize(pph, sc.grid), u, fit_iters=fit_iters)
    out["rapid_fit"] = ssim3d(ops.voxelize(*warm.params, sc.eval_grid), gt)
    return out


def compare(sc: Scanner, seeds, *, epochs: int, adam: recon.AdamConfig, fit_iters: int = 50, log=None) -> list:
    """Cold starts (FDK-gradient rule, and the FDK-intensity baseline) against
    warm start from the prior, per held-out phantom: the initialisation's 3D
    SSIM, PSNR before the first step, seconds/epochs to fixed levels, and
    Eq. 7's ratio (the fraction of the gradient-rule run's epochs the warm run
    needs to reach that run's best PSNR)."""
    rows = []
    for seed in seeds:
        ph = sc.phantom(seed)
        proj = sc.project(ph)
        vol_gt = ops.phantom_voxelize(ph, sc.eval_grid)
        inten = run_arm(sc, "fdk_intensity", seed, epochs=epochs, adam=adam, proj=proj, vol_gt=vol_gt)
        cold = run_arm(sc, "fdk_gradient", seed, epochs=epochs, adam=adam, proj=proj, vol_gt=vol_gt)
        warm = run_warm(sc, seed, epochs=epochs, adam=adam, proj=proj, vol_gt=vol_gt, fit_iters=fit_iters)
        row = dict(seed=seed, tau_iter=iteration_ratio(cold, warm, epochs),
                   tau_iter_gradient_vs_intensity=iteration_ratio(inten, cold, epochs),
                   init_ssim3d=init_quality(sc, seed, fit_iters=fit_iters))
        for name, r in (("intensity", inten), ("cold", cold), ("warm", warm)):
            row[name] = dict(init_s=r.init_s, psnr0=r.psnr0, psnr_final=r.history.psnr[-1],
                             levels={f"{lv:g}": dict(s=r.seconds_to(lv), epochs=r.epochs_to(lv)) for lv in LEVELS})
        rows.append(row)
        if log:
            log(f"phantom {seed}: {row}")
    return rows


def main(argv=None):
    """Warm start vs cold starts (gradient and intensity sampling) on held-out
    phantoms; JSON summary on stdout."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--held-out", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--fit-iters", type=int, default=50)
    a = ap.parse_args(argv)
    log = lambda m: print(f"[warm-start] {m}", file=sys.stderr, flush=True)
    sc = Scanner(ScanConfig(), torch.device("cuda:0"))
    rows = compare(sc, range(2000, 2000 + a.held_out), epochs=a.epochs, adam=recon.AdamConfig(lr_density=2e-3),
                   fit_iters=a.fit_iters, log=log)
    taus = [r["tau_iter"] for r in rows if r["tau_iter"] is not None]
    taus_gi = [r["tau_iter_gradient_vs_intensity"] for r in rows if r["tau_iter_gradient_vs_intensity"] is not None]
    arms = ("intensity", "cold", "warm")
    mean = lambda key: {n: float(np.mean([r[n][key] for r in rows])) for n in arms}
    summary = dict(epochs=a.epochs, fit_iters=a.fit_iters, tau_iter_mean=float(np.mean(taus)) if taus else None,
                   tau_reached=len(taus), of=len(rows),
                   tau_iter_gradient_vs_intensity=float(np.mean(taus_gi)) if taus_gi else None,
                   init_ssim3d={k: float(np.mean([r["init_ssim3d"][k] for r in rows]))
                                for k in rows[0]["init_ssim3d"]},
                   psnr0=mean("psnr0"), psnr_final=mean("psnr_final"), init_s=mean("init_s"),
                   per_phantom=rows)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
