"""GPU parity at the scaling workload: 500,000 Gaussians, 50 cone-beam views
of 2048x2048, 512^3 voxels; rasterizer lists rebuilt in the backward.

All 50 views are rendered (in chunks of 10 views per library call, each
chunk binned on its own, gradients accumulated across chunks in the
library); the oracle checks sampled pixels and voxels one by one and the
gradients of 64 random Gaussians (each depends only on its own support).
Central differences (h = 1e-3) of the GPU's own forward pin its backward
on single-Gaussian scenes with kappa = 6, where the cutoff is invisible at
that step."""
import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

TOL = 1e-4
BAND = 1e-5
DEV = "cuda"
VIEWS_PER_CALL = 10


@pytest.fixture(scope="module")
def case():
    import paper_2604_01844_amd as fgs
    fgs.lib()
    oracle.build(force=False)
    cfg = si.CONFIGS["scale"]
    gs = si.gaussians(cfg["n_gauss"], cfg["seed"])
    gd = si.geometry(cfg["det"])
    ang = si.angles(cfg["n_views"])
    d = {k: torch.from_numpy(v).to(DEV) for k, v in gs.items()}
    params = (d["mean"], d["log_scale"], d["quat"], d["density"])
    return fgs, cfg, gs, gd, ang, params


def test_scale_projection_sampled(case):
    fgs, cfg, gs, gd, ang, params = case
    geom = fgs.Geometry.from_dict(gd, ang)
    ws = fgs.Workspace(DEV)
    img = fgs.project_views(*params, geom, ws=ws, views_per_call=VIEWS_PER_CALL)
    torch.cuda.synchronize()
    rng = np.random.default_rng(15)
    for v in (0, 9, 10, 33, 49):  # both sides of a chunk boundary
        ys = rng.integers(0, cfg["det"], 400)
        xs = rng.integers(0, cfg["det"], 400)
        got = img[v][torch.from_numpy(ys).to(DEV), torch.from_numpy(xs).to(DEV)].cpu().numpy()
        ref = oracle.project_points(gs, gd, float(ang[v]), xs + 0.5, ys + 0.5)
        assert oracle.rel_l2(got, ref) < TOL, v
    # a chunked range renders exactly what one call renders
    sub = fgs.project_views(*params, geom, 30, 4, ws=ws)
    assert torch.equal(sub, img[30:34])


def test_scale_whole_view_every_pixel(case):
    """One complete 2048x2048 view (view 9, the last of the first 10-view
    call) in the launch configuration the benchmark times, every pixel
    against the oracle: |gpu - ref| <= 1e-4 max|ref| everywhere and within
    1e-5 max|ref| of the bracket that support decisions near the cutoff
    allow (the FP64 contributions of pairs with |d^2 - 9| <= 1e-3);
    relative L2 <= 1e-4."""
    fgs, cfg, gs, gd, ang, params = case
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*params, geom, 0, VIEWS_PER_CALL)[VIEWS_PER_CALL - 1].cpu().numpy()
    ref, band = oracle.project_banded(gs, gd, ang[VIEWS_PER_CALL - 1:VIEWS_PER_CALL])
    ref, band = ref[0], band[0]
    err = np.abs(img.astype(np.float64) - ref)
    top = np.abs(ref).max()
    beyond = np.maximum(err - band, 0.0)
    print(f"2048^2 view: max |diff| {err.max() / top:.2e} of max|ref|, beyond the band {beyond.max() / top:.2e}; "
          f"rel-L2 {oracle.rel_l2(img, ref):.2e}", flush=True)
    assert err.max() <= 1e-4 * top
    assert beyond.max() <= 1e-5 * top
    assert oracle.rel_l2(img, ref) < TOL


def test_scale_projection_gradients_sampled(case):
    fgs, cfg, gs, gd, ang, params = case
    geom = fgs.Geometry.from_dict(gd, ang)
    c = si.normals((cfg["n_views"], cfg["det"], cfg["det"]), 79)
    g = fgs.project_views_backward(*params, geom, torch.from_numpy(c).to(DEV), views_per_call=VIEWS_PER_CALL)
    sel = np.random.default_rng(16).choice(cfg["n_gauss"], 64, replace=False)
    got = {k: t.cpu().numpy().astype(np.float64)[..., sel] for k, t in
           zip(("mean", "log_scale", "quat", "density"), g)}
    ref = oracle.project_bwd(gs, gd, ang, c, sel=sel, band=BAND)
    errs = oracle.banded_grad_error(got, ref)
    assert max(errs.values()) < TOL, errs


def test_scale_projection_gradients_match_gpu_finite_differences(case):
    """FP32 central differences of the GPU forward (kappa = 6) against the GPU
    backward for 16 of the workload's Gaussians, each alone, over 2 views."""
    fgs, cfg, gs, gd, ang, params = case
    ang2 = np.array([ang[0], ang[27]], dtype=np.float32)
    geom = fgs.Geometry.from_dict(gd, ang2)
    c = torch.from_numpy(si.normals((2, cfg["det"], cfg["det"]), 80)).to(DEV)
    ws = fgs.Workspace(DEV)
    h = 1e-3
    sel = np.random.default_rng(17).choice(cfg["n_gauss"], 16, replace=False)
    worst = 0.0
    for i in sel:
        one = [p[..., i:i + 1].contiguous().clone() for p in params]
        loss = lambda q: float((c.double() * fgs.project_views(*q, geom, ws=ws, kappa=6.0).double()).sum())
        ana = fgs.project_views_backward(*one, geom, c, ws=ws, kappa=6.0)
        for k in range(4):
            flat = one[k].view(-1)
            num = np.zeros(flat.numel())
            for j in range(flat.numel()):
                x0 = float(flat[j])
                flat[j] = x0 + h
                xp, lp = float(flat[j]), loss(one)
                flat[j] = x0 - h
                xm, lm = float(flat[j]), loss(one)
                flat[j] = x0
                num[j] = (lp - lm) / (xp - xm)  # the FP32-rounded step actually taken
            a = ana[k].view(-1).cpu().numpy().astype(np.float64)
            err = np.linalg.norm(a - num) / max(np.linalg.norm(num), 1e-12)
            worst = max(worst, err)
    assert worst < 1e-2, worst


def test_scale_voxelize_sampled(case):
    fgs, cfg, gs, gd, ang, params = case
    gr = si.grid(cfg["vol"])
    vol = fgs.voxelize(*params, fgs.Grid.from_dict(gr))
    torch.cuda.synchronize()
    rng = np.random.default_rng(18)
    idx = rng.integers(0, cfg["vol"], size=(3000, 3))
    pts = -0.5 + (idx + 0.5) * gr["spacing"][0]
    ref = oracle.field_points(gs, pts, kappa=3.0)
    ii = torch.from_numpy(idx).to(DEV)
    got = vol[ii[:, 2], ii[:, 1], ii[:, 0]].cpu().numpy()
    assert oracle.rel_l2(got, ref) < TOL


def test_scale_voxelize_gradients_sampled(case):
    fgs, cfg, gs, gd, ang, params = case
    gr = si.grid(cfg["vol"])
    c = si.normals((cfg["vol"],) * 3, 81)
    g = fgs.voxelize_backward(*params, fgs.Grid.from_dict(gr), torch.from_numpy(c).to(DEV))
    sel = np.random.default_rng(19).choice(cfg["n_gauss"], 64, replace=False)
    got = {k: t.cpu().numpy().astype(np.float64)[..., sel] for k, t in
           zip(("mean", "log_scale", "quat", "density"), g)}
    ref = oracle.voxelize_bwd(gs, gr, c, sel=sel, band=BAND)
    errs = oracle.banded_grad_error(got, ref)
    assert max(errs.values()) < TOL, errs
