"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: images, volumes and gradients within 1e-4 relative L2 of the oracle
(FP32 kernels vs FP64 reference); integer binning bit-exact wherever the
decision is not within FP32 rounding of a tile edge; repeat runs
bit-identical. Every input is seeded (synth_inputs); nothing the GPU
computes is fed to the oracle.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

TOL = 1e-4
# Gradients: pairs within BAND of the support boundary d^2 = 9 have no unique
# answer (the hard cutoff is discontinuous there; FP32 and FP64 may decide
# differently). The oracle leaves them out and reports their absolute
# contribution; the GPU must match the rest to TOL. 1e-5 is about ten FP32
# ulps of 9: the kernels' d^2 carries the rounding of the projection and the
# conic, a few ulps (every gradient test also passes at this band on the GPU,
# and was run with 1e-3 and 1e-4 before).
BAND = 1e-5
DEV = "cuda"


@pytest.fixture(scope="module")
def fgs():
    import paper_2604_01844_amd as m
    m.lib()
    oracle.build(force=False)
    return m


def dev(gs):
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(DEV) for k, v in gs.items()}


def args(t):
    return t["mean"], t["log_scale"], t["quat"], t["density"]


def rel(a, b):
    return oracle.rel_l2(a, b)


def grads_rel(gpu, ref, sel=None):
    got = {}
    for t, k in zip(gpu, ("mean", "log_scale", "quat", "density")):
        a = t.detach().cpu().numpy().astype(np.float64)
        got[k] = a if sel is None else a[..., sel]
    return oracle.banded_grad_error(got, ref)


# ------------------------------------------------------------------ rasterizer forward

def test_projection_tiny_config(fgs):
    """2,000 Gaussians, 24 cone-beam views of 64x64 (SOD 1.5, SDD 2.0)."""
    gs = si.gaussians(2000, 0)
    gd = si.geometry(64)
    ang = si.angles(24)
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*args(dev(gs)), geom).cpu().numpy()
    ref = oracle.project(gs, gd, ang)
    for v in range(24):
        assert rel(img[v], ref[v]) < TOL, v
    assert rel(img, ref) < TOL


@pytest.mark.parametrize("mode", ["cone", "parallel"])
def test_projection_ragged_detector(fgs, mode):
    """Detector sizes that are not tile multiples, an off-centre principal point."""
    gs = si.gaussians(333, 3)
    gd = si.geometry(72, 56, mode=mode)
    gd["off_u"], gd["off_v"] = 3.25, -2.5
    ang = si.angles(5)
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*args(dev(gs)), geom).cpu().numpy()
    ref = oracle.project(gs, gd, ang)
    assert img.shape == (5, 56, 72)
    assert rel(img, ref) < TOL


def test_projection_view_subrange_and_single_gaussian(fgs):
    gs = si.gaussians(1, 4)
    gs["mean"][:] = 0.05
    gd = si.geometry(40)
    ang = si.angles(6)
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*args(dev(gs)), geom, 2, 3).cpu().numpy()
    ref = oracle.project(gs, gd, ang[2:5])
    assert rel(img, ref) < TOL


def test_projection_all_outside_is_zero(fgs):
    """Gaussians that project outside the detector give a zero image and zero gradient."""
    gs = si.gaussians(50, 5)
    gs["mean"][2, :] = 5.0  # far above the detector's field of view
    gd = si.geometry(32)
    ang = si.angles(3)
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    img = fgs.project_views(*args(t), geom)
    assert torch.count_nonzero(img).item() == 0
    g = fgs.project_views_backward(*args(t), geom, torch.ones_like(img))
    for x in g:
        assert torch.count_nonzero(x).item() == 0


def test_projection_is_deterministic(fgs):
    gs = si.gaussians(3000, 6)
    gd = si.geometry(96)
    geom = fgs.Geometry.from_dict(gd, si.angles(4))
    t = dev(gs)
    a = fgs.project_views(*args(t), geom)
    b = fgs.project_views(*args(t), geom)
    assert torch.equal(a, b)


def test_capacity_protocol(fgs):
    from paper_2604_01844_amd import _abi as A
    gs = si.gaussians(2000, 0)
    gd = si.geometry(64)
    geom = fgs.Geometry.from_dict(gd, si.angles(8))
    t = dev(gs)
    ws = fgs.Workspace(DEV, 1 << 10)
    g = A.fgs_gaussians(2000, *(A.ptr(x) for x in args(t)))
    gm = geom.struct()
    o = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1)
    img = torch.empty((8, 64, 64), device=DEV)
    ws.s.bytes = 1 << 10
    code = A.lib().fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 0, 8, ctypes.byref(o), A.ptr(img),
                                         ctypes.byref(ws.s), A.stream_ptr())
    assert code == A.FGS_E_CAPACITY and ws.s.needed > (1 << 10)
    out = fgs.project_views(*args(t), geom, ws=ws)
    assert rel(out.cpu().numpy(), oracle.project(gs, gd, si.angles(8))) < TOL


@pytest.mark.parametrize("views, det, model", [(8, 64, "splat"), (1, 200, "splat"), (3, 96, "exact")])
def test_workspace_query_bounds_the_need(fgs, views, det, model):
    """fgs_workspace_query: fixed + pairs * per-pair bytes is at least what a
    call with that many pairs asks for (forward, backward, voxelizer), both
    for calls with many tiles and for chunked one-view calls."""
    gs = si.gaussians(3000, 4)
    geom = fgs.Geometry.from_dict(si.geometry(det), si.angles(views))
    t = dev(gs)
    ws = fgs.Workspace(DEV)
    fgs.project_views(*args(t), geom, ws=ws, model=model)
    need = int(ws.s.needed)
    assert need <= fgs.workspace_bytes("project_fwd", 3000, ws.n_pairs, geom=geom, view_count=views, model=model)
    fgs.project_views_backward(*args(t), geom, torch.zeros((views, det, det), device=DEV), ws=ws, model=model)
    assert int(ws.s.needed) <= fgs.workspace_bytes("project_bwd", 3000, ws.n_pairs, geom=geom, view_count=views,
                                                   model=model)
    for gr in (si.grid(48), dict(origin=(-0.2, -0.1, 0.0), spacing=(0.01, 0.01, 0.01), dims=(32, 32, 32))):
        grid = fgs.Grid.from_dict(gr)
        wv = fgs.Workspace(DEV)
        fgs.voxelize(*args(t), grid, ws=wv)
        assert int(wv.s.needed) <= fgs.workspace_bytes("voxelize_fwd", 3000, wv.n_pairs, grid=grid)
    # a workspace of exactly the bound takes the call without a retry
    exact = fgs.Workspace(DEV)
    exact.buf = torch.empty(fgs.workspace_bytes("project_fwd", 3000, ws.n_pairs, geom=geom, view_count=views,
                                                model=model), dtype=torch.uint8, device=DEV)
    exact.s.ptr, exact.s.bytes = exact.buf.data_ptr(), exact.buf.numel()
    from paper_2604_01844_amd import _abi as A
    g = A.fgs_gaussians(3000, *(A.ptr(x) for x in args(t)))
    gm = geom.struct()
    o = fgs.ops._opts(3.0, 1e-2, model=model)
    img = torch.empty((views, det, det), device=DEV)
    assert A.lib().fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 0, views, ctypes.byref(o), A.ptr(img),
                                         ctypes.byref(exact.s), A.stream_ptr()) == A.FGS_OK


# ------------------------------------------------------------------ binning

def _ambiguous(c64, r64, band=2e-3):
    """Edges whose FP64 position is within `band` pixels of a tile boundary:
    there the FP32 decision may go either way."""
    lo = c64 - r64 - 0.5
    hi = c64 + r64 - 0.5
    near = lambda x: np.abs(x / 16.0 - np.round(x / 16.0)) * 16.0 < band
    return near(lo) | near(hi)


def test_binning_matches_integer_reference(fgs):
    gs = si.gaussians(1500, 9)
    gd = si.geometry(80, 48)
    ang = si.angles(5)
    geom = fgs.Geometry.from_dict(gd, ang)
    ws = fgs.Workspace(DEV)
    fgs.project_views(*args(dev(gs)), geom, ws=ws)
    torch.cuda.synchronize()
    d = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in fgs.binning_dump(ws).items()}
    rec = oracle.splat_records(gs, gd, ang)
    r64 = 3.0 * np.sqrt(rec["shat"][:, [0, 2]])
    b = oracle.bin_tiles(rec["uv"].astype(np.float32), r64.astype(np.float32), 80, 48, cull=rec["culled"],
                         n_views=5)
    amb = (_ambiguous(rec["uv"][:, 0], r64[:, 0]) | _ambiguous(rec["uv"][:, 1], r64[:, 1]))
    gcount = np.diff(d["offset"].astype(np.int64))
    ok = ~amb
    np.testing.assert_array_equal(gcount[ok], b["count"][ok])
    nz = ok & (gcount > 0)
    np.testing.assert_array_equal(d["rect"][nz].astype(np.int64) & 0xffff, b["rect"][nz])
    # per-tile lists: equal once ambiguous records are set aside; ascending
    # record index. Keys are view << tile_bits | tile, sorted by (tile, view).
    rng = d["tile_ranges"].astype(np.int64)
    tpv, tb = 5 * 3, d["tile_bits"]
    assert tb == 4 and d["n_tiles"] == 5 * tpv
    skeys = d["sorted_keys"].astype(np.int64)
    order = (skeys & ((1 << tb) - 1)) * 5 + (skeys >> tb)   # (tile, view) rank of each sorted key
    assert np.all(np.diff(order) >= 0)
    amb_ids = set(np.nonzero(amb)[0].tolist())
    covered = 0
    for t in range(d["n_tiles"]):
        v, tt = divmod(t, tpv)
        lo, hi = rng[t]
        covered += hi - lo
        gl = d["sorted_vals"][lo:hi].astype(np.int64)
        assert np.all(np.diff(gl) > 0)
        assert np.all(skeys[lo:hi] == (v << tb) | tt)
        ol = b["sorted_vals"][b["tile_start"][t]:b["tile_start"][t + 1]]
        gl2 = [x for x in gl.tolist() if x not in amb_ids]
        ol2 = [x for x in ol.tolist() if x not in amb_ids]
        assert gl2 == ol2, t
        if not amb.any():
            assert gl.tolist() == ol.tolist(), t
    assert covered == d["n_pairs"]


@pytest.mark.parametrize("n, w, h, views, seed", [(1, 32, 32, 1, 21), (3, 48, 40, 2, 22), (40, 64, 64, 3, 23),
                                                   (5000, 176, 144, 4, 24)])
def test_binning_ranges_across_sizes(fgs, n, w, h, views, seed):
    """Tile ranges, sorted keys and per-tile lists at sizes from a handful of
    keys (one partial wave of the ranges and emit kernels) to many waves with
    a ragged end, against the integer reference."""
    gs = si.gaussians(n, seed)
    gd = si.geometry(w, h)
    ang = si.angles(views)
    geom = fgs.Geometry.from_dict(gd, ang)
    ws = fgs.Workspace(DEV)
    fgs.project_views(*args(dev(gs)), geom, ws=ws)
    torch.cuda.synchronize()
    d = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in fgs.binning_dump(ws).items()}
    rec = oracle.splat_records(gs, gd, ang)
    r64 = 3.0 * np.sqrt(rec["shat"][:, [0, 2]])
    b = oracle.bin_tiles(rec["uv"].astype(np.float32), r64.astype(np.float32), w, h, cull=rec["culled"],
                         n_views=views)
    amb = (_ambiguous(rec["uv"][:, 0], r64[:, 0]) | _ambiguous(rec["uv"][:, 1], r64[:, 1]))
    amb_ids = set(np.nonzero(amb)[0].tolist())
    tpv = -(-w // 16) * -(-h // 16)
    tb = d["tile_bits"]
    assert d["n_tiles"] == views * tpv
    rng = d["tile_ranges"].astype(np.int64)
    skeys = d["sorted_keys"].astype(np.int64)
    covered = 0
    for t in range(d["n_tiles"]):
        v, tt = divmod(t, tpv)
        lo, hi = rng[t]
        assert 0 <= lo <= hi <= d["n_pairs"]
        assert hi > lo or lo == 0, t      # a tile without keys holds (0, 0)
        covered += hi - lo
        assert np.all(skeys[lo:hi] == (v << tb) | tt)
        gl = d["sorted_vals"][lo:hi].astype(np.int64)
        assert np.all(np.diff(gl) > 0)
        ol = b["sorted_vals"][b["tile_start"][t]:b["tile_start"][t + 1]]
        assert [x for x in gl.tolist() if x not in amb_ids] == [x for x in ol.tolist() if x not in amb_ids], t
    assert covered == d["n_pairs"]
    if n == 5000:
        assert d["n_pairs"] > 4 * 1024   # several waves of the ranges kernel


def test_binning_covers_support(fgs):
    """Every FP64 support pair with d^2 <= 9 - 1e-3 is in a tile the GPU lists."""
    gs = si.gaussians(400, 10)
    gd = si.geometry(64)
    ang = si.angles(2)
    geom = fgs.Geometry.from_dict(gd, ang)
    ws = fgs.Workspace(DEV)
    fgs.project_views(*args(dev(gs)), geom, ws=ws)
    torch.cuda.synchronize()
    d = fgs.binning_dump(ws)
    rng = d["tile_ranges"].cpu().numpy().astype(np.int64)
    vals = d["sorted_vals"].cpu().numpy().astype(np.int64)
    lists = [set(vals[rng[t, 0]:rng[t, 1]].tolist()) for t in range(d["n_tiles"])]
    rec = oracle.splat_records(gs, gd, ang)
    ys, xs = np.mgrid[0:64, 0:64]
    for r in range(800):
        v = r // 400
        du = xs + 0.5 - rec["uv"][r, 0]
        dv = ys + 0.5 - rec["uv"][r, 1]
        c0, c1, c2 = rec["conic"][r]
        inside = c0 * du * du + 2 * c1 * du * dv + c2 * dv * dv <= 9 - 1e-3
        for t in set((v * 16 + (ys[inside] // 16) * 4 + xs[inside] // 16).tolist()):
            assert r in lists[t]


# ------------------------------------------------------------------ rasterizer backward

def _proj_grad_case(fgs, n, seed, det, views, mode="cone", recompute=True):
    gs = si.gaussians(n, seed)
    gd = si.geometry(det, mode=mode)
    ang = si.angles(views)
    geom = fgs.Geometry.from_dict(gd, ang)
    c = si.normals((views, det, det), seed + 100)
    t = dev(gs)
    ws = fgs.Workspace(DEV)
    if not recompute:
        fgs.project_views(*args(t), geom, ws=ws)
    g = fgs.project_views_backward(*args(t), geom, torch.from_numpy(c).to(DEV), recompute=recompute, ws=ws)
    ref = oracle.project_bwd(gs, gd, ang, c.astype(np.float64), band=BAND)
    return g, ref


@pytest.mark.parametrize("mode", ["cone", "parallel"])
def test_projection_backward_matches_oracle(fgs, mode):
    g, ref = _proj_grad_case(fgs, 2000, 11, 64, 8, mode)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs


@pytest.mark.parametrize("w, h", [(80, 40), (96, 72), (48, 112)])
def test_projection_backward_ragged_tile_rows(fgs, w, h):
    """Detectors whose tile-row count is not a multiple of four (3, 5 and 7
    rows): the backward takes tiles in strips of four rows, the last one
    lower. Images and gradients against the oracle."""
    gs = si.gaussians(1500, 31)
    gd = si.geometry(w, h)
    ang = si.angles(3)
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    img = fgs.project_views(*args(t), geom).cpu().numpy()
    assert rel(img, oracle.project(gs, gd, ang)) < TOL
    c = si.normals((3, h, w), 32)
    g = fgs.project_views_backward(*args(t), geom, torch.from_numpy(c).to(DEV))
    ref = oracle.project_bwd(gs, gd, ang, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs


def test_large_gaussians_take_the_interior_path(fgs):
    """Gaussians spanning many tiles (here over 48 tiles per record, where
    the pixel kernels skip the cutoff test for all-interior quadrants):
    every pixel, and the gradients, against the oracle."""
    gs = si.gaussians(300, 21, log_scale_mean=math.log(0.15))
    gd = si.geometry(256)
    ang = si.angles(3)
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    ws = fgs.Workspace(DEV)
    img = fgs.project_views(*args(t), geom, ws=ws).cpu().numpy()
    assert ws.n_pairs >= 48 * 3 * 300, ws.n_pairs
    assert rel(img, oracle.project(gs, gd, ang)) < TOL
    c = si.normals((3, 256, 256), 22)
    g = fgs.project_views_backward(*args(t), geom, torch.from_numpy(c).to(DEV))
    ref = oracle.project_bwd(gs, gd, ang, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs


def test_backward_stored_lists_equal_recomputed(fgs):
    a, _ = _proj_grad_case(fgs, 1500, 12, 64, 4, recompute=True)
    b, _ = _proj_grad_case(fgs, 1500, 12, 64, 4, recompute=False)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_autograd_function_matches_direct_backward(fgs):
    gs = si.gaussians(800, 13)
    gd = si.geometry(48)
    ang = si.angles(3)
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    leaves = [x.clone().requires_grad_(True) for x in args(t)]
    c = torch.from_numpy(si.normals((3, 48, 48), 14)).to(DEV)
    img = fgs.ProjectViews.apply(*leaves, geom, 0, 3)
    (img * c).sum().backward()
    direct = fgs.project_views_backward(*args(t), geom, c)
    for lf, d in zip(leaves, direct):
        torch.testing.assert_close(lf.grad, d, rtol=0, atol=0)


# ------------------------------------------------------------------ voxelizer

def test_voxelize_tiny_config(fgs):
    gs = si.gaussians(2000, 0)
    gr = si.grid(64)
    vol = fgs.voxelize(*args(dev(gs)), fgs.Grid.from_dict(gr)).cpu().numpy()
    ref = oracle.voxelize(gs, gr)
    assert rel(vol, ref) < TOL


def test_voxelize_ragged_crop(fgs):
    """A non-cubic, non-tile-multiple sub-grid with an offset origin (a crop)."""
    gs = si.gaussians(900, 15)
    gr = dict(origin=(-0.31, -0.2, -0.45), spacing=(0.0125, 0.015, 0.011), dims=(40, 29, 37))
    vol = fgs.voxelize(*args(dev(gs)), fgs.Grid.from_dict(gr)).cpu().numpy()
    ref = oracle.voxelize(gs, gr)
    assert vol.shape == (37, 29, 40)
    assert rel(vol, ref) < TOL


def test_voxelize_small_and_large_boxes(fgs):
    """Small Gaussians (tile boxes of a few tiles, whose hit ballots the count
    pass keeps for the emission) mixed with large ones (boxes of over 512
    tiles, whose emission repeats the exact test): volume and gradients
    against the oracle."""
    small = si.gaussians(400, 41)
    large = si.gaussians(60, 42, log_scale_mean=math.log(0.15))
    gs = {k: np.concatenate([small[k], large[k]], axis=-1) for k in small}
    gr = si.grid(96)
    t = dev(gs)
    grid = fgs.Grid.from_dict(gr)
    vol = fgs.voxelize(*args(t), grid).cpu().numpy()
    assert rel(vol, oracle.voxelize(gs, gr)) < TOL
    c = si.normals((96, 96, 96), 43)
    g = fgs.voxelize_backward(*args(t), grid, torch.from_numpy(c).to(DEV))
    ref = oracle.voxelize_bwd(gs, gr, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs


def test_voxelize_deterministic(fgs):
    gs = si.gaussians(3000, 16)
    g = fgs.Grid.from_dict(si.grid(48))
    t = dev(gs)
    assert torch.equal(fgs.voxelize(*args(t), g), fgs.voxelize(*args(t), g))


def test_voxelize_backward_matches_oracle(fgs):
    gs = si.gaussians(1500, 17)
    gr = si.grid(40)
    c = si.normals((40, 40, 40), 18)
    g = fgs.voxelize_backward(*args(dev(gs)), fgs.Grid.from_dict(gr), torch.from_numpy(c).to(DEV))
    ref = oracle.voxelize_bwd(gs, gr, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs


def test_voxelize_backward_stored_equals_recomputed(fgs):
    gs = si.gaussians(1000, 19)
    grid = fgs.Grid.from_dict(si.grid(32))
    t = dev(gs)
    c = torch.from_numpy(si.normals((32, 32, 32), 20)).to(DEV)
    ws = fgs.Workspace(DEV)
    fgs.voxelize(*args(t), grid, ws=ws)
    a = fgs.voxelize_backward(*args(t), grid, c, recompute=False, ws=ws)
    b = fgs.voxelize_backward(*args(t), grid, c, recompute=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def _vox_binning(fgs, gs, gr):
    ws = fgs.Workspace(DEV)
    fgs.voxelize(*args(dev(gs)), fgs.Grid.from_dict(gr), ws=ws)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in fgs.binning_dump(ws).items()}


def _mixed_boxes():
    small = si.gaussians(400, 41)
    large = si.gaussians(60, 42, log_scale_mean=math.log(0.15))
    return {k: np.concatenate([small[k], large[k]], axis=-1) for k in small}, si.grid(96)


def _ragged_crop():
    return si.gaussians(900, 15), dict(origin=(-0.31, -0.2, -0.45), spacing=(0.0125, 0.015, 0.011),
                                       dims=(40, 29, 37))


def _clear_of_thresholds():
    # a scene with no decision near a threshold (checked in the test): the
    # whole binning must then be bit-exact
    return si.gaussians(700, 68, log_scale_mean=math.log(0.04)), si.grid(64)


def _crop_64_tiles():
    # a 32^3 crop of the 256^3 grid (the reconstruction loop's TV crop): 64 tiles
    return si.gaussians(6000, 69), dict(origin=(-0.1, -0.12, -0.05), spacing=(1 / 256,) * 3, dims=(32, 32, 32))


def _ragged_27_tiles():
    return si.gaussians(4500, 70), dict(origin=(-0.2, 0.05, -0.1), spacing=(0.011, 0.009, 0.013), dims=(20, 24, 17))


def _wide_64_tiles():
    # 64 tiles over most of the volume: about 15 k keys (four sort tiles of
    # 4096, the last ragged)
    return si.gaussians(6000, 73), dict(origin=(-0.45, -0.43, -0.44), spacing=(0.025,) * 3, dims=(32, 32, 31))


def _wide_64_tiles_dense():
    # about 35 k keys over 64 tiles
    return si.gaussians(14000, 74), dict(origin=(-0.45, -0.43, -0.44), spacing=(0.025,) * 3, dims=(32, 32, 31))


_VOX_CASES = dict(mixed_boxes=_mixed_boxes, ragged_crop=_ragged_crop, clear_of_thresholds=_clear_of_thresholds,
                  crop_64_tiles=_crop_64_tiles, ragged_27_tiles=_ragged_27_tiles, wide_64_tiles=_wide_64_tiles)


@pytest.mark.parametrize("case", ["crop_64_tiles", "ragged_27_tiles", "wide_64_tiles", "wide_64_tiles_dense"])
def test_voxelize_small_grids(fgs, case):
    """Grids of at most 64 tiles (a 6-bit sort, lists split into 16 chunks
    per tile): volume and gradients against the oracle, and the stored
    lists' backward equal to the recomputed one."""
    gs, gr = (_wide_64_tiles_dense if case == "wide_64_tiles_dense" else _VOX_CASES[case])()
    t = dev(gs)
    grid = fgs.Grid.from_dict(gr)
    ws = fgs.Workspace(DEV)
    vol = fgs.voxelize(*args(t), grid, ws=ws)
    assert ws.n_pairs > dict(wide_64_tiles=12000, wide_64_tiles_dense=24576).get(case, 1000)
    assert rel(vol.cpu().numpy(), oracle.voxelize(gs, gr)) < TOL
    nz, ny, nx = gr["dims"][2], gr["dims"][1], gr["dims"][0]
    c = si.normals((nz, ny, nx), 71)
    ct = torch.from_numpy(c).to(DEV)
    g = fgs.voxelize_backward(*args(t), grid, ct, recompute=False, ws=ws)
    ref = oracle.voxelize_bwd(gs, gr, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, ref)
    assert max(errs.values()) < TOL, errs
    for x, y in zip(g, fgs.voxelize_backward(*args(t), grid, ct, recompute=True)):
        assert torch.equal(x, y)


@pytest.mark.parametrize("case", list(_VOX_CASES))
def test_voxel_binning_matches_integer_reference(fgs, case):
    """The voxelizer's integer work against the oracle's FP64 binning
    (oracle.tiles.vox_bin_tiles): per-Gaussian key counts and tile
    rectangles, per-tile lists (stable: ascending Gaussian), sorted keys and
    tile starts, for every Gaussian none of whose decisions lies within
    rounding of its threshold (a box edge at a tile boundary, a tile at the
    culling threshold); bit-exact throughout when there is none. The mixed
    case holds rectangles of at most 512 tiles (whose hit ballots the count
    pass keeps) and larger ones (whose emission repeats the exact test)."""
    gs, gr = _VOX_CASES[case]()
    d = _vox_binning(fgs, gs, gr)
    b = oracle.tiles.vox_bin_tiles(gs, gr)
    if case == "clear_of_thresholds":
        assert not b["ambiguous"].any()
    n = gs["density"].shape[0]
    amb = b["ambiguous"]
    print(f"{case}: {d['n_pairs']} keys, {int(amb.sum())} of {n} Gaussians near a threshold", flush=True)
    assert d["n_records"] == n and d["n_tiles"] == int(np.prod(b["tiles"]))
    off = d["offset"].astype(np.int64)
    gcount = np.diff(off)
    np.testing.assert_array_equal(gcount[~amb], b["count"][~amb])
    nz = ~amb & (gcount > 0)
    np.testing.assert_array_equal(d["rect"][nz, :6].astype(np.int64) & 0xffff, b["rect"][nz])
    if case == "mixed_boxes":
        ntiles = np.prod(b["rect"][:, 3:] - b["rect"][:, :3] + 1, axis=1)
        assert (ntiles > 512).sum() >= 10 and (ntiles <= 512).sum() >= 300
    skeys = d["sorted_keys"].astype(np.int64)
    start = d["tile_start"].astype(np.int64)
    K, T = d["n_pairs"], d["n_tiles"]
    assert start[0] == 0 and start[T] == K and np.all(np.diff(start) >= 0)
    gauss = np.searchsorted(off, d["sorted_vals"].astype(np.int64), side="right") - 1
    amb_ids = set(np.nonzero(amb)[0].tolist())
    for t in range(T):
        lo, hi = start[t], start[t + 1]
        assert np.all(skeys[lo:hi] == t)
        gl = gauss[lo:hi]
        assert np.all(np.diff(gl) > 0), t
        ol = b["sorted_gauss"][b["tile_start"][t]:b["tile_start"][t + 1]]
        assert [x for x in gl.tolist() if x not in amb_ids] == [x for x in ol.tolist() if x not in amb_ids], t
    if not amb.any():
        np.testing.assert_array_equal(skeys, b["sorted_keys"])
        np.testing.assert_array_equal(start, b["tile_start"])
        np.testing.assert_array_equal(d["sorted_vals"].astype(np.int64), b["sorted_slots"])
        np.testing.assert_array_equal(off, b["offset"])


@pytest.mark.parametrize("case", list(_VOX_CASES))
def test_voxel_binning_covers_support(fgs, case):
    """Every (voxel, Gaussian) pair with FP64 d^2 <= 9 - 1e-3 has its tile in
    the Gaussian's list (oracle.tiles.vox_support_tiles, brute force over the
    voxels of each Gaussian's box)."""
    gs, gr = _VOX_CASES[case]()
    d = _vox_binning(fgs, gs, gr)
    off = d["offset"].astype(np.int64)
    gauss = np.searchsorted(off, d["sorted_vals"].astype(np.int64), side="right") - 1
    skeys = d["sorted_keys"].astype(np.int64)
    n = gs["density"].shape[0]
    listed = [set() for _ in range(n)]
    for g_, k_ in zip(gauss.tolist(), skeys.tolist()):
        listed[g_].add(k_)
    sup = oracle.tiles.vox_support_tiles(gs, gr, margin=1e-3)
    missing = [i for i in range(n) if not sup[i] <= listed[i]]
    assert not missing, missing[:10]
    assert sum(len(s) for s in sup) > 1000


def test_near_plane_cull(fgs):
    """Gaussians at or behind the near plane (camera depth <= 0.01) are left
    out of a view, with zero gradient; one just in front of it (depth 0.03,
    a splat wider than the detector) and ordinary ones are kept. Image and
    gradients against the oracle, which culls by the same rule."""
    base = si.gaussians(200, 51)
    # view 0 looks along -x from the source at (1.5, 0, 0): depth = 1.5 - x
    extra_x = np.array([1.495, 1.5, 1.62, 1.47, 1.0], dtype=np.float32)   # depths .005, 0, -.12, .03, .5
    k = extra_x.size
    ext = dict(mean=np.stack([extra_x, np.array([0.0, 0.01, -0.02, 0.004, 0.05]),
                              np.array([0.0, -0.01, 0.02, 0.003, -0.04])]).astype(np.float32),
               log_scale=np.full((3, k), math.log(0.02), np.float32),
               quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, k)),
               density=np.full(k, 0.5, np.float32))
    gs = {key: np.ascontiguousarray(np.concatenate([base[key], ext[key]], axis=-1)) for key in base}
    gd = si.geometry(64)
    ang = np.array([0.0, 0.4, 2.0], dtype=np.float32)
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    img = fgs.project_views(*args(t), geom).cpu().numpy()
    rec = oracle.splat_records(gs, gd, ang)
    n = 200 + k
    assert rec["culled"][n - k:n - k + 3].all() and not rec["culled"][n - 2:n].any()
    ref = oracle.project(gs, gd, ang)
    assert rel(img, ref) < TOL
    c = si.normals((3, 64, 64), 52)
    g = fgs.project_views_backward(*args(t), geom, torch.from_numpy(c).to(DEV))
    gref = oracle.project_bwd(gs, gd, ang, c.astype(np.float64), band=BAND)
    errs = grads_rel(g, gref)
    assert max(errs.values()) < TOL, errs
    # view 0 alone: the three culled Gaussians contribute nothing and get
    # exactly zero gradient; the one just in front of the plane does not
    g0 = fgs.project_views_backward(*args(t), geom, torch.from_numpy(c[:1].copy()).to(DEV), 0, 1)
    for gg in g0:
        a_ = gg.detach().cpu().numpy()
        assert np.all(a_[..., n - k:n - k + 3] == 0.0)
        assert np.any(a_[..., n - 2] != 0.0)
    img0 = fgs.project_views(*args(t), geom, 0, 1).cpu().numpy()
    keep = {key: np.ascontiguousarray(np.delete(gs[key], [n - k, n - k + 1, n - k + 2], axis=-1)) for key in gs}
    img0_kept = fgs.project_views(*args(dev(keep)), geom, 0, 1).cpu().numpy()
    assert rel(img0, img0_kept) < 1e-6


# ------------------------------------------------------------------ losses, optimiser, phantom

def test_l1_psnr_adam(fgs):
    a = si.normals((3, 17, 23), 21)
    b = si.normals((3, 17, 23), 22)
    b[0, 0, :5] = a[0, 0, :5]  # exact ties: sign(0) = 0
    loss, grad = fgs.l1_loss_grad(torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV))
    rl, rg = oracle.l1_loss_grad(a, b)
    assert loss.item() == pytest.approx(rl, rel=1e-6)
    np.testing.assert_allclose(grad.cpu().numpy(), rg, rtol=1e-7, atol=0)
    ps = fgs.psnr(torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV), float(b.max()))
    assert ps.item() == pytest.approx(oracle.psnr(a, b), abs=1e-4)
    p = si.normals(1000, 23); gg = si.normals(1000, 24)
    tp, tg = torch.from_numpy(p).to(DEV), torch.from_numpy(gg).to(DEV)
    m = torch.zeros_like(tp); v = torch.zeros_like(tp)
    rp, rm, rv = p.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        fgs.adam_step(tp, tg, m, v, step, 0.01, eps=1e-8)
        rp, rm, rv = oracle.adam_step(rp, gg.astype(np.float64), rm, rv, step, 0.01, eps=1e-8)
    np.testing.assert_allclose(tp.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)


def test_fp32_scalar_reductions_at_full_size(fgs):
    """The losses and PSNR reduce in FP32 (compensated per-thread sums, then
    pairwise trees). At the standard scan's size (75 views of 512^2, about
    20 M values) they stay within 1e-6 of the FP64 sums."""
    a = np.abs(si.normals((75, 512, 512), 25)) * 0.3
    b = np.abs(si.normals((75, 512, 512), 26)) * 0.3
    ta, tb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    loss, _ = fgs.l1_loss_grad(ta, tb, want_grad=False)
    rl, _ = oracle.l1_loss_grad(a, b)
    assert loss.item() == pytest.approx(rl, rel=1e-6)
    peak = float(b.max())
    ps = fgs.psnr(ta, tb, peak)
    assert ps.item() == pytest.approx(oracle.psnr(a, b), abs=1e-5)
    v = torch.from_numpy(a[:64].reshape(64, 512, 512)[:, :256, :256].copy()).to(DEV)
    tl, _ = fgs.tv_loss_grad(v, scale=1.0, want_grad=False)
    rtl, _ = oracle.tv_loss_grad(v.cpu().numpy(), scale=1.0)
    assert tl.item() == pytest.approx(rtl, rel=1e-6)


def test_phantom_matches_oracle(fgs):
    ph = si.phantom(10, 100)
    tph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in ph.items()}
    gd = si.geometry(64)
    ang = si.angles(6)
    img = fgs.phantom_project(tph, fgs.Geometry.from_dict(gd, ang)).cpu().numpy()
    ref = oracle.phantom_project(ph, gd, ang)
    assert rel(img, ref) < 1e-6
    gr = si.grid(48)
    vol = fgs.phantom_voxelize(tph, fgs.Grid.from_dict(gr)).cpu().numpy()
    vref = oracle.phantom_volume(ph, gr)
    # the indicator may differ only on voxels within FP64 rounding of a surface
    assert np.count_nonzero(np.abs(vol - vref) > 1e-6) <= 2


# ------------------------------------------------------------------ full-size (standard scan)

@pytest.fixture(scope="module")
def scan_case(fgs):
    cfg = si.CONFIGS["scan"]
    gs = si.gaussians(cfg["n_gauss"], cfg["seed"])
    gd = si.geometry(cfg["det"])
    ang = si.angles(cfg["n_views"])
    return cfg, gs, gd, ang


def test_full_size_projection_sampled(fgs, scan_case):
    """50,000 Gaussians, all 75 views of 512x512 in one call (the benchmark's
    launch configuration); 600 sampled pixels in each of 4 views vs the oracle."""
    cfg, gs, gd, ang = scan_case
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*args(dev(gs)), geom).cpu().numpy()
    rng = np.random.default_rng(5)
    for v in (0, 17, 41, 74):
        ys = rng.integers(0, 512, 600)
        xs = rng.integers(0, 512, 600)
        ref = oracle.project_points(gs, gd, float(ang[v]), xs + 0.5, ys + 0.5)
        assert rel(img[v, ys, xs], ref) < TOL, v


def _check_every_element(got, ref, band, what):
    """Element by element: within 1e-5 max|ref| of the bracket that support
    decisions near the cutoff allow (band: the FP64 contributions of the
    pairs with |d^2 - 9| <= 1e-3, which FP32 may put on either side; one such
    pair of a dense Gaussian moves a voxel by up to e^-4.5 rho, which can
    exceed 1e-4 max|ref|), and relative L2 <= 1e-4 overall."""
    err = np.abs(got.astype(np.float64) - ref)
    top = np.abs(ref).max()
    beyond = np.maximum(err - band, 0.0)
    print(f"{what}: max |diff| {err.max() / top:.2e} of max|ref|, beyond the band {beyond.max() / top:.2e}; "
          f"rel-L2 {rel(got, ref):.2e}; {np.count_nonzero(band)} elements touch the band", flush=True)
    assert beyond.max() <= 1e-5 * top, what
    assert rel(got, ref) < TOL, what


def test_full_size_whole_views_every_pixel(fgs, scan_case):
    """Three complete 512x512 views (the first, a middle and the last) of the
    75-view call the benchmark times, every pixel against the oracle."""
    cfg, gs, gd, ang = scan_case
    geom = fgs.Geometry.from_dict(gd, ang)
    img = fgs.project_views(*args(dev(gs)), geom).cpu().numpy()
    for v in (0, 41, 74):
        ref, band = oracle.project_banded(gs, gd, ang[v:v + 1])
        _check_every_element(img[v], ref[0], band[0], f"view {v}")


def test_full_size_single_view_calls_every_pixel(fgs, scan_case):
    """One-view calls of the standard scan (the reconstruction loop's unit:
    1024 tiles, lists split into work units of about 128 keys), with the
    pair count read back and at a fixed key capacity: every pixel against
    the oracle, the two calls bit-identical; their backward equals the
    batched call's for that view."""
    cfg, gs, gd, ang = scan_case
    geom = fgs.Geometry.from_dict(gd, ang)
    t = dev(gs)
    for v in (7, 52):
        ws = fgs.Workspace(DEV)
        img = fgs.project_views(*args(t), geom, v, 1, ws=ws).cpu().numpy()
        ref, band = oracle.project_banded(gs, gd, ang[v:v + 1])
        _check_every_element(img[0], ref[0], band[0], f"single view {v}")
        wc = fgs.Workspace(DEV)
        wc.set_capacity(int(1.3 * ws.n_pairs))
        img_c = fgs.project_views(*args(t), geom, v, 1, ws=wc).cpu().numpy()
        assert np.array_equal(img, img_c)
        c = torch.from_numpy(si.normals((1, 512, 512), 40 + v)).to(DEV)
        g1 = fgs.project_views_backward(*args(t), geom, c, v, 1, recompute=False, ws=wc)
        g2 = fgs.project_views_backward(*args(t), geom, c, v, 1, recompute=True)
        for x, y in zip(g1, g2):
            assert torch.equal(x, y)
        assert wc.overflowed() == (False, 0)


def test_full_size_voxel_slab_every_voxel(fgs, scan_case):
    """An 8-slice slab (z = 124..131) of the 256^3 volume that one voxelize
    call over the whole grid writes, every voxel against the oracle."""
    cfg, gs, gd, ang = scan_case
    gr = si.grid(cfg["vol"])
    vol = fgs.voxelize(*args(dev(gs)), fgs.Grid.from_dict(gr)).cpu().numpy()
    h = gr["spacing"][0]
    slab = dict(origin=(gr["origin"][0], gr["origin"][1], gr["origin"][2] + 124 * h), spacing=gr["spacing"],
                dims=(cfg["vol"], cfg["vol"], 8))
    ref, band = oracle.voxelize_banded(gs, slab)
    _check_every_element(vol[124:132], ref, band, "slab z 124-131")


def test_full_size_projection_gradients_sampled(fgs, scan_case):
    """Gradient of <c, I> over all 75 views for 64 random Gaussians vs the
    oracle's analytic gradient (each Gaussian's gradient depends only on its
    own support)."""
    cfg, gs, gd, ang = scan_case
    geom = fgs.Geometry.from_dict(gd, ang)
    c = si.normals((75, 512, 512), 77)
    g = fgs.project_views_backward(*args(dev(gs)), geom, torch.from_numpy(c).to(DEV))
    sel = np.random.default_rng(6).choice(cfg["n_gauss"], 64, replace=False)
    ref = oracle.project_bwd(gs, gd, ang, c, sel=sel, band=BAND)
    errs = grads_rel(g, ref, sel)
    assert max(errs.values()) < TOL, errs


def test_full_size_voxelize_sampled(fgs, scan_case):
    cfg, gs, gd, ang = scan_case
    gr = si.grid(cfg["vol"])
    vol = fgs.voxelize(*args(dev(gs)), fgs.Grid.from_dict(gr)).cpu().numpy()
    rng = np.random.default_rng(7)
    idx = rng.integers(0, cfg["vol"], size=(3000, 3))
    h = gr["spacing"][0]
    pts = -0.5 + (idx + 0.5) * h
    ref = oracle.field_points(gs, pts, kappa=3.0)
    got = vol[idx[:, 2], idx[:, 1], idx[:, 0]]
    assert rel(got, ref) < TOL


def test_full_size_voxelize_gradients_sampled(fgs, scan_case):
    """Voxelizer gradient at 256^3 for 64 random Gaussians vs the oracle."""
    cfg, gs, gd, ang = scan_case
    gr = si.grid(cfg["vol"])
    c = si.normals((cfg["vol"],) * 3, 78)
    g = fgs.voxelize_backward(*args(dev(gs)), fgs.Grid.from_dict(gr), torch.from_numpy(c).to(DEV))
    sel = np.random.default_rng(8).choice(cfg["n_gauss"], 64, replace=False)
    ref = oracle.voxelize_bwd(gs, gr, c, sel=sel, band=BAND)
    errs = grads_rel(g, ref, sel)
    assert max(errs.values()) < TOL, errs


# ------------------------------------------------------------------ initialisation (Sec. 3.1)

def test_fdk_matches_oracle(fgs):
    ph = si.phantom(10, 100)
    gd = si.geometry(96)
    ang = si.angles(24)
    img = oracle.phantom_project(ph, gd, ang).astype(np.float32)
    gr = dict(origin=(-0.5, -0.45, -0.4), spacing=(1 / 40, 0.9 / 36, 0.8 / 33), dims=(40, 36, 33))
    vol = fgs.fdk(torch.from_numpy(img).to(DEV), fgs.Geometry.from_dict(gd, ang), fgs.Grid.from_dict(gr))
    ref = oracle.fdk(img, gd, ang, gr)
    assert rel(vol.cpu().numpy(), ref) < TOL


@pytest.mark.parametrize("weighting", ["gradient", "intensity"])
def test_gradient_init_matches_oracle(fgs, weighting):
    """Same FP32 volume and the same uniforms: identical voxel choices (the
    integer decision), means, densities and nearest-neighbour scales, for the
    gradient rule and the intensity-sampling baseline."""
    ph = si.phantom(12, 105)
    gr = si.grid(40)
    vol = oracle.phantom_volume(ph, gr).astype(np.float32)
    vol += 0.02 * si.normals(vol.shape, 106)  # FDK-like noise
    n = 3000
    u = np.random.Generator(np.random.PCG64(107)).random((4, n))
    ref = oracle.gradient_init(vol, gr, u, weighting=weighting)
    out = fgs.gradient_init(torch.from_numpy(vol).to(DEV), fgs.Grid.from_dict(gr), torch.from_numpy(u).to(DEV),
                            weighting=weighting)
    mean, ls, quat, dens = (t.cpu().numpy().astype(np.float64) for t in out)
    h = np.array(gr["spacing"])
    o = np.array(gr["origin"])
    vox = np.floor((mean.T - o) / h).astype(np.int64)
    nx, ny, nz = gr["dims"]
    k = vox[:, 0] + nx * (vox[:, 1] + ny * vox[:, 2])
    # the voxel follows from the mean unless the in-voxel offset is within FP32 rounding of an edge
    clear = np.all((u[1:] > 1e-5) & (u[1:] < 1 - 1e-5), axis=0)
    np.testing.assert_array_equal(k[clear], ref["voxel"][clear])
    np.testing.assert_allclose(mean, ref["mean"], rtol=0, atol=1e-6)
    assert rel(dens, ref["density"]) < TOL
    assert rel(ls, ref["log_scale"]) < TOL
    np.testing.assert_array_equal(quat, ref["quat"])


# ------------------------------------------------------------------ TV prior and the crop step

@pytest.mark.parametrize("shape", [(32, 32, 32), (33, 29, 37), (1, 1, 5)])
def test_tv_loss_grad_matches_oracle(fgs, shape):
    v = si.normals(shape, 90 + shape[0])
    loss, g = fgs.tv_loss_grad(torch.from_numpy(v).to(DEV), scale=0.05)
    rl, rg = oracle.tv_loss_grad(v, scale=0.05)
    assert abs(float(loss.item()) - rl) <= 1e-6 * abs(rl)
    np.testing.assert_allclose(g.cpu().numpy(), rg, rtol=1e-6, atol=1e-12)


def test_voxelize_backward_accumulates(fgs):
    """opts.accumulate adds the crop's gradient to the projection gradient."""
    gs = si.gaussians(3000, 91)
    d = dev(gs)
    gr = fgs.Grid(tuple(np.float32(-0.5 + k / 64) for k in (5, 17, 40)), (np.float32(1 / 64),) * 3, (32, 32, 32))
    c = torch.from_numpy(si.normals((32, 32, 32), 92)).to(DEV)
    fresh = fgs.voxelize_backward(*args(d), gr, c)
    base = [torch.from_numpy(si.normals(t.shape, 93 + k)).to(DEV) for k, t in enumerate(fresh)]
    acc = [b.clone() for b in base]
    fgs.voxelize_backward(*args(d), gr, c, out=acc, accumulate=True)
    for a, b, f in zip(acc, base, fresh):
        np.testing.assert_allclose(a.cpu().numpy(), (b + f).cpu().numpy(), rtol=1e-6, atol=1e-6)
    ref = oracle.voxelize_bwd(gs, dict(origin=gr.origin, spacing=gr.spacing, dims=gr.dims), c.cpu().numpy(),
                              band=BAND)
    errs = grads_rel(fresh, ref)
    assert max(errs.values()) < TOL, errs


@pytest.mark.parametrize("shape", [(2, 64, 64), (3, 45, 71), (1, 7, 5)])
def test_ssim_loss_grad_matches_oracle(fgs, shape):
    x = np.abs(si.normals(shape, 94)) * 0.5
    y = np.abs(si.normals(shape, 95)) * 0.5
    xd, yd = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    loss, g = fgs.ssim_loss_grad(xd, yd, scale=0.25)
    rl, rg = oracle.ssim_loss_grad(x, y, scale=0.25)
    assert abs(float(loss.item()) - rl) <= 1e-5 * abs(rl)
    assert rel(g.cpu().numpy(), rg) < TOL
    base = torch.from_numpy(si.normals(shape, 96)).to(DEV)
    acc = base.clone()
    fgs.ssim_loss_grad(xd, yd, scale=0.25, grad=acc, accumulate=True)
    np.testing.assert_allclose(acc.cpu().numpy(), (base + g).cpu().numpy(), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("shape", [(20, 24, 28), (1, 9, 13), (150, 37, 21), (70, 16, 33), (9, 40, 17)])
def test_ssim3d_loss_grad_matches_oracle(fgs, shape):
    """[nz][ny][nx] volumes: one and several z-chunks of the fused kernel (64
    output slices each, the last one ragged), fewer slices than the window,
    and x/y extents that are not multiples of its 16 x 16 tiles."""
    x = np.abs(si.normals(shape, 97)) * 0.5
    y = np.abs(si.normals(shape, 98)) * 0.5
    xd, yd = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    loss, g = fgs.ssim3d_loss_grad(xd, yd, scale=0.2)
    rl, rg = oracle.ssim3d_loss_grad(x, y, scale=0.2)
    assert abs(float(loss.item()) - rl) <= 1e-5 * abs(rl)
    assert rel(g.cpu().numpy(), rg) < TOL


def test_ablation_switches_keep_the_results(fgs):
    """Switching parts of the rasterizer's design off (for the Table 3
    analogue) changes the work, not the result. Unculled quadrants only add
    exact zeros, but they shift the positions in the quadrant lists, and the
    forward sums each list's even and odd positions separately (rounding
    only); square boxes list more tiles, so the sums group their terms
    differently (rounding only); the per-pixel atomic backward sums the same
    terms in another, unordered, way."""
    gs = si.gaussians(3000, 99)
    d = dev(gs)
    gd = si.geometry(96)
    ang = si.angles(5)
    geom = fgs.Geometry.from_dict(gd, ang)
    c = torch.from_numpy(si.normals((5, 96, 96), 100)).to(DEV)
    base_img = fgs.project_views(*args(d), geom)
    base_g = fgs.project_views_backward(*args(d), geom, c)
    for flag in (fgs.ops.ABLATE_SQUARE_BOX, fgs.ops.ABLATE_QUADRANT_CULL, fgs.ops.ABLATE_PER_PIXEL_BWD, 7):
        img = fgs.project_views(*args(d), geom, ablate=flag)
        if flag & (fgs.ops.ABLATE_SQUARE_BOX | fgs.ops.ABLATE_QUADRANT_CULL):
            assert rel(img.cpu().numpy(), base_img.cpu().numpy()) < 1e-6, flag
        else:
            assert torch.equal(img, base_img), flag
        g = fgs.project_views_backward(*args(d), geom, c, ablate=flag)
        for a, b in zip(g, base_g):
            assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-5, flag
