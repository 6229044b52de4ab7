"""The one-call optimiser step (fgs_recon_step) and the fixed key capacity
(fgs_workspace.key_capacity) against the separate library calls they
compose.

The step issues the same kernels on the same inputs as the separate calls
(forward, L1, SSIM, backward, crop voxelization, TV, voxelizer backward,
Adam), so after a few steps from the same state the parameters, moments and
gradients must be bit-identical. With a fixed capacity the lists are the
same as with a read-back pair count; a call that needs more pairs than its
capacity bins nothing, reports it, and leaves no gradient behind.
"""
import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def fgs():
    import paper_2604_01844_amd as m
    m.lib()
    return m


def _scene(fgs, n=3000, views=8, det=128, vol=64):
    gs = si.gaussians(n, 21)
    geom = fgs.Geometry.from_dict(si.geometry(det), si.angles(views), DEV)
    grid = fgs.Grid.from_dict(si.grid(vol))
    ph = {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in si.phantom(10, 105).items()}
    gt = fgs.phantom_project(ph, geom)
    return gs, geom, grid, gt


def _model(fgs, gs):
    from paper_2604_01844_amd import recon
    t = [torch.from_numpy(np.ascontiguousarray(gs[k], dtype=np.float32)).to(DEV)
         for k in ("mean", "log_scale", "quat", "density")]
    return recon.GaussianModel(*t)


@pytest.mark.parametrize("ssim, tv_weight, graphs", [(0.0, 0.0, False), (0.25, 0.05, False), (0.25, 0.05, True)])
def test_native_step_equals_separate_calls(fgs, ssim, tv_weight, graphs):
    from paper_2604_01844_amd import recon
    gs, geom, grid, gt = _scene(fgs)
    adam = recon.AdamConfig()
    views = [3, 1, 6, 0, 5]
    a, b = _model(fgs, gs), _model(fgs, gs)
    tv_a = recon.CropTV(grid, tv_weight, 32, DEV) if tv_weight else None
    tv_b = recon.CropTV(grid, tv_weight, 32, DEV) if tv_weight else None
    step = recon.ViewStep(a, geom, adam, ssim_weight=ssim, tv=tv_a, graphs=graphs)
    rng_a = np.random.Generator(np.random.PCG64(7))
    for v in views:
        step(v, gt[v], rng_a)
    rng_b = np.random.Generator(np.random.PCG64(7))
    ws_p, ws_l, ws_s = fgs.Workspace(DEV), fgs.Workspace(DEV, 1 << 16), fgs.Workspace(DEV)
    img = torch.empty((1, geom.det_h, geom.det_w), device=DEV)
    for v in views:
        fgs.project_views(*b.params, geom, v, 1, ws=ws_p, out=img)
        l1, g = fgs.l1_loss_grad(img, gt[v:v + 1], ws=ws_l)
        losses = [float(l1)]
        if ssim:
            ls, _ = fgs.ssim_loss_grad(img, gt[v:v + 1], scale=ssim, ws=ws_s, grad=g, accumulate=True)
            losses.append(float(ls))
        fgs.project_views_backward(*b.params, geom, g, v, 1, recompute=False, ws=ws_p, out=b.grads)
        if tv_b is not None:
            losses.append(float(tv_b.add_grad(b.params, b.grads, rng_b)))
        b.adam(adam)
    torch.cuda.synchronize()
    assert step.check_overflow() == 0
    # the last step's loss terms: the same sums, added up in another order
    got = step.loss.cpu().numpy()[:len(losses)]
    np.testing.assert_allclose(got, losses, rtol=2e-5, atol=0)
    for name, xa, xb in (("params", a.params, b.params), ("m", a.m, b.m), ("v", a.v, b.v),
                         ("grads", a.grads, b.grads)):
        for k, (ta, tb) in enumerate(zip(xa, xb)):
            assert torch.equal(ta, tb), (name, k, float((ta - tb).abs().max()))
    assert a.step == b.step == len(views)
    assert float(step.img.abs().max()) > 0


def test_fixed_capacity_lists_equal_read_back_lists(fgs):
    """Rasterizer and voxelizer forward/backward with key_capacity set (no
    wait) give the same images, volumes and gradients as with the pair count
    read back, and the same sorted lists."""
    gs, geom, grid, gt = _scene(fgs, views=4)
    t = [torch.from_numpy(np.ascontiguousarray(gs[k], dtype=np.float32)).to(DEV)
         for k in ("mean", "log_scale", "quat", "density")]
    ws0 = fgs.Workspace(DEV)
    img0 = fgs.project_views(*t, geom, ws=ws0)
    K = ws0.n_pairs
    d0 = fgs.binning_dump(ws0)
    c = torch.from_numpy(si.normals((4, 128, 128), 3)).to(DEV)
    g0 = fgs.project_views_backward(*t, geom, c, recompute=False, ws=ws0)
    wsc = fgs.Workspace(DEV)
    wsc.set_capacity(int(K * 1.7) + 123)
    img1 = fgs.project_views(*t, geom, ws=wsc)
    d1 = fgs.binning_dump(wsc)
    g1 = fgs.project_views_backward(*t, geom, c, recompute=False, ws=wsc)
    assert torch.equal(img0, img1)
    for x, y in zip(g0, g1):
        assert torch.equal(x, y)
    for key in ("sorted_keys", "sorted_vals"):
        assert torch.equal(d0[key][:K], d1[key][:K]), key
    assert torch.equal(d0["tile_ranges"], d1["tile_ranges"])
    assert wsc.overflowed() == (False, 0)
    wv0, wv1 = fgs.Workspace(DEV), fgs.Workspace(DEV)
    vol0 = fgs.voxelize(*t, grid, ws=wv0)
    wv1.set_capacity(wv0.n_pairs + 1)
    vol1 = fgs.voxelize(*t, grid, ws=wv1)
    assert torch.equal(vol0, vol1)
    cv = torch.from_numpy(si.normals((64, 64, 64), 4)).to(DEV)
    for x, y in zip(fgs.voxelize_backward(*t, grid, cv, recompute=False, ws=wv0),
                    fgs.voxelize_backward(*t, grid, cv, recompute=False, ws=wv1)):
        assert torch.equal(x, y)
    assert wv1.overflowed() == (False, 0)


def test_capacity_overflow_bins_nothing_and_reports(fgs):
    """Capacities below the pairs needed: the forward renders zero, the
    backward gives zero gradients, the voxelizer likewise, and the overflow
    words hold the pairs needed; an overflowed first optimiser step leaves
    the parameters where they were (zero gradient, zero moments)."""
    from paper_2604_01844_amd import recon
    gs, geom, grid, gt = _scene(fgs, views=2)
    t = [torch.from_numpy(np.ascontiguousarray(gs[k], dtype=np.float32)).to(DEV)
         for k in ("mean", "log_scale", "quat", "density")]
    ws0 = fgs.Workspace(DEV)
    fgs.project_views(*t, geom, ws=ws0)
    K = ws0.n_pairs
    ws = fgs.Workspace(DEV)
    ws.set_capacity(K // 3)
    img = fgs.project_views(*t, geom, ws=ws)
    assert float(img.abs().max()) == 0.0
    c = torch.from_numpy(si.normals((2, 128, 128), 5)).to(DEV)
    for x in fgs.project_views_backward(*t, geom, c, recompute=False, ws=ws):
        assert float(x.abs().max()) == 0.0
    assert ws.overflowed() == (True, K)
    assert ws.overflowed() == (False, 0)          # the read cleared it
    wv0 = fgs.Workspace(DEV)
    fgs.voxelize(*t, grid, ws=wv0)
    wv = fgs.Workspace(DEV)
    wv.set_capacity(max(1, wv0.n_pairs // 2))
    assert float(fgs.voxelize(*t, grid, ws=wv).abs().max()) == 0.0
    assert wv.overflowed() == (True, wv0.n_pairs)
    # a 32^3 crop (64 tiles) the same way
    crop = fgs.Grid.from_dict(dict(origin=(-0.1, -0.1, -0.1), spacing=(1 / 256,) * 3, dims=(32, 32, 32)))
    wc0, wc = fgs.Workspace(DEV), fgs.Workspace(DEV)
    assert float(fgs.voxelize(*t, crop, ws=wc0).abs().max()) > 0.0
    wc.set_capacity(max(1, wc0.n_pairs // 2))
    assert float(fgs.voxelize(*t, crop, ws=wc).abs().max()) == 0.0
    cc = torch.from_numpy(si.normals((32, 32, 32), 6)).to(DEV)
    for x in fgs.voxelize_backward(*t, crop, cc, recompute=False, ws=wc):
        assert float(x.abs().max()) == 0.0
    assert wc.overflowed() == (True, wc0.n_pairs)
    wc.set_capacity(wc0.n_pairs)
    assert torch.equal(fgs.voxelize(*t, crop, ws=wc), fgs.voxelize(*t, crop, ws=wc0))
    model = _model(fgs, gs)
    before = [p.clone() for p in model.params]
    step = recon.ViewStep(model, geom, recon.AdamConfig())
    step.ws_proj.set_capacity(100)
    step(0, gt[0])
    torch.cuda.synchronize()
    for p, q in zip(model.params, before):
        assert torch.equal(p, q)
    assert step.check_overflow() == 1
    assert int(step.ws_proj.s.key_capacity) > K // 2
    step(1, gt[1])
    torch.cuda.synchronize()
    assert step.check_overflow() == 0
    assert any(not torch.equal(p, q) for p, q in zip(model.params, before))


def test_graph_replays_equal_direct_steps(fgs):
    """Steps replayed from per-view HIP graphs (fgs_step_graph_launch) give
    the parameters, moments and gradients of the same steps issued directly
    (fgs_recon_step), bit for bit, after every step: views replayed several
    times, the crop moved and Adam's step advanced between replays, with
    other eager GPU work and synchronisations in between."""
    from paper_2604_01844_amd import recon
    gs, geom, grid, gt = _scene(fgs)
    adam = recon.AdamConfig()
    a, b = _model(fgs, gs), _model(fgs, gs)
    sa = recon.ViewStep(a, geom, adam, ssim_weight=0.25, tv=recon.CropTV(grid, 0.05, 32, DEV), graphs=True)
    sb = recon.ViewStep(b, geom, adam, ssim_weight=0.25, tv=recon.CropTV(grid, 0.05, 32, DEV), graphs=False)
    ra = np.random.Generator(np.random.PCG64(11))
    rb = np.random.Generator(np.random.PCG64(11))
    other = torch.zeros(4096, device=DEV)
    for k, v in enumerate([2, 5, 2, 2, 7, 5, 2, 7]):
        sa(v, gt[v], ra)
        other.add_(float(k))                     # eager work between replays
        sb(v, gt[v], rb)
        torch.cuda.synchronize()
        for name, xa, xb in (("params", a.params, b.params), ("m", a.m, b.m), ("v", a.v, b.v),
                             ("grads", a.grads, b.grads)):
            for j, (ta, tb) in enumerate(zip(xa, xb)):
                assert torch.equal(ta, tb), (k, v, name, j, float((ta - tb).abs().max()))
        assert torch.equal(sa.loss, sb.loss), k
    assert sorted(sa._graphs) == [2, 5, 7]
    assert float(other[0]) == sum(range(8))
    assert sa.check_overflow() == 0 and sb.check_overflow() == 0


def test_graph_capture_after_workspace_growth(fgs):
    """Captures that stop on a workspace to grow, first in the crop branch
    (which runs on a second stream), then in the view's forward, leave no
    error behind: the capture after the growth succeeds and its replays
    equal direct steps bit for bit."""
    from paper_2604_01844_amd import recon
    gs, geom, grid, gt = _scene(fgs)
    adam = recon.AdamConfig()
    a, b = _model(fgs, gs), _model(fgs, gs)
    sa = recon.ViewStep(a, geom, adam, ssim_weight=0.25, tv=recon.CropTV(grid, 0.05, 32, DEV), graphs=True)
    sb = recon.ViewStep(b, geom, adam, ssim_weight=0.25, tv=recon.CropTV(grid, 0.05, 32, DEV), graphs=False)
    for st in (sa, sb):
        st.ws_proj.set_capacity(int(st.ws_proj.s.key_capacity) * 16)
        st.ws_crop.set_capacity(int(st.ws_crop.s.key_capacity) * 16)
    ra = np.random.Generator(np.random.PCG64(12))
    rb = np.random.Generator(np.random.PCG64(12))
    for k, v in enumerate([1, 4, 1]):
        sa(v, gt[v], ra)
        sb(v, gt[v], rb)
        torch.cuda.synchronize()
        for name, xa, xb in (("params", a.params, b.params), ("m", a.m, b.m), ("v", a.v, b.v),
                             ("grads", a.grads, b.grads)):
            for j, (ta, tb) in enumerate(zip(xa, xb)):
                assert torch.equal(ta, tb), (k, v, name, j)
    assert sorted(sa._graphs) == [1, 4]
    assert sa.check_overflow() == 0 and sb.check_overflow() == 0


def test_graph_capture_needs_fixed_capacity(fgs):
    """A captured step may not wait for the GPU: capture without key_capacity
    in the rasterizer workspace is refused before anything is recorded."""
    import ctypes
    from paper_2604_01844_amd import recon, _abi as A
    gs, geom, grid, gt = _scene(fgs, views=2)
    st = recon.ViewStep(_model(fgs, gs), geom, recon.AdamConfig(), graphs=True)
    st._bind()
    st.ws_proj.s.key_capacity = 0
    st.sp.step = 1
    h = ctypes.c_void_p()
    code = A.lib().fgs_step_graph_capture(*st._args(0, gt[0], None), ctypes.byref(h))
    assert code == A.FGS_E_INVALID and not h.value
    assert "key_capacity" in A.lib().fgs_last_error().decode()
