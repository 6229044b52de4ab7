"""The workspace-free rasterizer forward (fgs_project_views_fwd_noalloc)
against the workspace entry point it shares its kernels with.

Both run the same kernels in the same order on the same seeded inputs, so
the images must be bit-identical. Two calls in a row, the second smaller,
check that the scratch array's leftovers from the first call do not leak
into the second. A call beyond the scratch maximum must be refused with
FGS_E_CAPACITY before any kernel runs, leaving the output untouched.
"""
import ctypes

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


def _case(fgs, n, seed, det, views):
    gs = si.gaussians(n, seed)
    t = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(DEV) for k, v in gs.items()}
    geom = fgs.Geometry.from_dict(si.geometry(det), si.angles(views), DEV)
    return (t["mean"], t["log_scale"], t["quat"], t["density"]), geom


def _noalloc(fgs, params, geom, view_begin, view_count, out):
    from paper_2604_01844_amd import _abi as A
    g = A.fgs_gaussians(params[3].numel(), *(A.ptr(p) for p in params))
    gm = geom.struct()
    o = A.fgs_opts(3.0, 1e-2, 1, 0, 0, A.FGS_MODEL_SPLAT, None)
    return A.lib().fgs_project_views_fwd_noalloc(ctypes.byref(g), ctypes.byref(gm), view_begin, view_count,
                                                 ctypes.byref(o), A.ptr(out), A.stream_ptr(out.device))


def test_noalloc_forward_equals_workspace_forward_twice(fgs):
    cases = [(_case(fgs, 20000, 11, 256, 6), 1, 4),   # first call: 4 views of 256^2, 20k Gaussians
             (_case(fgs, 700, 12, 72, 3), 0, 2)]      # second, smaller: 2 ragged-free 72^2 views
    for (params, geom), vb, vc in cases:
        ref = fgs.project_views(*params, geom, vb, vc)
        out = torch.full_like(ref, float("nan"))
        code = _noalloc(fgs, params, geom, vb, vc, out)
        assert code == 0, fgs.lib().fgs_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"max |diff| {float((out - ref).abs().max())}"
        assert float(ref.abs().max()) > 0


def test_noalloc_forward_refuses_beyond_scratch(fgs):
    from paper_2604_01844_amd import _abi as A
    # 75 views x 50k Gaussians: the per-record arrays alone (about 400 MB)
    # exceed the 64 MiB scratch, so the call stops before launching anything
    params, geom = _case(fgs, 50000, 1, 512, 75)
    out = torch.full((75, 512, 512), 7.0, device=DEV)
    code = _noalloc(fgs, params, geom, 0, 75, out)
    assert code == A.FGS_E_CAPACITY
    assert "scratch" in fgs.lib().fgs_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # the entry point still works after a refusal
    params, geom = _case(fgs, 700, 12, 72, 3)
    ref = fgs.project_views(*params, geom, 0, 3)
    out = torch.empty_like(ref)
    assert _noalloc(fgs, params, geom, 0, 3, out) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
