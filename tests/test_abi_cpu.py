"""The C-ABI library loads and exports every symbol include/factgs.h declares;
host-side argument validation (no GPU work) behaves as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "factgs.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fgs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("fgs_project_views_fwd", "fgs_project_views_bwd", "fgs_voxelize_fwd", "fgs_voxelize_bwd"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2604_01844_amd import _abi
    lib = _abi.lib()
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert s in _abi.SIGNATURES, s
    assert set(_abi.SIGNATURES) == set(declared_symbols())


def test_version_and_error_strings():
    from paper_2604_01844_amd import _abi
    lib = _abi.lib()
    assert lib.fgs_version().decode().startswith("factgs")
    assert isinstance(lib.fgs_last_error().decode(), str)


def test_validation_rejects_bad_arguments_without_gpu_work():
    from paper_2604_01844_amd import _abi as A
    lib = A.lib()
    ws = A.fgs_workspace()
    o = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1)
    # null Gaussians
    assert lib.fgs_project_views_fwd(None, None, 0, 1, ctypes.byref(o), None, ctypes.byref(ws), None) == A.FGS_E_INVALID
    g = A.fgs_gaussians(10, 16, 16, 16, 16)  # fake non-null pointers, never dereferenced on invalid input
    gm = A.fgs_geom(A.FGS_CONE, 4, 16, 1.5, 2.0, 64, 64, 0.04, 0.04, 0.0, 0.0)
    # view range out of bounds
    assert lib.fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 3, 2, ctypes.byref(o), 16,
                                     ctypes.byref(ws), None) == A.FGS_E_INVALID
    assert "view range" in lib.fgs_last_error().decode()
    # kappa <= 0
    bad = A.fgs_opts(kappa=0.0, near_plane=1e-2, recompute=1)
    assert lib.fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 0, 1, ctypes.byref(bad), 16,
                                     ctypes.byref(ws), None) == A.FGS_E_INVALID
    # unknown ablation bits, unknown model, ablation of the ray-exact model
    for bad in (A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1, ablate=8),
                A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1, model=2)):
        assert lib.fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 0, 1, ctypes.byref(bad), 16,
                                         ctypes.byref(ws), None) == A.FGS_E_INVALID
    abl = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1, ablate=1, model=A.FGS_MODEL_RAY_EXACT)
    assert lib.fgs_project_views_fwd(ctypes.byref(g), ctypes.byref(gm), 0, 1, ctypes.byref(abl), 16,
                                     ctypes.byref(ws), None) == A.FGS_E_UNSUPPORTED
    # the voxelizer has one model
    gr1 = A.fgs_grid((ctypes.c_float * 3)(-0.5, -0.5, -0.5), (ctypes.c_float * 3)(0.1, 0.1, 0.1),
                     (ctypes.c_int32 * 3)(10, 10, 10))
    vm = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1, model=1)
    assert lib.fgs_voxelize_fwd(ctypes.byref(g), ctypes.byref(gr1), ctypes.byref(vm), 16, ctypes.byref(ws),
                                None) == A.FGS_E_INVALID
    # zero Gaussians
    g0 = A.fgs_gaussians(0, 16, 16, 16, 16)
    gr = A.fgs_grid((ctypes.c_float * 3)(-0.5, -0.5, -0.5), (ctypes.c_float * 3)(0.1, 0.1, 0.1),
                    (ctypes.c_int32 * 3)(10, 10, 10))
    assert lib.fgs_voxelize_fwd(ctypes.byref(g0), ctypes.byref(gr), ctypes.byref(o), 16, ctypes.byref(ws),
                                None) == A.FGS_E_INVALID
    # non-positive grid
    gr2 = A.fgs_grid((ctypes.c_float * 3)(0, 0, 0), (ctypes.c_float * 3)(0.1, 0.0, 0.1),
                     (ctypes.c_int32 * 3)(10, 10, 10))
    assert lib.fgs_voxelize_fwd(ctypes.byref(g), ctypes.byref(gr2), ctypes.byref(o), 16, ctypes.byref(ws),
                                None) == A.FGS_E_INVALID
    # a workspace that holds no lists
    off = (ctypes.c_uint64 * 9)()
    cnt = (ctypes.c_uint64 * 3)()
    assert lib.fgs_binning_layout(ctypes.byref(ws), off, cnt) == A.FGS_E_INVALID
    # backward without recompute needs the forward's lists
    o0 = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=0)
    gg = A.fgs_gaussian_grads(16, 16, 16, 16)
    assert lib.fgs_project_views_bwd(ctypes.byref(g), ctypes.byref(gm), 0, 1, ctypes.byref(o0), 16,
                                     ctypes.byref(gg), ctypes.byref(ws), None) == A.FGS_E_INVALID


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2604_01844_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


def test_workspace_query_is_host_arithmetic():
    """fgs_workspace_query runs without a GPU: the per-pair bytes match the
    layout (at 512^2 with 75 views the tile field and the record index fit
    one 32-bit word: 2 uint32 arrays for the words and their sort copy, a
    32-byte pair slot, about one byte of sort histogram and the work-unit
    table: 41 for the splat; with key and value arrays, 49;
    64-byte slots for the ray-exact model; the voxelizer adds the gid array
    and 40-byte slots), and the fixed part grows with the records."""
    from paper_2604_01844_amd import _abi as A
    lib = A.lib()
    fixed, per = ctypes.c_uint64(), ctypes.c_uint64()
    g = A.fgs_gaussians(50000, None, None, None, None)
    gm = A.fgs_geom(A.FGS_CONE, 75, 16, 1.5, 2.0, 512, 512, 0.0055, 0.0055, 0.0, 0.0)
    o = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1)
    q = lambda op, gptr, geom, grid, vc, opts: lib.fgs_workspace_query(op, gptr, geom, grid, vc, opts,
                                                                        ctypes.byref(fixed), ctypes.byref(per))
    assert q(A.FGS_OP_PROJECT_BWD, ctypes.byref(g), ctypes.byref(gm), None, 75, ctypes.byref(o)) == A.FGS_OK
    assert 41 <= per.value <= 42
    fixed75 = fixed.value
    assert fixed75 > 75 * 50000 * 100
    assert q(A.FGS_OP_PROJECT_BWD, ctypes.byref(g), ctypes.byref(gm), None, 1, ctypes.byref(o)) == A.FGS_OK
    assert fixed.value < fixed75 / 50
    oe = A.fgs_opts(kappa=3.0, near_plane=1e-2, recompute=1, model=A.FGS_MODEL_RAY_EXACT)
    assert q(A.FGS_OP_PROJECT_FWD, ctypes.byref(g), ctypes.byref(gm), None, 75, ctypes.byref(oe)) == A.FGS_OK
    assert 73 <= per.value <= 74
    # 2048^2 views (14-bit tile field) of 500,000 Gaussians: key/value lists
    g5 = A.fgs_gaussians(500000, None, None, None, None)
    gm2 = A.fgs_geom(A.FGS_CONE, 50, 16, 1.5, 2.0, 2048, 2048, 0.0014, 0.0014, 0.0, 0.0)
    assert q(A.FGS_OP_PROJECT_FWD, ctypes.byref(g5), ctypes.byref(gm2), None, 10, ctypes.byref(o)) == A.FGS_OK
    assert 49 <= per.value <= 50
    gr = A.fgs_grid((ctypes.c_float * 3)(-0.5, -0.5, -0.5), (ctypes.c_float * 3)(1 / 256, 1 / 256, 1 / 256),
                    (ctypes.c_int32 * 3)(256, 256, 256))
    assert q(A.FGS_OP_VOXELIZE_FWD, ctypes.byref(g), None, ctypes.byref(gr), 0, ctypes.byref(o)) == A.FGS_OK
    assert 61 <= per.value <= 62
    assert q(7, ctypes.byref(g), None, ctypes.byref(gr), 0, ctypes.byref(o)) == A.FGS_E_INVALID
    assert q(A.FGS_OP_PROJECT_FWD, ctypes.byref(g), ctypes.byref(gm), None, 76, ctypes.byref(o)) == A.FGS_E_INVALID
