"""FP64 CPU oracle for the Gaussian X-ray rasterizer and voxelizer.

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers. The product path (the
HIP library and its Python binding) never imports this package, and this
package never imports the product: the two share nothing but the seeded
input generators in ``synth_inputs``.

The numerical core is ``oracle.c`` (plain double-precision C, built with
gcc into ``liboracle.so``); this module wraps it with ctypes and adds the
pieces that are clearer in NumPy: Gauss-Legendre quadrature of the ray
integral (Eq. 3), the integer tile-binning reference, the L1 loss and its
gradient (Eq. 5), Adam, PSNR and finite differences.

Parity status of each function (what pins it in ``tests/test_oracle_pins.py``):

* ``project`` / ``project_points`` (Eq. 4, method splat M): pinned by
  parallel-beam equality with the exact line integral and quadrature, by the
  mu identity at the splat centre in cone beam, by the small-Gaussian limit
  M -> E, by the 2D splat-mass closed form and by brute force.
* ``exact_points`` (Eq. 3): pinned by quadrature.
* ``exact_project`` / ``exact_points_cut`` (the ray-exact model: Eq. 3 with
  the kappa support): pinned by the isotropic closed form with its cutoff,
  quadrature at large kappa, brute force over every pixel, and equality with
  the splat in parallel beam (where the two models coincide).
* ``exact_bwd``: pinned by Richardson finite differences at kappa = 8 and,
  at kappa = 3, by finite differences of the uncut integrals over the
  unperturbed support.
* ``voxelize`` (Eq. 2, Sec. 3.3): pinned by the 3D mass closed form and
  brute force.
* ``project_banded`` / ``voxelize_banded``: their first output is
  ``project`` / ``voxelize`` (checked for equality); the band sum is pinned
  by brute force on a small scene.
* ``project_bwd`` / ``voxelize_bwd``: pinned by Richardson finite
  differences of the forward functions.
* ``phantom_project`` / ``phantom_volume``: pinned by the sphere chord and
  by quadrature of the indicator.
* ``bin_tiles``: pinned by the superset property against FP64 support pairs.
* ``tiles.quad_min`` (the exact smallest Mahalanobis distance over a box),
  ``tiles.vox_bin_tiles`` (voxel-tile binning) and
  ``tiles.vox_support_tiles``: pinned by dense sampling, SciPy's bounded
  minimiser, the isotropic closed form, a hand-computed binning and the
  superset property (tests/test_culling_cpu.py).
* ``l1_loss_grad``, ``adam_step``, ``psnr``: pinned by hand-computed values.
* ``initialisation.fdk`` (FDK, Sec. 3.1): pinned by the reconstruction of
  uniform spheres and ellipsoids from their exact projections.
* ``initialisation.gradient_init`` (both weightings, gradient and the
  intensity baseline): pinned by hand-computed weights and draws, sampling
  frequencies against the exact multinomial law, trilinear exactness on
  linear fields and brute-force nearest neighbours.
* ``tv_loss_grad``: pinned by a hand-computed volume, finite differences
  and the invariances of a total variation.
* ``ssim_loss_grad``, ``ssim3d_loss_grad``: pinned by SSIM(x, x) = 1, a
  brute-force windowed sum at every pixel (voxel) of a small case, and
  finite differences of the loss.
* ``mlp`` (learned initializer): BF16 rounding pinned against torch's
  bfloat16 conversion, the backward against finite differences of the
  unrounded network, the canonical targets against their defining
  invariances.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KAPPA = 3.0


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2, no fast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (0: all host cores); returns the
    count now in force. Timing control only."""
    lib = _load()
    lib.orc_set_threads(ctypes.c_int(int(n)))
    return int(lib.orc_max_threads())


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _geom_vec(geom: dict) -> np.ndarray:
    return np.array([1.0 if geom["mode"] == "parallel" else 0.0, geom["sod"], geom["sdd"],
                     geom["det_w"], geom["det_h"], geom["pitch_u"], geom["pitch_v"],
                     geom["off_u"], geom["off_v"], geom["near"]], dtype=np.float64)


def _grid_vec(grid: dict) -> np.ndarray:
    return np.array(list(grid["origin"]) + list(grid["spacing"]) + list(grid["dims"]),
                    dtype=np.float64)


def _gauss_args(gs: dict):
    n = gs["density"].shape[0]
    keep = []
    ptrs = []
    for k in ("mean", "log_scale", "quat", "density"):
        a, p = _d(gs[k])
        keep.append(a)
        ptrs.append(p)
    return n, keep, ptrs


# ---------------------------------------------------------------- Eq. 4 (M)

def splat_records(gs: dict, geom: dict, angles) -> dict:
    """Per-(view, Gaussian) splat quantities, record r = v * n + i."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    V = ang.shape[0]
    R = V * n
    uv = np.zeros(2 * R); sh = np.zeros(3 * R); co = np.zeros(3 * R)
    mu = np.zeros(R); w = np.zeros(R); cul = np.zeros(R, dtype=np.int32)
    g, pg = _d(_geom_vec(geom))
    lib.orc_splat_records(pg, ctypes.c_int(V), pa, ctypes.c_long(n), *p,
                          _ptr(uv),
                          _ptr(sh), _ptr(co), _ptr(mu), _ptr(w),
                          cul.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return dict(uv=uv.reshape(R, 2), shat=sh.reshape(R, 3), conic=co.reshape(R, 3), mu=mu, w=w,
                culled=cul.astype(bool))


def project(gs: dict, geom: dict, angles, kappa: float = KAPPA, brute: bool = False, tau: float = 0.0) -> np.ndarray:
    """Method projection M for every pixel of every view: [V][H][W] float64.
    tau > 0: the density-aware support d^2 <= min(kappa^2, 2 ln(w / tau))
    (Sec. 3.5 boxes that take the density into account; w = rho mu the splat's peak)."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    V = ang.shape[0]
    img = np.zeros((V, geom["det_h"], geom["det_w"]))
    g, pg = _d(_geom_vec(geom))
    fn = lib.orc_project_brute if brute else lib.orc_project
    fn(pg, ctypes.c_double(kappa), ctypes.c_double(tau), ctypes.c_int(V), pa, ctypes.c_long(n), *p,
       img.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return img


def project_points(gs: dict, geom: dict, angle: float, u, v, kappa: float = KAPPA, tau: float = 0.0) -> np.ndarray:
    """M of one view at arbitrary detector points (pixel coordinates)."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    uu, pu = _d(u); vv, pv = _d(v)
    out = np.zeros(uu.shape[0])
    g, pg = _d(_geom_vec(geom))
    lib.orc_project_points(pg, ctypes.c_double(kappa), ctypes.c_double(tau), ctypes.c_double(angle),
                           ctypes.c_long(n), *p,
                           ctypes.c_long(uu.shape[0]), pu, pv,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


# ---------------------------------------------------------------- Eq. 3 (E)

def exact_points(gs: dict, geom: dict, angle: float, u, v) -> np.ndarray:
    """Exact line integral of the Gaussian field (no cutoff) along the ray
    through each detector point."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    uu, pu = _d(u); vv, pv = _d(v)
    out = np.zeros(uu.shape[0])
    g, pg = _d(_geom_vec(geom))
    lib.orc_exact_points(pg, ctypes.c_double(angle), ctypes.c_long(n), *p, ctypes.c_long(uu.shape[0]),
                         pu, pv, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


# ---------------------------------------------------------------- ray-exact model (Eq. 3, kappa support)

def exact_project(gs: dict, geom: dict, angles, kappa: float = KAPPA, brute: bool = False) -> np.ndarray:
    """Ray-exact model for every pixel of every view: each Gaussian adds its
    exact line integral (Eq. 3) to the rays that pass within Mahalanobis
    distance kappa of its mean. [V][H][W] float64."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    V = ang.shape[0]
    img = np.zeros((V, geom["det_h"], geom["det_w"]))
    g, pg = _d(_geom_vec(geom))
    lib.orc_exact_project(pg, ctypes.c_double(kappa), ctypes.c_int(V), pa, ctypes.c_long(n), *p,
                          ctypes.c_int(1 if brute else 0), _ptr(img))
    return img


def exact_points_cut(gs: dict, geom: dict, angle: float, u, v, kappa: float = KAPPA) -> np.ndarray:
    """The ray-exact model of one view at arbitrary detector points."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    uu, pu = _d(u); vv, pv = _d(v)
    out = np.zeros(uu.shape[0])
    g, pg = _d(_geom_vec(geom))
    lib.orc_exact_points_cut(pg, ctypes.c_double(kappa), ctypes.c_double(angle), ctypes.c_long(n), *p,
                             ctypes.c_long(uu.shape[0]), pu, pv, _ptr(out))
    return out


def exact_bwd(gs: dict, geom: dict, angles, grad_img, kappa: float = KAPPA, sel=None,
              band: float = 0.0) -> dict:
    """Gradient of sum(grad_img * E_kappa) (the ray-exact model), support held
    fixed; ``band`` as in project_bwd, on the ray's squared Mahalanobis
    distance to the mean."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    gi, pgi = _d(grad_img)
    sel = np.arange(n, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    dm, dl, dq, dr = _bwd_out(sel.shape[0])
    babs = np.zeros((11, sel.shape[0]))
    g, pg = _d(_geom_vec(geom))
    lib.orc_exact_bwd(pg, ctypes.c_double(kappa), ctypes.c_int(ang.shape[0]), pa, ctypes.c_long(n), *p,
                      pgi, ctypes.c_long(sel.shape[0]), sel.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                      _ptr(dm), _ptr(dl), _ptr(dq), _ptr(dr), ctypes.c_double(band), _ptr(babs))
    out = dict(mean=dm, log_scale=dl, quat=dq, density=dr)
    if band > 0:
        out["band_abs"] = _split11(babs)
    return out


def rays(geom: dict, angle: float, u, v):
    """Origin and unit direction of the ray through each detector point."""
    lib = _load()
    uu, pu = _d(u); vv, pv = _d(v)
    m = uu.shape[0]
    o = np.zeros(3 * m); d = np.zeros(3 * m)
    g, pg = _d(_geom_vec(geom))
    lib.orc_rays(pg, ctypes.c_double(angle), ctypes.c_long(m), pu, pv,
                 o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return o.reshape(m, 3), d.reshape(m, 3)


def field_points(gs: dict, x, kappa: float = float("inf"), tau: float = 0.0) -> np.ndarray:
    """Density field sigma(x) (Eq. 2) at points x[m][3]; kappa=inf: no cutoff;
    tau > 0: also d^2 <= 2 ln(rho / tau) (see project)."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    xx, px = _d(np.asarray(x).reshape(-1, 3))
    out = np.zeros(xx.shape[0])
    lib.orc_field_points(ctypes.c_double(kappa), ctypes.c_double(tau), ctypes.c_long(n), *p, ctypes.c_long(xx.shape[0]), px,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def quadrature_points(gs: dict, geom: dict, angle: float, u, v, t_lo: float, t_hi: float,
                      order: int = 400, panels: int = 8) -> np.ndarray:
    """Composite Gauss-Legendre quadrature of Eq. 3 along each ray over the
    ray parameter interval [t_lo, t_hi] (no cutoff)."""
    o, d = rays(geom, angle, u, v)
    xg, wg = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(t_lo, t_hi, panels + 1)
    ts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        ts.append(0.5 * (b - a) * xg + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wg)
    ts = np.concatenate(ts); ws = np.concatenate(ws)
    out = np.zeros(o.shape[0])
    for k in range(o.shape[0]):
        pts = o[k][None, :] + ts[:, None] * d[k][None, :]
        out[k] = np.dot(ws, field_points(gs, pts))
    return out


def project_banded(gs: dict, geom: dict, angles, band: float = 1e-3, kappa: float = KAPPA, tau: float = 0.0):
    """(img, band_img): project() and, per pixel, the sum of the contributions
    of the pairs with |d^2 - kappa^2| <= band (inside or just outside the
    support). An evaluation whose support decisions differ from FP64 only on
    such pairs stays within band_img of img, pixel by pixel."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    img = np.zeros((ang.shape[0], geom["det_h"], geom["det_w"]))
    bimg = np.zeros_like(img)
    g, pg = _d(_geom_vec(geom))
    lib.orc_project_banded(pg, ctypes.c_double(kappa), ctypes.c_double(tau), ctypes.c_int(ang.shape[0]), pa,
                           ctypes.c_long(n), *p,
                           ctypes.c_double(band), _ptr(img), _ptr(bimg))
    return img, bimg


# ---------------------------------------------------------------- voxelizer

def voxelize(gs: dict, grid: dict, kappa: float = KAPPA, brute: bool = False, tau: float = 0.0) -> np.ndarray:
    """Density sum at voxel centres: [nz][ny][nx] float64; tau as in project
    with the peak rho."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    nx, ny, nz = grid["dims"]
    vol = np.zeros((nz, ny, nx))
    gr, pgr = _d(_grid_vec(grid))
    fn = lib.orc_voxelize_brute if brute else lib.orc_voxelize
    fn(ctypes.c_double(kappa), ctypes.c_double(tau), pgr, ctypes.c_long(n), *p,
       vol.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return vol


def voxelize_banded(gs: dict, grid: dict, band: float = 1e-3, kappa: float = KAPPA, tau: float = 0.0):
    """(vol, band_vol) as project_banded, for the voxelizer."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    nx, ny, nz = grid["dims"]
    vol = np.zeros((nz, ny, nx))
    bvol = np.zeros_like(vol)
    gr, pgr = _d(_grid_vec(grid))
    lib.orc_voxelize_banded(ctypes.c_double(kappa), ctypes.c_double(tau), pgr, ctypes.c_long(n), *p,
                            ctypes.c_double(band), _ptr(vol),
                            _ptr(bvol))
    return vol, bvol


# ---------------------------------------------------------------- gradients

def _bwd_out(n_sel):
    return (np.zeros((3, n_sel)), np.zeros((3, n_sel)), np.zeros((4, n_sel)), np.zeros(n_sel))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _split11(a):
    return dict(mean=a[0:3], log_scale=a[3:6], quat=a[6:10], density=a[10])


def project_bwd(gs: dict, geom: dict, angles, grad_img, kappa: float = KAPPA, sel=None,
                band: float = 0.0, tau: float = 0.0) -> dict:
    """Gradient of sum(grad_img * M) w.r.t. mean, log_scale, quat, density of
    the Gaussians in ``sel`` (default all), support held fixed.

    With band > 0, (pixel, Gaussian) pairs with |d^2 - kappa^2| <= band are
    left out and ``result["band_abs"]`` holds, per parameter, the sum of the
    absolute per-pair gradients over them: the boundary pairs whose inclusion
    no finite-precision evaluation decides uniquely."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    ang, pa = _d(angles)
    gi, pgi = _d(grad_img)
    sel = np.arange(n, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    dm, dl, dq, dr = _bwd_out(sel.shape[0])
    babs = np.zeros((11, sel.shape[0]))
    g, pg = _d(_geom_vec(geom))
    lib.orc_project_bwd(pg, ctypes.c_double(kappa), ctypes.c_double(tau), ctypes.c_int(ang.shape[0]), pa,
                        ctypes.c_long(n), *p,
                        pgi, ctypes.c_long(sel.shape[0]), sel.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                        _ptr(dm), _ptr(dl), _ptr(dq), _ptr(dr), ctypes.c_double(band), _ptr(babs))
    out = dict(mean=dm, log_scale=dl, quat=dq, density=dr)
    if band > 0:
        out["band_abs"] = _split11(babs)
    return out


def voxelize_bwd(gs: dict, grid: dict, grad_vol, kappa: float = KAPPA, sel=None, band: float = 0.0,
                 tau: float = 0.0) -> dict:
    """Gradient of sum(grad_vol * V); ``band`` as in project_bwd."""
    lib = _load()
    n, keep, p = _gauss_args(gs)
    gv, pgv = _d(grad_vol)
    gr, pgr = _d(_grid_vec(grid))
    sel = np.arange(n, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    dm, dl, dq, dr = _bwd_out(sel.shape[0])
    babs = np.zeros((11, sel.shape[0]))
    lib.orc_voxelize_bwd(ctypes.c_double(kappa), ctypes.c_double(tau), pgr, ctypes.c_long(n), *p, pgv, ctypes.c_long(sel.shape[0]),
                         sel.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                         _ptr(dm), _ptr(dl), _ptr(dq), _ptr(dr), ctypes.c_double(band), _ptr(babs))
    out = dict(mean=dm, log_scale=dl, quat=dq, density=dr)
    if band > 0:
        out["band_abs"] = _split11(babs)
    return out


def banded_grad_error(got: dict, ref: dict) -> dict:
    """Per parameter group: relative L2 of the part of |got - ref| that the
    boundary band (ref["band_abs"]) cannot explain."""
    out = {}
    for k in ("mean", "log_scale", "quat", "density"):
        g = np.asarray(got[k], dtype=np.float64)
        r = ref[k]
        excess = np.maximum(np.abs(g - r) - ref["band_abs"][k], 0.0)
        out[k] = float(np.linalg.norm(excess.ravel()) / np.linalg.norm(r.ravel()))
    return out


# ---------------------------------------------------------------- phantom

def _phantom_args(ph: dict):
    keep = [np.ascontiguousarray(ph[k], dtype=np.float64) for k in ("centre", "semi", "quat", "amp")]
    return keep, [_ptr(a) for a in keep]


def phantom_volume(ph: dict, grid: dict) -> np.ndarray:
    lib = _load()
    keep, p = _phantom_args(ph)
    nx, ny, nz = grid["dims"]
    vol = np.zeros((nz, ny, nx))
    gr, pgr = _d(_grid_vec(grid))
    lib.orc_phantom_volume(ctypes.c_long(ph["amp"].shape[0]), *p, pgr, _ptr(vol))
    return vol


def phantom_project(ph: dict, geom: dict, angles) -> np.ndarray:
    lib = _load()
    keep, p = _phantom_args(ph)
    ang, pa = _d(angles)
    img = np.zeros((ang.shape[0], geom["det_h"], geom["det_w"]))
    g, pg = _d(_geom_vec(geom))
    lib.orc_phantom_project(pg, ctypes.c_int(ang.shape[0]), pa, ctypes.c_long(ph["amp"].shape[0]), *p,
                            _ptr(img))
    return img


# ---------------------------------------------------------------- binning

def bin_tiles(uv32, r32, det_w: int, det_h: int, tile: int = 16, cull=None, n_views: int = 1):
    """Integer tile binning from FP32 splat centres and support half-extents.

    uv32[R][2], r32[R][2] are float32 (centre and kappa-scaled half-extents in
    pixels). A record covers the tiles whose pixel-centre columns lie in
    [floor(u - ru - 1/2), floor(u + ru - 1/2)] (and likewise for rows),
    clipped to the image; all arithmetic is float32 subtraction followed by
    floor, the same decision the GPU takes. Records are r = v * n + i.
    Returns dict with rect[R][4] (tx0, ty0, tx1, ty1; empty when tx0 > tx1),
    count[R], offset[R+1], keys (view * tiles_per_view + tile id, emitted in
    record order, row-major inside each rect), vals (record index), the
    stably sorted keys/vals and the per-tile start array.
    """
    uv32 = np.asarray(uv32, dtype=np.float32)
    r32 = np.asarray(r32, dtype=np.float32)
    R = uv32.shape[0]
    n = R // n_views
    tx_n = (det_w + tile - 1) // tile
    ty_n = (det_h + tile - 1) // tile
    half = np.float32(0.5)
    lim = np.float32(1 << 24)

    def span(c, r, n_tiles):
        lo = np.floor(np.clip((c - r) - half, -lim, lim)).astype(np.int64)
        hi = np.floor(np.clip((c + r) - half, -lim, lim)).astype(np.int64)
        t0 = np.maximum(np.floor_divide(lo, tile), 0)
        t1 = np.minimum(np.floor_divide(hi, tile), n_tiles - 1)
        return t0, t1

    tx0, tx1 = span(uv32[:, 0], r32[:, 0], tx_n)
    ty0, ty1 = span(uv32[:, 1], r32[:, 1], ty_n)
    empty = (tx0 > tx1) | (ty0 > ty1)
    if cull is not None:
        empty |= np.asarray(cull, dtype=bool)
    count = np.where(empty, 0, (tx1 - tx0 + 1) * (ty1 - ty0 + 1)).astype(np.int64)
    offset = np.zeros(R + 1, dtype=np.int64)
    np.cumsum(count, out=offset[1:])
    keys = np.empty(offset[-1], dtype=np.int64)
    vals = np.empty(offset[-1], dtype=np.int64)
    tpv = tx_n * ty_n
    for r in np.nonzero(count)[0]:
        v = r // n
        ys, xs = np.meshgrid(np.arange(ty0[r], ty1[r] + 1), np.arange(tx0[r], tx1[r] + 1), indexing="ij")
        k = v * tpv + (ys * tx_n + xs).ravel()
        keys[offset[r]:offset[r + 1]] = k
        vals[offset[r]:offset[r + 1]] = r
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    svals = vals[order]
    start = np.searchsorted(skeys, np.arange(n_views * tpv + 1), side="left")
    rect = np.stack([tx0, ty0, tx1, ty1], axis=1)
    return dict(rect=rect, count=count, offset=offset, keys=keys, vals=vals, sorted_keys=skeys,
                sorted_vals=svals, tile_start=start, tiles_x=tx_n, tiles_y=ty_n)


# ---------------------------------------------------------------- losses

def l1_loss_grad(img, gt):
    """Eq. 5's L1 term: mean |I - I_gt| over the pixels of each view, summed
    over views; gradient sign(I - I_gt) / P with sign(0) = 0."""
    img = np.asarray(img, dtype=np.float64)
    gt = np.asarray(gt, dtype=np.float64)
    P = img[0].size if img.ndim >= 3 else img.size
    diff = img - gt
    loss = np.abs(diff).sum() / P
    return loss, np.sign(diff) / P


def adam_step(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update (Kingma and Ba, Algorithm 1) with bias correction."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def tv_loss_grad(vol32, scale: float = 1.0):
    """3D total variation (the TV term of Eq. 5): scale/n times the sum over
    voxels and axes of |V(i + e_a) - V(i)| (forward differences inside the
    grid, n = voxel count), and its gradient. The differences and their signs
    are taken in FP32 (the input's precision), the sums in FP64."""
    v = np.asarray(vol32, dtype=np.float32)
    n = v.size
    loss = 0.0
    grad = np.zeros(v.shape)
    for axis in range(3):
        d = np.diff(v, axis=axis)             # FP32 forward differences
        loss += np.abs(d.astype(np.float64)).sum()
        sg = np.sign(d).astype(np.float64)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        grad[tuple(lo)] -= sg                 # V(i) enters d(i) with sign -1
        grad[tuple(hi)] += sg                 # V(i + e_a) enters d(i) with sign +1
    return scale * loss / n, grad * (scale / n)


def ssim_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """Normalised 1D Gaussian window of the SSIM index (the 2D window is its
    outer product)."""
    k = np.arange(size) - (size - 1) / 2
    w = np.exp(-k * k / (2 * sigma * sigma))
    return w / w.sum()


def ssim_loss_grad(img, gt, scale: float = 1.0, c1: float = 1e-4, c2: float = 9e-4, size: int = 11,
                   sigma: float = 1.5):
    """SSIM term of Eq. 5: scale * (1 - mean SSIM(img, gt)) over all views and
    pixels, SSIM(p) = (2 mx my + c1)(2 sxy + c2) / ((mx^2 + my^2 + c1)(sx^2 +
    sy^2 + c2)) with local statistics under a Gaussian window (zero outside
    the image), and its gradient with respect to img. img, gt [V][H][W]."""
    from scipy.ndimage import correlate
    x = np.asarray(img, dtype=np.float64)
    y = np.asarray(gt, dtype=np.float64)
    w1 = ssim_window(size, sigma)
    w2 = np.outer(w1, w1)[None]
    conv = lambda a: correlate(a, w2, mode="constant", cval=0.0)
    mx, my = conv(x), conv(y)
    exx, eyy, exy = conv(x * x), conv(y * y), conv(x * y)
    A = 2 * mx * my + c1
    B = 2 * (exy - mx * my) + c2
    C = mx * mx + my * my + c1
    D = (exx - mx * mx) + (eyy - my * my) + c2
    S = A * B / (C * D)
    n = x.size
    loss = scale * (1.0 - S.mean())
    # dS/d(mx, exx, exy) with the other local statistics fixed
    g_mx = (2 * my * B - 2 * my * A) / (C * D) - S * (2 * mx / C - 2 * mx / D)
    g_exx = -S / D
    g_exy = 2 * A / (C * D)
    # the window is symmetric: the adjoint of the correlation is itself
    grad = -(scale / n) * (conv(g_mx) + 2 * x * conv(g_exx) + y * conv(g_exy))
    return loss, grad


def ssim3d_loss_grad(vol, gt, scale: float = 1.0, c1: float = 1e-4, c2: float = 9e-4, size: int = 11,
                     sigma: float = 1.5):
    """The 3D SSIM term of Eq. 6: scale * (1 - mean SSIM) over the voxels of
    vol, gt [nz][ny][nx], with local statistics under the separable 3D
    Gaussian window (zero outside the grid), and its gradient with respect
    to vol. Same per-voxel formula as ssim_loss_grad."""
    from scipy.ndimage import correlate
    x = np.asarray(vol, dtype=np.float64)
    y = np.asarray(gt, dtype=np.float64)
    w1 = ssim_window(size, sigma)
    w3 = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    conv = lambda a: correlate(a, w3, mode="constant", cval=0.0)
    mx, my = conv(x), conv(y)
    exx, eyy, exy = conv(x * x), conv(y * y), conv(x * y)
    A = 2 * mx * my + c1
    B = 2 * (exy - mx * my) + c2
    C = mx * mx + my * my + c1
    D = (exx - mx * mx) + (eyy - my * my) + c2
    S = A * B / (C * D)
    loss = scale * (1.0 - S.mean())
    g_mx = (2 * my * B - 2 * my * A) / (C * D) - S * (2 * mx / C - 2 * mx / D)
    grad = -(scale / x.size) * (conv(g_mx) + 2 * x * conv(-S / D) + y * conv(2 * A / (C * D)))
    return loss, grad


def psnr(vol, gt):
    """10 log10(max(gt)^2 / MSE) over the whole grid."""
    vol = np.asarray(vol, dtype=np.float64)
    gt = np.asarray(gt, dtype=np.float64)
    mse = np.mean((vol - gt) ** 2)
    return 10.0 * np.log10(gt.max() ** 2 / mse)


from .initialisation import fdk, gradient_init, sampling_weights, trilinear  # noqa: E402,F401
from . import mlp  # noqa: E402,F401
from . import tiles  # noqa: E402,F401


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
