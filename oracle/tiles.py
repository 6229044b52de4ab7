"""Voxel-tile binning reference (FP64 NumPy) and the exact box test it uses.

TEST INFRASTRUCTURE ONLY: called by the test suite; the product path never
imports it, and it imports nothing from the product.

The voxelizer limits each Gaussian to its kappa-sigma ellipsoid (Sec. 3.3)
and bins Gaussians into 3D tiles by their position and radius (Sec. 3.5), as
the rasterizer does on the detector. The binning written out here:

* a Gaussian's centre in voxel-index coordinates is (p - origin) / h - 1/2
  (voxel (i, j, k) has its centre at index coordinates (i, j, k)); its
  half-extents are kappa sqrt(Sigma_aa) / h_a, the exact box of the
  ellipsoid;
* its tile rectangle spans tiles floor(floor(c - r) / 8) to
  floor(floor(c + r) / 8) per axis, clipped to the grid's tiles;
* of those, a tile is listed iff the support ellipsoid, widened to
  d^2 <= kappa^2 * slack (slack 1.001, a Mahalanobis radius 0.05% larger),
  reaches a point of the tile's voxel-centre box [8t, 8t + 7]^3: the
  smallest d^2 over the box, an exact convex minimisation (quad_min);
* with the density-aware support (tau > 0; Sec. 3.5 boxes that take the density
  into account) Gaussian i keeps d^2 <= k2_i = min(kappa^2, 2 ln(rho_i / tau))
  and is dropped when rho_i <= tau: its half-extents are sqrt(k2_i)
  sqrt(Sigma_aa) / h_a and its tile test d^2 <= k2_i + kappa^2 (slack - 1)
  (the same widening as at the kappa support);
* keys are tile ids (tz * nty + ty) * ntx + tx, emitted Gaussian by
  Gaussian in row-major order inside the rectangle (x fastest); a stable
  sort by key leaves each tile's list in ascending Gaussian index.

``vox_support_tiles`` gives, independently of the box test, the tiles that
hold a voxel centre of each Gaussian's support (brute force over the voxels
of its box); any correct binning lists a superset of them.

Pins (tests/test_culling_cpu.py): quad_min against dense sampling of the
box, SciPy's bounded minimiser and the isotropic closed form (squared
distance to the box); vox_bin_tiles against a hand-computed case and against
vox_support_tiles (superset).
"""
from __future__ import annotations

import itertools

import numpy as np


def covariances(gs: dict) -> np.ndarray:
    """Sigma[n][3][3] = R(q / |q|) diag(exp(2 log_scale)) R^T (Eq. 1), FP64."""
    q = np.asarray(gs["quat"], dtype=np.float64)
    w, x, y, z = q / np.linalg.norm(q, axis=0)
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    R = np.moveaxis(R, -1, 0)                                   # [n][3][3]
    s2 = np.exp(2.0 * np.asarray(gs["log_scale"], dtype=np.float64)).T   # [n][3]
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


def quad_min(A, lo, hi) -> np.ndarray:
    """Exact min of d^T A d over the box lo <= d <= hi, for symmetric
    positive definite A[..., k, k] and boxes lo, hi [..., k] (k = 2 or 3).

    Every face of the box (each coordinate fixed at its lower bound, at its
    upper bound, or free: 3^k faces, the vertices and the interior included)
    is tried: with the free coordinates F and the fixed ones C, the
    minimiser of the form on the face's affine hull is
    d_F = -A_FF^{-1} A_FC d_C. Those that lie inside the box are candidates,
    and the smallest candidate value is the minimum: the box minimiser lies in
    the relative interior of some face, where it is that face's minimiser
    (A is positive definite, so each face's minimiser is unique)."""
    A = np.asarray(A, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    k = A.shape[-1]
    best = np.full(lo.shape[:-1], np.inf)
    for choice in itertools.product((0, 1, 2), repeat=k):      # 0 lower, 1 upper, 2 free
        free = [a for a in range(k) if choice[a] == 2]
        fixed = [a for a in range(k) if choice[a] != 2]
        d = np.zeros(lo.shape)
        for a in fixed:
            d[..., a] = lo[..., a] if choice[a] == 0 else hi[..., a]
        ok = np.ones(lo.shape[:-1], dtype=bool)
        if free:
            AFF = A[..., free, :][..., :, free]
            rhs = np.zeros(lo.shape[:-1] + (len(free),))
            for a in fixed:
                rhs -= A[..., free, a] * d[..., a:a + 1]
            dF = np.linalg.solve(AFF, rhs[..., None])[..., 0]
            for j, a in enumerate(free):
                d[..., a] = dF[..., j]
                ok &= (dF[..., j] >= lo[..., a]) & (dF[..., j] <= hi[..., a])
        val = np.einsum("...i,...ij,...j->...", d, A, d)
        best = np.where(ok, np.minimum(best, val), best)
    return best


def support_k2(kappa: float, tau: float, peak) -> np.ndarray:
    """Per Gaussian, the bound on d^2 of its support: kappa^2, or with the
    density-aware support (tau > 0) min(kappa^2, 2 ln(peak / tau)); -1 where
    peak <= tau (the Gaussian contributes nothing)."""
    peak = np.asarray(peak, dtype=np.float64)
    k2 = np.full(peak.shape, kappa * kappa)
    if tau > 0:
        with np.errstate(divide="ignore", invalid="ignore"):
            k2 = np.where(peak > tau, np.minimum(k2, 2.0 * np.log(peak / tau)), -1.0)
    return k2


def _voxel_frame(gs: dict, grid: dict, kappa: float, tau: float = 0.0):
    """Centres in voxel-index coordinates [n][3], half-extents in voxels
    [n][3], inverse covariances in voxel-index units [n][3][3], and the
    per-Gaussian support bound on d^2 [n] (support_k2)."""
    h = np.asarray(grid["spacing"], dtype=np.float64)
    o = np.asarray(grid["origin"], dtype=np.float64)
    p = np.asarray(gs["mean"], dtype=np.float64).T
    c = (p - o) / h - 0.5
    S = covariances(gs) / (h[:, None] * h[None, :])
    k2 = support_k2(kappa, tau, np.asarray(gs["density"], dtype=np.float64))
    r = np.sqrt(np.maximum(k2, 0.0))[:, None] * np.sqrt(np.diagonal(S, axis1=1, axis2=2))
    return c, r, np.linalg.inv(S), k2


def vox_bin_tiles(gs: dict, grid: dict, kappa: float = 3.0, tile: int = 8, slack: float = 1.001,
                  band_edge: float = 1e-3, band_cull: float = 1e-4, tau: float = 0.0,
                  band_tau: float = 1e-5) -> dict:
    """The voxel-tile lists of the module docstring.

    Returns rect[n][6] (tx0, ty0, tz0, tx1, ty1, tz1; all -1 when empty),
    count[n], offset[n + 1], emit_keys / emit_gauss (emission order),
    sorted_keys / sorted_gauss / sorted_slots (stable sort by key; a slot is
    a position in the emission order), tile_start[T + 1] and tiles
    (ntx, nty, ntz). ``ambiguous[n]`` flags Gaussians with a decision near
    its threshold, where FP32 evaluation may decide either way: a box edge
    within band_edge voxels of a tile boundary, or a tile whose smallest d^2
    is within band_cull * kappa^2 * slack of kappa^2 * slack. Both bands are
    many times the FP32 rounding of those quantities at the sizes here
    (coordinates below 2^12 voxels, forms of a few hundred). With tau > 0 a
    Gaussian whose density is within a relative band_tau of tau is
    ambiguous too (FP32 decides whether it is dropped)."""
    dims = np.asarray(grid["dims"], dtype=np.int64)
    nt = (dims + tile - 1) // tile
    c, r, A, k2 = _voxel_frame(gs, grid, kappa, tau)
    n = c.shape[0]
    lo_e, hi_e = c - r, c + r
    t0 = np.maximum(np.floor_divide(np.floor(lo_e), tile), 0).astype(np.int64)
    t1 = np.minimum(np.floor_divide(np.floor(hi_e), tile), nt - 1).astype(np.int64)
    near = lambda x: np.abs(x / tile - np.round(x / tile)) * tile < band_edge
    amb = np.any(near(lo_e) | near(hi_e), axis=1)
    if tau > 0:
        rho = np.asarray(gs["density"], dtype=np.float64)
        amb |= np.abs(rho - tau) <= band_tau * tau
    empty = np.any(t0 > t1, axis=1) | (k2 < 0)
    widen = kappa * kappa * (slack - 1.0)
    rect = np.full((n, 6), -1, dtype=np.int64)
    lists = []
    for i in range(n):
        if empty[i]:
            lists.append(np.zeros(0, dtype=np.int64))
            continue
        rect[i, :3], rect[i, 3:] = t0[i], t1[i]
        tz, ty, tx = np.meshgrid(np.arange(t0[i, 2], t1[i, 2] + 1), np.arange(t0[i, 1], t1[i, 1] + 1),
                                 np.arange(t0[i, 0], t1[i, 0] + 1), indexing="ij")
        tx, ty, tz = tx.ravel(), ty.ravel(), tz.ravel()          # row-major, x fastest
        blo = np.stack([tx, ty, tz], axis=1) * tile - c[i]
        m = quad_min(np.broadcast_to(A[i], (tx.size, 3, 3)), blo, blo + (tile - 1))
        thr = k2[i] + widen
        amb[i] |= bool(np.any(np.abs(m - thr) <= band_cull * kappa * kappa * slack))
        hit = m <= thr
        lists.append(((tz[hit] * nt[1] + ty[hit]) * nt[0] + tx[hit]).astype(np.int64))
    count = np.array([len(l) for l in lists], dtype=np.int64)
    offset = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(count, out=offset[1:])
    emit_keys = np.concatenate(lists) if n else np.zeros(0, dtype=np.int64)
    emit_gauss = np.repeat(np.arange(n, dtype=np.int64), count)
    order = np.argsort(emit_keys, kind="stable")
    T = int(nt.prod())
    skeys = emit_keys[order]
    return dict(rect=rect, count=count, offset=offset, emit_keys=emit_keys, emit_gauss=emit_gauss,
                sorted_keys=skeys, sorted_gauss=emit_gauss[order], sorted_slots=order,
                tile_start=np.searchsorted(skeys, np.arange(T + 1), side="left"),
                tiles=tuple(int(t) for t in nt), ambiguous=amb)


def vox_support_tiles(gs: dict, grid: dict, kappa: float = 3.0, tile: int = 8, margin: float = 1e-3,
                      tau: float = 0.0) -> list:
    """Per Gaussian, the set of tile ids holding a voxel centre of the grid
    with d^2 <= k2_i - margin, k2_i its support bound (support_k2; kappa^2
    when tau = 0), by brute force over the voxels of its FP64 box, widened
    by one voxel."""
    dims = np.asarray(grid["dims"], dtype=np.int64)
    nt = (dims + tile - 1) // tile
    c, r, A, k2 = _voxel_frame(gs, grid, kappa, tau)
    out = []
    for i in range(c.shape[0]):
        if k2[i] < 0:
            out.append(set())
            continue
        lo = np.maximum(np.floor(c[i] - r[i]).astype(np.int64) - 1, 0)
        hi = np.minimum(np.ceil(c[i] + r[i]).astype(np.int64) + 1, dims - 1)
        if np.any(lo > hi):
            out.append(set())
            continue
        z, y, x = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                              np.arange(lo[0], hi[0] + 1), indexing="ij")
        d = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) - c[i]
        inside = np.einsum("ki,ij,kj->k", d, A[i], d) <= k2[i] - margin
        t = ((z.ravel()[inside] // tile) * nt[1] + y.ravel()[inside] // tile) * nt[0] + x.ravel()[inside] // tile
        out.append(set(t.tolist()))
    return out
