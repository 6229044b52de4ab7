"""CPU checks of the kernels' exact culling rules and of the oracle's tile
binning (no GPU).

The pixel kernels cull (tile quadrant, Gaussian) pairs, and the voxel
binning culls (tile, Gaussian) pairs, with a closed construction for the
largest value of the (negative) quadratic exponent over a box of pixel or
voxel centres:

* 2D (8x8 quadrants): the minimiser of a convex quadratic over a rectangle
  lies on the line x = clamp(u) or on the line y = clamp(v), and on each the
  best point is the clamped 1D minimiser;
* 3D (8^3 tiles): the minimiser lies on one of the three planes
  x_a = clamp(p_a); on each, the 2D rule above applies to the restricted
  form over the face.

Below, those constructions are written out in FP64 NumPy (the same steps
the kernels take) and compared on many random instances with
``oracle.tiles.quad_min``, which minimises by enumerating every face of the
box. The oracle itself is pinned here against dense sampling and SciPy's
bounded minimiser.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import tiles

RNG_SEED = 2024


def _spd(rng, n, k, cond_max=1e3):
    """n random symmetric positive definite k x k matrices, condition up to cond_max."""
    Q, _ = np.linalg.qr(rng.normal(size=(n, k, k)))
    ev = np.exp(rng.uniform(0.0, np.log(cond_max), size=(n, k))) * rng.uniform(0.05, 2.0, size=(n, 1))
    return np.einsum("nij,nj,nkj->nik", Q, ev, Q)


def _boxes(rng, n, k, side=7.0, spread=12.0):
    lo = rng.uniform(-spread, spread, size=(n, k))
    return lo, lo + side


# ---------------------------------------------------------------- the oracle's exact minimum

@pytest.mark.parametrize("k", [2, 3])
def test_quad_min_against_sampling_and_scipy(k):
    rng = np.random.default_rng(RNG_SEED + k)
    n = 60
    A = _spd(rng, n, k)
    lo, hi = _boxes(rng, n, k)
    lo[:5] = -3.0                                    # boxes holding the centre: minimum 0
    hi[:5] = 4.0
    m = tiles.quad_min(A, lo, hi)
    assert np.all(m[:5] == 0.0)
    for i in range(n):
        f = lambda d: d @ A[i] @ d
        best = min((minimize(f, x0, jac=lambda d: 2 * A[i] @ d, method="L-BFGS-B",
                             bounds=list(zip(lo[i], hi[i])), options=dict(ftol=1e-15, gtol=1e-12)).fun
                    for x0 in (lo[i], hi[i], 0.5 * (lo[i] + hi[i]))))
        assert m[i] <= best + 1e-9 * (1 + best)
        assert best <= m[i] + 1e-6 * (1 + m[i])
        # dense sampling: never below the exact minimum, and within what the
        # sampling step allows of it (a point delta from the minimiser x* adds
        # at most 2 |A x*| |delta| + lambda_max |delta|^2; |A x| is largest at
        # a corner of the box)
        steps = 40 if k == 3 else 200
        g = np.stack(np.meshgrid(*[np.linspace(lo[i, a], hi[i, a], steps + 1) for a in range(k)],
                                 indexing="ij"), axis=-1).reshape(-1, k)
        s = np.einsum("ki,ij,kj->k", g, A[i], g)
        assert s.min() >= m[i] - 1e-9 * (1 + m[i])
        delta = 0.5 * np.sqrt(k) * (hi[i] - lo[i]).max() / steps
        grad_bound = 2 * max(np.linalg.norm(A[i] @ c) for c in np.stack(np.meshgrid(
            *[[lo[i, a], hi[i, a]] for a in range(k)], indexing="ij"), axis=-1).reshape(-1, k))
        lam = np.linalg.eigvalsh(A[i]).max()
        assert s.min() <= m[i] + grad_bound * delta + lam * delta ** 2 + 1e-9


def test_quad_min_isotropic_is_squared_distance():
    """For A = I the minimum is the squared distance from the origin to the box."""
    rng = np.random.default_rng(RNG_SEED)
    lo, hi = _boxes(rng, 200, 3)
    dist = np.maximum(np.maximum(lo, -hi), 0.0)
    np.testing.assert_allclose(tiles.quad_min(np.broadcast_to(np.eye(3), (200, 3, 3)), lo, hi),
                               (dist ** 2).sum(axis=1), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- the kernels' constructions

def _rect_min(C, u, v, x0, x1, y0, y1):
    """The 2D rule of the splat kernels' quadrant test (FP64): smallest
    d^2 = [dx dy] C [dx dy]^T over [x0, x1] x [y0, y1] around (u, v)."""
    c00, c01, c11 = C[:, 0, 0], C[:, 0, 1], C[:, 1, 1]
    rx, ry = c01 / c11, c01 / c00
    X = np.clip(u, x0, x1)
    dxa = X - u
    dya = np.clip(v - rx * dxa, y0, y1) - v
    qa = c00 * dxa ** 2 + 2 * c01 * dxa * dya + c11 * dya ** 2
    Y = np.clip(v, y0, y1)
    dyb = Y - v
    dxb = np.clip(u - ry * dyb, x0, x1) - u
    qb = c00 * dxb ** 2 + 2 * c01 * dxb * dyb + c11 * dyb ** 2
    return np.minimum(qa, qb)


def _box_min(M, p, lo, hi):
    """The 3D rule of the voxel binning's tile test (FP64): smallest
    (x - p)^T M (x - p) over the box; per plane x_a = clamp(p_a), the 2D rule
    on the face, with the restricted form's centre (ybh, ych)."""
    best = np.full(p.shape[0], np.inf)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        D = np.clip(p[:, a], lo[:, a], hi[:, a]) - p[:, a]
        lb, hb = lo[:, b] - p[:, b], hi[:, b] - p[:, b]
        lc, hc = lo[:, c] - p[:, c], hi[:, c] - p[:, c]
        mbb, mcc, mbc = M[:, b, b], M[:, c, c], M[:, b, c]
        mab, mac = M[:, a, b], M[:, a, c]
        det = mbb * mcc - mbc * mbc
        ybh = -D * (mcc * mab - mbc * mac) / det
        ych = -D * (mbb * mac - mbc * mab) / det
        yb1 = np.clip(ybh, lb, hb)
        yc1 = np.clip(-(mbc * yb1 + D * mac) / mcc, lc, hc)
        yc2 = np.clip(ych, lc, hc)
        yb2 = np.clip(-(mbc * yc2 + D * mab) / mbb, lb, hb)
        base = M[:, a, a] * D * D
        f1 = base + 2 * D * (mab * yb1 + mac * yc1) + yb1 * (mbb * yb1 + 2 * mbc * yc1) + mcc * yc1 * yc1
        f2 = base + 2 * D * (mab * yb2 + mac * yc2) + yb2 * (mbb * yb2 + 2 * mbc * yc2) + mcc * yc2 * yc2
        best = np.minimum(best, np.minimum(f1, f2))
    return best


def test_quadrant_rule_is_exact():
    """The splat kernels' quadrant test equals the exact minimum over 8x8
    pixel-centre squares (100,000 random ellipses and squares, centres inside
    and outside, condition numbers up to 1e4)."""
    rng = np.random.default_rng(RNG_SEED + 10)
    n = 100_000
    C = _spd(rng, n, 2, cond_max=1e4)
    uv = rng.uniform(-20.0, 20.0, size=(n, 2))
    x0 = np.floor(rng.uniform(-24.0, 16.0, size=n)) + 0.5
    y0 = np.floor(rng.uniform(-24.0, 16.0, size=n)) + 0.5
    got = _rect_min(C, uv[:, 0], uv[:, 1], x0, x0 + 7, y0, y0 + 7)
    lo = np.stack([x0 - uv[:, 0], y0 - uv[:, 1]], axis=1)
    want = tiles.quad_min(C, lo, lo + 7)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9)


def test_tile_box_rule_is_exact():
    """The voxel binning's tile test equals the exact minimum over 8^3
    voxel-centre boxes (50,000 random ellipsoids and boxes)."""
    rng = np.random.default_rng(RNG_SEED + 11)
    n = 50_000
    M = _spd(rng, n, 3, cond_max=1e4)
    p = rng.uniform(-20.0, 20.0, size=(n, 3))
    lo = np.floor(rng.uniform(-24.0, 16.0, size=(n, 3)))
    got = _box_min(M, p, lo, lo + 7)
    want = tiles.quad_min(M, lo - p, lo + 7 - p)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9)


def test_tile_rules_on_degenerate_positions():
    """Centres exactly on faces, edges and corners of the box, and inside it."""
    M = np.broadcast_to(np.array([[2.0, 0.7, -0.3], [0.7, 1.0, 0.2], [-0.3, 0.2, 0.5]]), (27 + 1, 3, 3))
    lo = np.zeros((28, 3))
    pts = [np.array(c, dtype=float) for c in np.ndindex(3, 3, 3)]
    p = np.array([c * 3.5 for c in pts] + [[3.0, 2.0, 1.0]])   # {0, 3.5, 7}^3 and an interior point
    np.testing.assert_allclose(_box_min(M, p, lo, lo + 7), 0.0, atol=1e-12)
    p2 = np.array([[-1.0, 3.0, 3.0], [8.0, -2.0, 3.0], [-1.0, -1.0, -1.0], [9.0, 9.0, 9.0]])
    np.testing.assert_allclose(_box_min(M[:4], p2, lo[:4], lo[:4] + 7),
                               tiles.quad_min(M[:4], lo[:4] - p2, lo[:4] + 7 - p2), rtol=1e-12)


# ---------------------------------------------------------------- the oracle's voxel binning

def test_vox_bin_tiles_hand_case():
    """One isotropic Gaussian, sigma = 2 voxels at 64^3 (voxel size 1/64):
    centre at voxel-index coordinates (10.25, 20.5, 33.0), so its 3-sigma box
    spans voxels 4.25..16.25, 14.5..26.5, 27..39, i.e. tiles 0..2, 1..3,
    3..4. A tile is listed iff the squared distance from the centre to its
    voxel-centre box is at most (3 sigma)^2 * 1.001."""
    h = 1.0 / 64
    c = np.array([10.25, 20.5, 33.0])
    gs = dict(mean=((c + 0.5) * h - 0.5).reshape(3, 1).astype(np.float64),
              log_scale=np.full((3, 1), np.log(2 * h)), quat=np.array([[1.0], [0.0], [0.0], [0.0]]),
              density=np.array([1.0]))
    gr = dict(origin=(-0.5, -0.5, -0.5), spacing=(h, h, h), dims=(64, 64, 64))
    b = tiles.vox_bin_tiles(gs, gr)
    assert b["rect"][0].tolist() == [0, 1, 3, 2, 3, 4]
    want = []
    for tz in range(3, 5):
        for ty in range(1, 4):
            for tx in range(0, 3):
                lo = np.array([tx, ty, tz]) * 8.0
                d = np.maximum(np.maximum(lo - c, c - (lo + 7)), 0.0)
                if (d ** 2).sum() <= 36.0 * 1.001:
                    want.append((tz * 8 + ty) * 8 + tx)
    assert b["emit_keys"].tolist() == want
    assert b["count"][0] == len(want) < 18        # the cull removes some of the box's tiles
    assert b["tile_start"][-1] == len(want)


def test_vox_bin_tiles_superset_of_support():
    """Every tile holding a support voxel (d^2 <= 9 - 1e-3, brute force) is
    listed for its Gaussian; listed tiles are sorted stably (ascending
    Gaussian within a tile); tile_start partitions the sorted keys."""
    import synth_inputs as si
    gs = si.gaussians(300, 77, log_scale_mean=np.log(0.05))
    gr = dict(origin=(-0.5, -0.45, -0.5), spacing=(1 / 40, 1 / 36, 1 / 44), dims=(40, 35, 44))
    b = tiles.vox_bin_tiles(gs, gr)
    sup = tiles.vox_support_tiles(gs, gr)
    listed = [set(b["emit_keys"][b["offset"][i]:b["offset"][i + 1]].tolist()) for i in range(300)]
    for i in range(300):
        assert sup[i] <= listed[i], i
    assert sum(len(s) for s in sup) > 1000
    assert sum(len(s) for s in listed) < 1.8 * sum(len(s) for s in sup)   # the cull is tight
    sk, sg, st = b["sorted_keys"], b["sorted_gauss"], b["tile_start"]
    for t in range(len(st) - 1):
        assert np.all(sk[st[t]:st[t + 1]] == t)
        assert np.all(np.diff(sg[st[t]:st[t + 1]]) > 0)


def test_vox_bin_tiles_density_aware_support():
    """The density-aware support (tau > 0): for a hand-picked isotropic
    Gaussian (sigma 2 voxels, rho = 1) and tau = exp(-2), the support is
    d^2 <= 2 ln(1 / tau) = 4, i.e. a radius of 2 sigma = 4 voxels, so the
    box spans voxels 6.25..14.25, 16.5..24.5, 29..37 (tiles 0..1, 2..3,
    3..4). A Gaussian with rho <= tau gets no tile. For the random scene,
    every brute-force support tile is listed, the lists are a subset of the
    kappa lists, and a tau far below every density reproduces them."""
    import synth_inputs as si
    h = 1.0 / 64
    c = np.array([10.25, 20.5, 33.0])
    gs = dict(mean=np.repeat(((c + 0.5) * h - 0.5).reshape(3, 1), 2, axis=1),
              log_scale=np.full((3, 2), np.log(2 * h)), quat=np.array([[1.0, 1.0], [0, 0], [0, 0], [0, 0]]),
              density=np.array([1.0, 0.1]))
    gr = dict(origin=(-0.5, -0.5, -0.5), spacing=(h, h, h), dims=(64, 64, 64))
    tau = np.exp(-2.0)
    b = tiles.vox_bin_tiles(gs, gr, tau=tau)
    assert b["rect"][0].tolist() == [0, 2, 3, 1, 3, 4]
    assert b["count"][1] == 0 and b["rect"][1].tolist() == [-1] * 6
    want = []
    for tz in range(3, 5):
        for ty in range(2, 4):
            for tx in range(0, 2):
                lo = np.array([tx, ty, tz]) * 8.0
                d = np.maximum(np.maximum(lo - c, c - (lo + 7)), 0.0)
                if (d ** 2).sum() <= 16.0 + 36.0 * 0.001:
                    want.append((tz * 8 + ty) * 8 + tx)
    assert b["emit_keys"].tolist() == want

    gs = si.gaussians(300, 78, log_scale_mean=np.log(0.05))
    gr = dict(origin=(-0.5, -0.45, -0.5), spacing=(1 / 40, 1 / 36, 1 / 44), dims=(40, 35, 44))
    b0 = tiles.vox_bin_tiles(gs, gr)
    bt = tiles.vox_bin_tiles(gs, gr, tau=0.2)
    sup = tiles.vox_support_tiles(gs, gr, tau=0.2)
    rho = gs["density"].astype(np.float64)
    for i in range(300):
        lt = set(bt["emit_keys"][bt["offset"][i]:bt["offset"][i + 1]].tolist())
        l0 = set(b0["emit_keys"][b0["offset"][i]:b0["offset"][i + 1]].tolist())
        assert sup[i] <= lt <= l0, i
        if rho[i] <= 0.2:
            assert not lt
    assert bt["count"].sum() < 0.8 * b0["count"].sum()
    tiny = tiles.vox_bin_tiles(gs, gr, tau=1e-6)   # 2 ln(rho / tau) > 9 for every rho >= 0.1
    np.testing.assert_array_equal(tiny["emit_keys"], b0["emit_keys"])
    np.testing.assert_array_equal(tiny["rect"], b0["rect"])
