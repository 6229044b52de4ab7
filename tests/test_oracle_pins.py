"""Pins of the FP64 oracle against facts the paper and mathematics fix.

None of these tests re-types an oracle formula. Each compares the oracle
with something independent of it: the exact line integral and its
quadrature (Eq. 3), closed-form Gaussian masses, SciPy's rotation
convention, brute force, exact geometric symmetries and finite differences.
Each pin is chosen so that a plausible slip in the oracle (a dropped
Jacobian term, a wrong sign, a transposed rotation, a mis-scaled mu) fails
at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.spatial.transform import Rotation
from scipy.special import erfc

import oracle
import synth_inputs as si


def one(mean, log_scale, quat, density):
    return dict(mean=np.array(mean, dtype=np.float64).reshape(3, 1),
                log_scale=np.array(log_scale, dtype=np.float64).reshape(3, 1),
                quat=np.array(quat, dtype=np.float64).reshape(4, 1),
                density=np.array([density], dtype=np.float64))


def subset(gs, idx):
    idx = np.asarray(idx)
    return {k: (v[..., idx] if v.ndim > 1 else v[idx]) for k, v in gs.items()}


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


# --------------------------------------------------------------- Eq. 1 conventions

def test_quaternion_and_covariance_convention_matches_scipy():
    """The field of one Gaussian along its principal axis j, taken from
    SciPy's rotation of the same (w, x, y, z) quaternion, falls off with
    the j-th scale: rho * exp(-delta^2 / (2 s_j^2)). A transposed rotation,
    a scalar-last/first mix-up or a scale squared twice fails this."""
    rng = np.random.default_rng(5)
    for _ in range(5):
        q = rng.normal(size=4)
        ls = np.log(rng.uniform(0.02, 0.08, size=3))
        p = rng.uniform(-0.2, 0.2, size=3)
        g = one(p, ls, q, 0.7)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        for j in range(3):
            delta = 1.3 * math.exp(ls[j])
            x = p + delta * R[:, j]
            val = oracle.field_points(g, x[None, :])[0]
            assert val == pytest.approx(0.7 * math.exp(-0.5 * 1.3 ** 2), rel=1e-12)


# --------------------------------------------------------------- Eq. 3 / Eq. 4

def _random_scene(n, seed, sigma=0.04):
    rng = np.random.default_rng(seed)
    return dict(mean=rng.uniform(-0.25, 0.25, size=(3, n)),
                log_scale=np.log(sigma) + 0.3 * rng.normal(size=(3, n)),
                quat=rng.normal(size=(4, n)),
                density=rng.uniform(0.2, 1.0, size=n))


def test_exact_integral_matches_quadrature_cone_and_parallel():
    """Eq. 3's closed-form line integral equals Gauss-Legendre quadrature of
    the density field along the same physical ray."""
    gs = _random_scene(4, 1)
    for mode in ("cone", "parallel"):
        geom = si.geometry(64, mode=mode)
        ang = 0.7
        rec = oracle.splat_records(gs, geom, [ang])
        u = rec["uv"][:, 0] + np.array([0.3, -1.1, 2.0, 0.0])
        v = rec["uv"][:, 1] + np.array([-0.4, 0.9, 0.0, 1.7])
        e = oracle.exact_points(gs, geom, ang, u, v)
        if mode == "cone":
            lo, hi = 1.5 - 1.0, 1.5 + 1.0
        else:
            lo, hi = 2.0 - 1.0, 2.0 + 1.0
        q = oracle.quadrature_points(gs, geom, ang, u, v, lo, hi)
        np.testing.assert_allclose(e, q, rtol=1e-9, atol=1e-14)


def test_parallel_beam_splat_equals_exact_integral():
    """In parallel beam the projection of a 3D Gaussian is exactly a 2D
    Gaussian (Eq. 3 -> Eq. 4), so M with no cutoff equals E everywhere."""
    gs = _random_scene(6, 2)
    geom = si.geometry(64, mode="parallel")
    rng = np.random.default_rng(3)
    for ang in (0.0, 1.1, 4.0):
        u = rng.uniform(16, 48, size=200)
        v = rng.uniform(16, 48, size=200)
        m = oracle.project_points(gs, geom, ang, u, v, kappa=1e6)
        e = oracle.exact_points(gs, geom, ang, u, v)
        np.testing.assert_allclose(m, e, rtol=1e-10, atol=1e-14)


def test_cone_beam_mu_identity_at_splat_centre():
    """At the projected centre the ray passes through the mean, where the
    exact integral is rho * sqrt(2 pi / (d^T Sigma^-1 d)). M there is
    rho * mu, so the two agree for any Gaussian and view (pins mu)."""
    gs = _random_scene(8, 4, sigma=0.06)
    geom = si.geometry(64, mode="cone")
    for ang in (0.3, 2.2):
        rec = oracle.splat_records(gs, geom, [ang])
        for i in range(8):
            g1 = subset(gs, [i])
            u, v = rec["uv"][i]
            e = oracle.exact_points(g1, geom, ang, [u], [v])[0]
            m = oracle.project_points(g1, geom, ang, [u], [v], kappa=1e6)[0]
            assert m == pytest.approx(rec["w"][i], rel=1e-14)
            assert m == pytest.approx(e, rel=1e-11)


def test_cone_beam_splat_converges_to_exact_integral_for_small_gaussians():
    """The splat is a local affine approximation of the cone-beam integral:
    its footprint error relative to E must vanish as the Gaussian shrinks.
    A wrong ray-space Jacobian gives an O(1) footprint error that does not."""
    gaps = []
    base = _random_scene(1, 7, sigma=1.0)
    for sigma in (0.04, 0.02, 0.01, 0.005):
        g = dict(base)
        g["log_scale"] = base["log_scale"] + math.log(sigma)
        g["mean"] = np.array([[0.21], [-0.13], [0.17]])
        geom = si.geometry(2048, mode="cone")
        ang = 0.9
        rec = oracle.splat_records(g, geom, [ang])
        u0, v0 = rec["uv"][0]
        a, b, c = rec["shat"][0]
        su, sv = math.sqrt(a), math.sqrt(c)
        uu, vv = np.meshgrid(np.linspace(-2.5, 2.5, 21), np.linspace(-2.5, 2.5, 21))
        u = u0 + su * uu.ravel()
        v = v0 + sv * vv.ravel()
        m = oracle.project_points(g, geom, ang, u, v, kappa=1e6)
        e = oracle.exact_points(g, geom, ang, u, v)
        gaps.append(oracle.rel_l2(m, e))
    assert gaps[-1] < 2e-3
    for g0, g1 in zip(gaps[:-1], gaps[1:]):
        assert g1 < 0.6 * g0


def test_splat_mass_closed_form():
    """Sum over pixels of one splat = w 2 pi sqrt(det S^) times the mass
    inside the support ellipse (1 - e^-kappa^2/2)."""
    g = one([0.05, -0.03, 0.02], np.log([0.03, 0.05, 0.04]), [0.9, 0.2, -0.3, 0.1], 0.8)
    geom = si.geometry(256, mode="cone")
    ang = 0.4
    rec = oracle.splat_records(g, geom, [ang])
    a, b, c = rec["shat"][0]
    w = rec["w"][0]
    full = w * 2 * math.pi * math.sqrt(a * c - b * b)
    img6 = oracle.project(g, geom, [ang], kappa=6.0)
    assert img6.sum() == pytest.approx(full * (1 - math.exp(-18.0)), rel=1e-9)
    img3 = oracle.project(g, geom, [ang], kappa=3.0)
    assert img3.sum() == pytest.approx(full * (1 - math.exp(-4.5)), rel=2e-3)


def test_density_aware_support_closed_forms():
    """Density-aware support (Sec. 3.5 boxes that take the density into account):
    a pair counts only while its contribution w exp(-d^2/2) >= tau. For one
    splat whose cut 2 ln(w / tau) lies below kappa^2 the pixel sum is then
    2 pi sqrt(det S^) (w - tau); for one voxel Gaussian it is
    rho (2 pi)^(3/2) sqrt(det S) P(chi2_3 <= 2 ln(rho / tau)), with
    P(chi2_3 <= r^2) = erf(r / sqrt 2) - sqrt(2 / pi) r exp(-r^2 / 2).
    A Gaussian whose peak is below tau contributes nothing."""
    g = one([0.05, -0.03, 0.02], np.log([0.03, 0.05, 0.04]), [0.9, 0.2, -0.3, 0.1], 0.8)
    geom = si.geometry(256, mode="cone")
    ang = 0.4
    rec = oracle.splat_records(g, geom, [ang])
    a, b, c = rec["shat"][0]
    w = rec["w"][0]
    tau = 0.05 * w
    assert 2 * math.log(w / tau) < 9.0
    img = oracle.project(g, geom, [ang], tau=tau)
    assert img.sum() == pytest.approx(2 * math.pi * math.sqrt(a * c - b * b) * (w - tau), rel=2e-3)
    assert img[img > 0].min() >= tau * (1 - 1e-12)
    assert not oracle.project(g, geom, [ang], tau=1.01 * w).any()
    # tau small enough that kappa = 3 still binds: unchanged
    np.testing.assert_array_equal(oracle.project(g, geom, [ang], tau=1e-3 * w), oracle.project(g, geom, [ang]))

    ls = np.log([0.03, 0.045, 0.035])
    gv = one([0.02, -0.01, 0.03], ls, [0.3, -0.5, 0.7, 0.2], 0.9)
    grid = si.grid(64)
    h3 = np.prod(grid["spacing"])
    tau_v = 0.9 * math.exp(-0.5 * 5.0)           # cut at d^2 = 5
    r = math.sqrt(5.0)
    inside = math.erf(r / math.sqrt(2)) - math.sqrt(2 / math.pi) * r * math.exp(-0.5 * r * r)
    full = 0.9 * (2 * math.pi) ** 1.5 * math.exp(ls.sum())
    v = oracle.voxelize(gv, grid, tau=tau_v)
    assert v.sum() * h3 == pytest.approx(full * inside, rel=5e-3)
    assert not oracle.voxelize(gv, grid, tau=0.95).any()


def test_density_aware_support_reduces_to_a_smaller_kappa():
    """For one Gaussian in one view the density-aware support is the plain
    support with kappa_eff^2 = 2 ln(w / tau) (w = rho mu from the splat
    records; rho for the voxelizer): images, volumes and gradients equal
    those of kappa_eff with no density term; brute force equals the box
    variants; several Gaussians sum their own supports."""
    g = one([0.05, -0.03, 0.02], np.log([0.04, 0.06, 0.05]), [0.9, 0.2, -0.3, 0.1], 0.8)
    geom = si.geometry(64, mode="cone")
    ang = [1.1]
    w = oracle.splat_records(g, geom, ang)["w"][0]
    tau = 0.1 * w
    keff = math.sqrt(2 * math.log(w / tau))
    np.testing.assert_array_equal(oracle.project(g, geom, ang, tau=tau), oracle.project(g, geom, ang, kappa=keff))
    c = np.random.default_rng(4).normal(size=(1, 64, 64))
    ga = oracle.project_bwd(g, geom, ang, c, tau=tau)
    gb = oracle.project_bwd(g, geom, ang, c, kappa=keff)
    for k in ga:
        np.testing.assert_array_equal(ga[k], gb[k])
    grid = si.grid(40)
    keff_v = math.sqrt(2 * math.log(0.8 / 0.2))
    np.testing.assert_array_equal(oracle.voxelize(g, grid, tau=0.2), oracle.voxelize(g, grid, kappa=keff_v))
    cv = np.random.default_rng(5).normal(size=(40, 40, 40))
    va = oracle.voxelize_bwd(g, grid, cv, tau=0.2)
    vb = oracle.voxelize_bwd(g, grid, cv, kappa=keff_v)
    for k in va:
        np.testing.assert_array_equal(va[k], vb[k])
    gs = si.gaussians(200, 33, log_scale_mean=math.log(0.05))
    ang3 = si.angles(3)
    tau = 0.02
    np.testing.assert_allclose(oracle.project(gs, geom, ang3, tau=tau), oracle.project(gs, geom, ang3, tau=tau, brute=True),
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.voxelize(gs, grid, tau=0.3), oracle.voxelize(gs, grid, tau=0.3, brute=True),
                               rtol=1e-13, atol=1e-15)
    split = oracle.project(subset(gs, np.arange(0, 90)), geom, ang3, tau=tau) + \
        oracle.project(subset(gs, np.arange(90, 200)), geom, ang3, tau=tau)
    np.testing.assert_allclose(split, oracle.project(gs, geom, ang3, tau=tau), rtol=1e-12, atol=1e-14)


def test_projection_brute_force_equals_box_variant():
    gs = si.gaussians(300, 11)
    geom = si.geometry(48, mode="cone")
    ang = si.angles(3)
    a = oracle.project(gs, geom, ang)
    b = oracle.project(gs, geom, ang, brute=True)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------- Eq. 2, Sec. 3.3

def test_banded_projection_and_voxelization():
    """The banded variants return project()/voxelize() unchanged, and their
    band sums equal a brute-force sum over the pairs with |d^2 - 9| <= band
    (from the per-record conics); perturbing kappa^2 by less than the band
    moves no pixel or voxel by more than its band sum."""
    gs = si.gaussians(120, 31, log_scale_mean=math.log(0.06))
    gd = si.geometry(40, 36)
    ang = si.angles(3)
    band = 0.05
    img, bimg = oracle.project_banded(gs, gd, ang, band=band)
    np.testing.assert_array_equal(img, oracle.project(gs, gd, ang))
    rec = oracle.splat_records(gs, gd, ang)
    ys, xs = np.mgrid[0:36, 0:40] + 0.5
    want = np.zeros_like(bimg)
    for r in range(3 * 120):
        if rec["culled"][r]:
            continue
        du, dv = xs - rec["uv"][r, 0], ys - rec["uv"][r, 1]
        c0, c1, c2 = rec["conic"][r]
        d2 = c0 * du * du + 2 * c1 * du * dv + c2 * dv * dv
        want[r // 120] += np.where(np.abs(d2 - 9.0) <= band, rec["w"][r] * np.exp(-0.5 * d2), 0.0)
    np.testing.assert_allclose(bimg, want, rtol=1e-12, atol=1e-15)
    assert np.count_nonzero(bimg) > 100
    for k2 in (9.0 - 0.9 * band, 9.0 + 0.9 * band):
        moved = oracle.project(gs, gd, ang, kappa=math.sqrt(k2))
        assert np.all(np.abs(moved - img) <= bimg + 1e-12)
    gr = dict(origin=(-0.5, -0.45, -0.4), spacing=(1 / 24, 0.9 / 20, 0.8 / 22), dims=(24, 20, 22))
    vol, bvol = oracle.voxelize_banded(gs, gr, band=band)
    np.testing.assert_array_equal(vol, oracle.voxelize(gs, gr))
    assert np.count_nonzero(bvol) > 100
    for k2 in (9.0 - 0.9 * band, 9.0 + 0.9 * band):
        moved = oracle.voxelize(gs, gr, kappa=math.sqrt(k2), brute=True)
        assert np.all(np.abs(moved - vol) <= bvol + 1e-12)


def test_voxel_mass_closed_form():
    """Sum of voxel values times voxel volume = rho (2 pi)^(3/2) sqrt(det S)
    times the chi-square(3) mass inside kappa."""
    ls = np.log([0.03, 0.045, 0.035])
    g = one([0.02, -0.01, 0.03], ls, [0.3, -0.5, 0.7, 0.2], 0.9)
    grid = si.grid(64)
    h3 = np.prod(grid["spacing"])
    full = 0.9 * (2 * math.pi) ** 1.5 * math.exp(ls.sum())
    v8 = oracle.voxelize(g, grid, kappa=8.0)
    assert v8.sum() * h3 == pytest.approx(full, rel=1e-8)
    tail = erfc(3 / math.sqrt(2)) + math.sqrt(2 / math.pi) * 3 * math.exp(-4.5)
    v3 = oracle.voxelize(g, grid, kappa=3.0)
    assert v3.sum() * h3 == pytest.approx(full * (1 - tail), rel=5e-3)


def test_voxelizer_brute_force_equals_box_variant():
    gs = si.gaussians(300, 12)
    grid = dict(origin=(-0.5, -0.4, -0.45), spacing=(1 / 40, 1 / 36, 1 / 44), dims=(40, 29, 37))
    a = oracle.voxelize(gs, grid)
    b = oracle.voxelize(gs, grid, brute=True)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------- invariances

def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_invariances():
    gs = {k: v.astype(np.float64) for k, v in si.gaussians(200, 13).items()}
    geom = si.geometry(40, mode="cone")
    ang = [0.8]
    base = oracle.project(gs, geom, ang)
    # quaternion sign and scale
    for f in (-1.0, 3.0):
        g2 = dict(gs); g2["quat"] = f * gs["quat"]
        np.testing.assert_allclose(oracle.project(g2, geom, ang), base, rtol=1e-12, atol=1e-14)
    # permutation
    perm = np.random.default_rng(0).permutation(200)
    np.testing.assert_allclose(oracle.project(subset(gs, perm), geom, ang), base, rtol=1e-12, atol=1e-14)
    # linearity in density and additivity over subsets
    g2 = dict(gs); g2["density"] = 2.5 * gs["density"]
    np.testing.assert_allclose(oracle.project(g2, geom, ang), 2.5 * base, rtol=1e-12, atol=1e-14)
    a = oracle.project(subset(gs, np.arange(0, 80)), geom, ang)
    b = oracle.project(subset(gs, np.arange(80, 200)), geom, ang)
    np.testing.assert_allclose(a + b, base, rtol=1e-12, atol=1e-14)


def test_rotation_about_axis_equals_view_shift():
    """Rotating every Gaussian by phi about z and viewing at theta equals the
    unrotated scene at theta - phi (the orbit is a rotation about z)."""
    gs = {k: v.astype(np.float64) for k, v in si.gaussians(150, 14).items()}
    phi, theta = 0.61, 1.9
    Rz = np.array([[math.cos(phi), -math.sin(phi), 0], [math.sin(phi), math.cos(phi), 0], [0, 0, 1]])
    qz = np.array([math.cos(phi / 2), 0, 0, math.sin(phi / 2)])
    rot = dict(gs)
    rot["mean"] = Rz @ gs["mean"]
    rot["quat"] = np.stack([_qmul(qz, gs["quat"][:, i]) for i in range(150)], axis=1)
    geom = si.geometry(48, mode="cone")
    a = oracle.project(rot, geom, [theta])
    b = oracle.project(gs, geom, [theta - phi])
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------- gradients

def _fd_check(fwd, gs, analytic, h, rtol):
    for key in ("mean", "log_scale", "quat", "density"):
        arr = gs[key]
        num = np.zeros_like(arr)
        flat = arr.reshape(-1)
        for j in range(flat.size):
            def f(step):
                g2 = {k: v.copy() for k, v in gs.items()}
                g2[key].reshape(-1)[j] += step
                return fwd(g2)
            d1 = (f(h) - f(-h)) / (2 * h)
            d2 = (f(h / 2) - f(-h / 2)) / h
            num.reshape(-1)[j] = (4 * d2 - d1) / 3
        ana = analytic[key].reshape(num.shape)
        err = np.linalg.norm(ana - num) / max(np.linalg.norm(num), 1e-30)
        assert err < rtol, (key, err)


def test_projection_gradient_matches_finite_differences():
    """Analytic gradient of <c, M> (support held fixed: kappa = 8 makes the
    cutoff invisible at FD step size) vs Richardson central differences."""
    gs = _random_scene(4, 21, sigma=0.05)
    for mode in ("cone", "parallel"):
        geom = si.geometry(32, mode=mode)
        ang = [0.35, 2.4]
        c = np.random.default_rng(2).normal(size=(2, 32, 32))
        fwd = lambda g: float(np.sum(c * oracle.project(g, geom, ang, kappa=8.0)))
        ana = oracle.project_bwd(gs, geom, ang, c, kappa=8.0)
        _fd_check(fwd, gs, ana, 1e-4, 1e-7)


def test_projection_gradient_matches_finite_differences_at_2048_detector():
    """The scaling workload's geometry (2048^2 detector, F ~ 1450 px): three
    of its Gaussians, two views, kappa = 8, Richardson central differences
    with h = 1e-3."""
    full = si.gaussians(500000, 2)
    idx = np.array([11, 250000, 499999])
    gs = {k: np.ascontiguousarray(v[..., idx], dtype=np.float64) for k, v in full.items()}
    geom = si.geometry(2048)
    ang = [0.0, 2.2]
    c = np.random.default_rng(9).normal(size=(2, 2048, 2048))
    fwd = lambda g: float(np.sum(c * oracle.project(g, geom, ang, kappa=8.0)))
    ana = oracle.project_bwd(gs, geom, ang, c, kappa=8.0)
    _fd_check(fwd, gs, ana, 1e-3, 1e-6)


# --------------------------------------------------------------- ray-exact model (Eq. 3 with the support)

def test_ray_exact_isotropic_closed_form_with_cutoff():
    """An isotropic Gaussian (any rotation) integrates along a ray at
    perpendicular distance r from its mean to rho sigma sqrt(2 pi)
    exp(-r^2 / (2 sigma^2)), and the model keeps it iff r <= kappa sigma.
    r comes from the cross product with the ray's unit direction."""
    rng = np.random.default_rng(31)
    n = 5
    sig = np.array([0.03, 0.05, 0.02, 0.04, 0.06])
    gs = dict(mean=rng.uniform(-0.2, 0.2, size=(3, n)), log_scale=np.tile(np.log(sig), (3, 1)),
              quat=rng.normal(size=(4, n)), density=rng.uniform(0.3, 1.0, size=n))
    for mode in ("cone", "parallel"):
        geom = si.geometry(64, mode=mode)
        ang = 1.3
        rec = oracle.splat_records(gs, geom, [ang])
        for i in range(n):
            g1 = subset(gs, [i])
            # points around the projected centre, out to beyond the support
            u = rec["uv"][i, 0] + rng.uniform(-12, 12, size=300)
            v = rec["uv"][i, 1] + rng.uniform(-12, 12, size=300)
            o, d = oracle.rays(geom, ang, u, v)
            r = np.linalg.norm(np.cross(gs["mean"][:, i] - o, d), axis=1)
            ref = gs["density"][i] * sig[i] * math.sqrt(2 * math.pi) * np.exp(-0.5 * (r / sig[i]) ** 2)
            ref[r > 3.0 * sig[i]] = 0.0
            got = oracle.exact_points_cut(g1, geom, ang, u, v, kappa=3.0)
            far = np.abs(r / sig[i] - 3.0) > 1e-9
            assert 0 < np.sum(ref > 0) < 300
            np.testing.assert_allclose(got[far], ref[far], rtol=1e-10, atol=1e-15)


def test_ray_exact_large_kappa_matches_quadrature():
    gs = _random_scene(4, 32)
    for mode in ("cone", "parallel"):
        geom = si.geometry(64, mode=mode)
        ang = 2.1
        rec = oracle.splat_records(gs, geom, [ang])
        u = rec["uv"][:, 0] + np.array([0.4, -2.1, 1.0, 0.0])
        v = rec["uv"][:, 1] + np.array([-0.7, 0.3, 2.0, -1.2])
        lo, hi = (0.5, 2.5) if mode == "cone" else (1.0, 3.0)
        q = oracle.quadrature_points(gs, geom, ang, u, v, lo, hi)
        np.testing.assert_allclose(oracle.exact_points_cut(gs, geom, ang, u, v, kappa=20.0), q,
                                   rtol=1e-9, atol=1e-14)


def test_ray_exact_image_boxed_equals_brute_force_and_points():
    """The per-Gaussian pixel boxes are a superset of the support (brute
    force over every pixel gives the same image), and image pixels equal the
    point evaluation at pixel centres."""
    gs = _random_scene(30, 33, sigma=0.05)
    for mode in ("cone", "parallel"):
        geom = si.geometry(40, 36, mode=mode)
        geom["off_u"], geom["off_v"] = 2.5, -1.25
        ang = [0.2, 3.9]
        a = oracle.exact_project(gs, geom, ang)
        b = oracle.exact_project(gs, geom, ang, brute=True)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)
        ys, xs = np.meshgrid(np.arange(36), np.arange(40), indexing="ij")
        pts = oracle.exact_points_cut(gs, geom, ang[1], xs.ravel() + 0.5, ys.ravel() + 0.5)
        np.testing.assert_allclose(a[1].ravel(), pts, rtol=1e-13, atol=1e-15)
        assert a.max() > 0.1


def test_ray_exact_equals_splat_in_parallel_beam():
    """For parallel rays the projected 3D Gaussian is exactly the 2D splat and
    the ray's Mahalanobis distance is the splat's, so E_kappa = M_kappa
    pixel for pixel (away from the support boundary)."""
    gs = _random_scene(20, 34, sigma=0.05)
    geom = si.geometry(48, mode="parallel")
    ang = [0.6, 2.0]
    e = oracle.exact_project(gs, geom, ang)
    m = oracle.project(gs, geom, ang)
    np.testing.assert_allclose(e, m, rtol=1e-9, atol=1e-12 * m.max())


def test_ray_exact_differs_from_splat_in_cone_beam():
    """In cone beam the model gap is real: on the standard scan's geometry the
    splat's image departs from the ray-exact one by a fraction of a percent."""
    gs = si.gaussians(300, 35)
    geom = si.geometry(128)
    ang = si.angles(3)
    e = oracle.exact_project(gs, geom, ang)
    m = oracle.project(gs, geom, ang)
    gap = oracle.rel_l2(m, e)
    assert 1e-4 < gap < 5e-2, gap


def test_ray_exact_gradient_matches_finite_differences():
    """Analytic FP64 gradient of <c, E_kappa> (kappa = 8: the cutoff is
    invisible at the step size) vs Richardson central differences."""
    gs = _random_scene(4, 36, sigma=0.05)
    for mode in ("cone", "parallel"):
        geom = si.geometry(32, mode=mode)
        ang = [0.45, 2.9]
        c = np.random.default_rng(5).normal(size=(2, 32, 32))
        fwd = lambda g: float(np.sum(c * oracle.exact_project(g, geom, ang, kappa=8.0)))
        ana = oracle.exact_bwd(gs, geom, ang, c, kappa=8.0)
        _fd_check(fwd, gs, ana, 1e-4, 1e-7)


def test_ray_exact_gradient_holds_the_support_fixed():
    """At kappa = 3 the gradient is that of the uncut integrals summed over
    the pixels in the support at the unperturbed parameters."""
    gs = _random_scene(3, 37, sigma=0.1)
    geom = si.geometry(32)
    ang = [1.0]
    c = np.random.default_rng(6).normal(size=(1, 32, 32))
    ys, xs = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    u, v = xs.ravel() + 0.5, ys.ravel() + 0.5
    ana = oracle.exact_bwd(gs, geom, ang, c, kappa=3.0)
    for i in range(3):
        g1 = subset(gs, [i])
        inside = oracle.exact_points_cut(g1, geom, ang[0], u, v, kappa=3.0) > 0
        assert 20 < inside.sum() < 1024
        cu, uu, vv = c[0].ravel()[inside], u[inside], v[inside]
        fwd = lambda g: float(np.sum(cu * oracle.exact_points(g, geom, ang[0], uu, vv)))
        _fd_check(fwd, g1, {k: ana[k][..., i:i + 1] for k in ana}, 1e-4, 1e-7)


def test_voxelizer_gradient_matches_finite_differences():
    gs = _random_scene(4, 22, sigma=0.06)
    grid = si.grid(24)
    c = np.random.default_rng(3).normal(size=(24, 24, 24))
    fwd = lambda g: float(np.sum(c * oracle.voxelize(g, grid, kappa=8.0)))
    ana = oracle.voxelize_bwd(gs, grid, c, kappa=8.0)
    _fd_check(fwd, gs, ana, 1e-4, 1e-7)


def test_gradient_subset_selection_is_consistent():
    gs = si.gaussians(100, 23)
    geom = si.geometry(32)
    ang = si.angles(3)
    c = np.random.default_rng(4).normal(size=(3, 32, 32))
    full = oracle.project_bwd(gs, geom, ang, c)
    sel = np.array([5, 17, 99, 0])
    part = oracle.project_bwd(gs, geom, ang, c, sel=sel)
    for k in full:
        np.testing.assert_array_equal(part[k], full[k][..., sel])


# --------------------------------------------------------------- phantom

def test_phantom_sphere_chord():
    """A sphere of radius r projects to amp * 2 sqrt(r^2 - b^2), b = distance
    of the ray from the centre."""
    ph = dict(centre=np.array([[0.05, -0.02, 0.03]]), semi=np.array([[0.2, 0.2, 0.2]]),
              quat=np.array([[0.3, 0.1, -0.4, 0.8]]), amp=np.array([0.7]))
    geom = si.geometry(64, mode="cone")
    ang = 1.2
    img = oracle.phantom_project(ph, geom, [ang])[0]
    ys, xs = np.nonzero(np.ones((64, 64)))
    o, d = oracle.rays(geom, ang, xs + 0.5, ys + 0.5)
    c = ph["centre"][0]
    oc = o - c
    b2 = np.sum(oc * oc, axis=1) - np.sum(oc * d, axis=1) ** 2
    expect = np.where(b2 < 0.04, 0.7 * 2 * np.sqrt(np.maximum(0.04 - b2, 0)), 0.0)
    np.testing.assert_allclose(img[ys, xs], expect, rtol=1e-10, atol=1e-12)


def test_phantom_ellipsoid_chord_by_root_finding():
    """Chord of a rotated ellipsoid = distance between the two roots of
    f(t) = |diag(1/a) R^T (o + t d - c)|^2 - 1, found numerically (SciPy
    rotation of the (w, x, y, z) quaternion)."""
    ph = dict(centre=np.array([[0.02, 0.05, -0.04]]), semi=np.array([[0.25, 0.1, 0.15]]),
              quat=np.array([[0.6, -0.3, 0.5, 0.2]]), amp=np.array([1.0]))
    geom = si.geometry(96, mode="cone")
    ang = 0.5
    img = oracle.phantom_project(ph, geom, [ang])[0]
    q = ph["quat"][0]
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    a = ph["semi"][0]
    inside = np.argwhere(img > 0)
    assert len(inside) > 20
    rng = np.random.default_rng(0)
    picks = list(inside[rng.choice(len(inside), 25, replace=False)])
    picks += [np.array([y, x]) for y, x in rng.integers(0, 96, size=(25, 2))]
    checked = 0
    for y, x in picks:
        o, d = oracle.rays(geom, ang, [x + 0.5], [y + 0.5])
        o, d = o[0], d[0]
        f = lambda t: np.sum(((R.T @ (o + t * d - ph["centre"][0])) / a) ** 2) - 1
        ts = np.linspace(0.5, 2.5, 801)
        fs = np.array([f(t) for t in ts])
        k = np.argmin(fs)
        if fs[k] >= 0:
            assert img[y, x] == 0.0
            continue
        t0 = brentq(f, 0.5, ts[k], xtol=1e-14)
        t1 = brentq(f, ts[k], 2.5, xtol=1e-14)
        assert img[y, x] == pytest.approx(t1 - t0, rel=1e-9, abs=1e-12)
        checked += 1
    assert checked >= 25


def test_phantom_volume_membership():
    ph = si.phantom(6, 3)
    grid = si.grid(20)
    vol = oracle.phantom_volume(ph, grid)
    rng = np.random.default_rng(1)
    for _ in range(50):
        ix, iy, iz = rng.integers(0, 20, size=3)
        x = np.array(grid["origin"]) + (np.array([ix, iy, iz]) + 0.5) * np.array(grid["spacing"])
        acc = 0.0
        for e in range(6):
            q = ph["quat"][e]
            R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
            y = (R.T @ (x - ph["centre"][e])) / ph["semi"][e]
            if y @ y <= 1.0:
                acc += ph["amp"][e]
        assert vol[iz, iy, ix] == pytest.approx(acc, abs=1e-12)


# --------------------------------------------------------------- binning reference

def test_binning_hand_cases():
    """Hand-computed tile rectangles for 16x16 tiles on a 64x48 detector."""
    uv = np.array([[16.0, 16.0], [0.2, 0.2], [63.9, 47.9], [-10.0, 5.0], [30.0, 20.0]], np.float32)
    r = np.array([[0.4, 0.4], [0.1, 0.1], [20.0, 1.0], [3.0, 3.0], [2.5, 13.0]], np.float32)
    b = oracle.bin_tiles(uv, r, 64, 48)
    # pixel centres 15.5 .. 16.4 -> column 15 only -> tile 0
    assert list(b["rect"][0]) == [0, 0, 0, 0]
    # centre 0.2, half 0.1: floor(0.1 - 0.5) = -1 .. floor(0.3 - 0.5) = -1 -> clipped lo 0, hi -1 -> empty
    assert b["count"][1] == 0
    # x: floor(43.4)=43 -> tile 2 .. floor(83.4)=83 -> tile 5, clipped to 3; y: floor(46.4)=46 -> tile 2 .. floor(48.4)=48 -> tile 3, clipped to 2
    assert list(b["rect"][2]) == [2, 2, 3, 2]
    assert b["count"][3] == 0
    # x: floor(27.0)=27 .. floor(32.0)=32 -> tiles 1..2; y: floor(6.5)=6 .. floor(32.5)=32 -> tiles 0..2
    assert list(b["rect"][4]) == [1, 0, 2, 2]
    assert b["count"].tolist() == [1, 0, 2, 0, 6]
    assert b["offset"].tolist() == [0, 1, 1, 3, 3, 9]
    # keys emitted row-major inside each rect, tiles_x = 4
    assert b["keys"].tolist() == [0, 10, 11, 1, 2, 5, 6, 9, 10]
    assert b["sorted_keys"].tolist() == sorted(b["keys"].tolist())
    # stable: the two records on tile 10 keep record order (2 before 4)
    assert b["sorted_keys"].tolist() == [0, 1, 2, 5, 6, 9, 10, 10, 11]
    assert b["sorted_vals"].tolist() == [0, 4, 4, 4, 4, 4, 2, 4, 2]
    assert b["tile_start"].tolist() == [0, 1, 2, 3, 3, 3, 4, 5, 5, 5, 6, 8, 9]


def test_binning_covers_every_support_pixel():
    """Every FP64 support pair with d^2 <= 9 - 1e-4 lies in a tile the
    FP32 binning lists for its record."""
    gs = si.gaussians(400, 31)
    geom = si.geometry(64)
    ang = si.angles(2)
    rec = oracle.splat_records(gs, geom, ang)
    uv32 = rec["uv"].astype(np.float32)
    r32 = (np.float32(3.0) * np.sqrt(rec["shat"][:, [0, 2]].astype(np.float32))).astype(np.float32)
    b = oracle.bin_tiles(uv32, r32, 64, 64, cull=rec["culled"], n_views=2)
    n = 400
    ys, xs = np.mgrid[0:64, 0:64]
    for r in range(2 * n):
        if rec["culled"][r]:
            continue
        du = xs + 0.5 - rec["uv"][r, 0]
        dv = ys + 0.5 - rec["uv"][r, 1]
        c0, c1, c2 = rec["conic"][r]
        d2 = c0 * du * du + 2 * c1 * du * dv + c2 * dv * dv
        inside = d2 <= 9 - 1e-4
        if not inside.any():
            continue
        tx0, ty0, tx1, ty1 = b["rect"][r]
        tx = xs[inside] // 16
        ty = ys[inside] // 16
        assert b["count"][r] > 0
        assert tx.min() >= tx0 and tx.max() <= tx1 and ty.min() >= ty0 and ty.max() <= ty1


def test_binning_sort_is_stable_and_ranges_partition():
    gs = si.gaussians(300, 32)
    geom = si.geometry(64)
    ang = si.angles(3)
    rec = oracle.splat_records(gs, geom, ang)
    uv32 = rec["uv"].astype(np.float32)
    r32 = (np.float32(3.0) * np.sqrt(rec["shat"][:, [0, 2]].astype(np.float32))).astype(np.float32)
    b = oracle.bin_tiles(uv32, r32, 64, 64, cull=rec["culled"], n_views=3)
    start = b["tile_start"]
    assert start[0] == 0 and start[-1] == b["sorted_keys"].size
    for t in range(start.size - 1):
        seg_k = b["sorted_keys"][start[t]:start[t + 1]]
        seg_v = b["sorted_vals"][start[t]:start[t + 1]]
        assert np.all(seg_k == t)
        assert np.all(np.diff(seg_v) > 0)  # ascending record index within a tile


# --------------------------------------------------------------- losses / metrics

def test_l1_psnr_adam_hand_values():
    img = np.array([[[1.0, 2.0], [3.0, 4.0]]])
    gt = np.array([[[1.5, 2.0], [2.0, 6.0]]])
    loss, g = oracle.l1_loss_grad(img, gt)
    assert loss == pytest.approx((0.5 + 0.0 + 1.0 + 2.0) / 4)
    assert g.tolist() == [[[-0.25, 0.0], [0.25, -0.25]]]
    vol = np.array([1.0, 2.0, 3.0, 4.0])
    ref = np.array([1.0, 2.0, 3.0, 2.0])
    assert oracle.psnr(vol, ref) == pytest.approx(10 * math.log10(9 / 1.0))
    p, m, v = oracle.adam_step(np.array([1.0]), np.array([0.5]), np.zeros(1), np.zeros(1), 1, 0.1,
                               eps=0.0)
    # first step of Adam moves by lr * sign(g)
    assert p[0] == pytest.approx(0.9)
    assert m[0] == pytest.approx(0.05) and v[0] == pytest.approx(0.00025)


def test_gradient_band_brackets_cutoff_perturbations():
    """Moving the hard cutoff anywhere inside the boundary band changes the
    gradient by at most the band's absolute contribution mass; with a
    vanishing band the banded gradient is the plain one."""
    gs = si.gaussians(300, 41)
    gd = si.geometry(48)
    ang = si.angles(3)
    c = si.normals((3, 48, 48), 42).astype(np.float64)
    core = oracle.project_bwd(gs, gd, ang, c, band=1e-3)
    assert sum(float(np.abs(v).sum()) for v in core["band_abs"].values()) > 0
    for kap in (3.0 * (1 - 1e-5), 3.0, 3.0 * (1 + 1e-5)):
        plain = oracle.project_bwd(gs, gd, ang, c, kappa=kap)
        for k, e in oracle.banded_grad_error(plain, core).items():
            assert e < 1e-12, (kap, k, e)
    tiny = oracle.project_bwd(gs, gd, ang, c, band=1e-300)
    plain = oracle.project_bwd(gs, gd, ang, c)
    for k in ("mean", "log_scale", "quat", "density"):
        np.testing.assert_array_equal(tiny[k], plain[k])
    # voxelizer
    gr = si.grid(24)
    cv = si.normals((24, 24, 24), 43).astype(np.float64)
    vcore = oracle.voxelize_bwd(gs, gr, cv, band=1e-3)
    for kap in (3.0 * (1 - 1e-5), 3.0 * (1 + 1e-5)):
        plain = oracle.voxelize_bwd(gs, gr, cv, kappa=kap)
        for k, e in oracle.banded_grad_error(plain, vcore).items():
            assert e < 1e-12, (kap, k, e)


# --------------------------------------------------------------- initialisation (Sec. 3.1)

def test_fdk_reconstructs_uniform_sphere_and_ellipsoid():
    """FDK of the exact projections of a uniform body returns its density in
    the interior (within the discretisation error of 75 views of 128^2)."""
    for semi, quat, amp in (((0.2, 0.2, 0.2), (1.0, 0, 0, 0), 1.0), ((0.22, 0.15, 0.18), (0.8, 0.3, -0.2, 0.4), 0.6)):
        ph = dict(centre=np.array([[0.05, -0.03, 0.02]]), semi=np.array([semi]), quat=np.array([quat]),
                  amp=np.array([amp]))
        gd = si.geometry(128)
        ang = si.angles(75)
        img = oracle.phantom_project(ph, gd, ang)
        gr = dict(origin=(-0.07, -0.15, -0.10), spacing=(0.01, 0.01, 0.01), dims=(24, 24, 24))
        vol = oracle.fdk(img.astype(np.float32), gd, ang, gr).reshape(-1)
        x = oracle.initialisation._centres(gr)
        q = np.array(quat) / np.linalg.norm(quat)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        y = (x - ph["centre"][0]) @ R / np.array(semi)
        inner = np.sum(y * y, axis=1) < 0.55 ** 2
        assert inner.sum() > 200
        assert np.all(np.abs(vol[inner] / amp - 1.0) < 0.03)
        assert abs(vol[inner].mean() / amp - 1.0) < 0.01


def test_gradient_sampling_hand_case():
    """A 4-voxel row [0, 1, 1, 0]: central differences 0.5, 0.5, -0.5, -0.5,
    equal weights 2^24 each; draws land in quarter intervals of u."""
    vol = np.zeros((1, 1, 4), dtype=np.float32)
    vol[0, 0, 1:3] = 1.0
    w = oracle.sampling_weights(vol)
    assert w.reshape(-1).tolist() == [1 << 24] * 4
    grid = dict(origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), dims=(4, 1, 1))
    u = np.array([[0.0, 0.24, 0.26, 0.99], [0.5] * 4, [0.5] * 4, [0.5] * 4])
    out = oracle.gradient_init(vol, grid, u)
    assert out["voxel"].tolist() == [0, 0, 1, 3]
    np.testing.assert_allclose(out["mean"][0], [0.5, 0.5, 1.5, 3.5])
    # density = 0.15 * value at the voxel centre (jitter 1/2 puts the mean there)
    np.testing.assert_allclose(out["density"], 0.15 * np.array([0.0, 0.0, 1.0, 0.0]))
    assert np.all(out["quat"][0] == 1) and np.all(out["quat"][1:] == 0)


def test_gradient_sampling_background_threshold_and_frequencies():
    """Voxels below 5% of the maximum do not contribute; draws follow the
    integer weights (chi-square test against the exact multinomial law)."""
    rng = np.random.default_rng(3)
    vol = rng.uniform(0.0, 1.0, size=(6, 7, 8)).astype(np.float32)
    vol[vol < 0.2] = 0.01  # below 5% of the max after thresholding -> zero
    w = oracle.sampling_weights(vol).reshape(-1).astype(np.float64)
    p = w / w.sum()
    n = 200000
    u = rng.random((4, n))
    grid = dict(origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), dims=(8, 7, 6))
    k = oracle.gradient_init(vol, grid, u)["voxel"]
    counts = np.bincount(k, minlength=w.size)
    assert np.all(counts[w == 0] == 0)
    nz = p > 0
    chi2 = np.sum((counts[nz] - n * p[nz]) ** 2 / (n * p[nz]))
    dof = nz.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_intensity_sampling_hand_case():
    """Intensity baseline on the row [0.01, 1, 3, -2] (max 3, threshold
    0.15): weights floor(v * 2^24 / 3) = [0, 5592405, 2^24, 0]; total
    22369621, so u0 = 0.2 lands in voxel 1 and u0 = 0.3 in voxel 2 (the
    interval edge sits at u0 = 5592405 / 22369621 = 0.25000000...)."""
    vol = np.array([[[0.01, 1.0, 3.0, -2.0]]], dtype=np.float32)
    w = oracle.sampling_weights(vol, weighting="intensity")
    assert w.reshape(-1).tolist() == [0, 5592405, 1 << 24, 0]
    grid = dict(origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), dims=(4, 1, 1))
    u = np.array([[0.0, 0.2, 0.24999, 0.25001, 0.3, 0.999999], [0.5] * 6, [0.5] * 6, [0.5] * 6])
    out = oracle.gradient_init(vol, grid, u, weighting="intensity")
    assert out["voxel"].tolist() == [1, 1, 1, 2, 2, 2]
    np.testing.assert_allclose(out["density"], 0.15 * np.array([1.0, 1.0, 1.0, 3.0, 3.0, 3.0]), rtol=1e-7)
    # the gradient rule on the same (thresholded) row [0, 1, 3, 0]: central
    # differences 0.5, 1.5, -0.5, -1.5, so it weighs the edges, not the mass
    g = oracle.sampling_weights(vol).reshape(-1)
    assert g.tolist() == [5592405, 1 << 24, 5592405, 1 << 24]


def test_intensity_sampling_frequencies():
    """Draws follow the thresholded intensities (chi-square against the exact
    multinomial law of the integer weights, whose ratios are those of the
    values to within 2^-24)."""
    rng = np.random.default_rng(4)
    vol = rng.uniform(-0.2, 1.0, size=(5, 6, 7)).astype(np.float32)
    w = oracle.sampling_weights(vol, weighting="intensity").reshape(-1).astype(np.float64)
    v = vol.reshape(-1).astype(np.float64)
    keep = v >= np.float32(0.05) * np.float32(vol.max())
    assert np.all(w[~keep] == 0)
    np.testing.assert_allclose(w[keep] / w.max(), v[keep] / v.max(), atol=2 ** -23)
    n = 200000
    u = rng.random((4, n))
    grid = dict(origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), dims=(7, 6, 5))
    k = oracle.gradient_init(vol, grid, u, weighting="intensity")["voxel"]
    counts = np.bincount(k, minlength=w.size)
    p = w / w.sum()
    assert np.all(counts[w == 0] == 0)
    nz = p > 0
    chi2 = np.sum((counts[nz] - n * p[nz]) ** 2 / (n * p[nz]))
    dof = nz.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_trilinear_is_exact_on_linear_fields_and_nn_scale_is_brute_force():
    nz, ny, nx = 5, 6, 7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = 0.3 + 0.1 * x - 0.05 * y + 0.02 * z
    c = np.random.default_rng(0).uniform(0, 4, size=(100, 3))
    np.testing.assert_allclose(oracle.trilinear(vol, c), 0.3 + 0.1 * c[:, 0] - 0.05 * c[:, 1] + 0.02 * c[:, 2],
                               rtol=1e-12)
    vol32 = np.ones((6, 6, 6), dtype=np.float32)
    vol32[2:4, 2:4, 2:4] = 2.0
    grid = dict(origin=(-0.3, -0.3, -0.3), spacing=(0.1, 0.1, 0.1), dims=(6, 6, 6))
    u = np.random.default_rng(1).random((4, 300))
    out = oracle.gradient_init(vol32, grid, u)
    m = out["mean"].T
    d = np.sqrt(((m[:, None, :] - m[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    np.testing.assert_allclose(out["log_scale"][0], np.log(np.maximum(d.min(1), 1e-4)), rtol=1e-12)


# ---------------------------------------------------------------------------
# Learned initializer (MLP oracle)

def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100),
                        np.array([0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9,
                                  1.0 + 3 * 2 ** -9, -1.0 - 2 ** -9, 65504.0])])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    np.testing.assert_array_equal(oracle.mlp.bf16_round(x), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert oracle.mlp.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    assert oracle.mlp.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


def _mlp_case(rng, n, k=544, h=128, o=32):
    w = dict(w1=rng.normal(0, 0.06, (h, k)), b1=rng.normal(0, 0.1, h), w2=rng.normal(0, 0.12, (h, h)),
             b2=rng.normal(0, 0.1, h), w3=rng.normal(0, 0.12, (o, h)), b3=rng.normal(0, 0.5, o))
    x = rng.normal(0, 1, (n, k))
    ls = rng.normal(-3, 0.5, (3, n))
    q = rng.normal(0, 1, (4, n))
    t = oracle.mlp.canonical_target(rng.uniform(0.1, 1, n), ls, q)
    return w, x, t


def _mlp_loss(x, w, t):
    a = oracle.mlp.forward(x, w["w1"], w["b1"], w["w2"], w["b2"], w["w3"], w["b3"], round_between=False)
    return oracle.mlp.heads(a["z3"], t)[1]


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    w, x, t = _mlp_case(rng, 24, k=40, h=16, o=32)
    a = oracle.mlp.forward(x, w["w1"], w["b1"], w["w2"], w["b2"], w["w3"], w["b3"], round_between=False)
    _, _, dz3 = oracle.mlp.heads(a["z3"], t)
    g = oracle.mlp.backward(x, a, w["w2"], w["w3"], dz3, round_between=False)
    eps = 1e-6
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        flat = w[name].reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = _mlp_loss(x, w, t)
            flat[idx] = old - eps
            lm = _mlp_loss(x, w, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g["d" + name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_mlp_heads_gradient_and_quaternion_sign_invariance():
    rng = np.random.default_rng(12)
    n = 30
    z3 = rng.normal(0, 1, (n, 32))
    _, _, t = _mlp_case(rng, n)
    base = rng.normal(-4, 0.5, n)
    t[[3, 9], 0] = 0.0  # two dead targets: only their density term counts
    for b in (None, base):
        p, loss, g = oracle.mlp.heads(z3, t, b)
        assert np.all(g[:, 8:] == 0)
        assert np.all(g[[3, 9], 1:8] == 0)
        eps = 1e-6
        for i, j in [(0, 0), (1, 1), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 2), (9, 0), (9, 1)]:
            zp = z3.copy(); zp[i, j] += eps
            zm = z3.copy(); zm[i, j] -= eps
            fd = (oracle.mlp.heads(zp, t, b)[1] - oracle.mlp.heads(zm, t, b)[1]) / (2 * eps)
            assert abs(fd - g[i, j]) <= 1e-7, (i, j, fd, g[i, j])
    np.testing.assert_allclose(p[1:4], base[None, :] + z3[:, 1:4].T, rtol=1e-15)
    # a dead target's shape terms do not count: changing its predicted shape leaves the loss
    zd = z3.copy(); zd[3, 1:8] += 0.7
    assert oracle.mlp.heads(zd, t, base)[1] == pytest.approx(loss, abs=1e-15)
    p, loss, g = oracle.mlp.heads(z3, t)
    # q and -q describe one rotation: predictions and targets of either sign give one loss
    zf = z3.copy(); zf[:, 4:8] *= -1
    tf = t.copy(); tf[:, 4:8] *= -1
    assert oracle.mlp.heads(zf, t)[1] == pytest.approx(loss, abs=1e-14)
    assert oracle.mlp.heads(z3, tf)[1] == pytest.approx(loss, abs=1e-14)
    # the scale of the raw quaternion does not matter; softplus closed form
    zs = z3.copy(); zs[:, 4:8] *= 3.7
    assert oracle.mlp.heads(zs, t)[1] == pytest.approx(loss, abs=1e-13)
    np.testing.assert_allclose(p[0], np.log1p(np.exp(z3[:, 0])), rtol=1e-14)
    # a perfect prediction has zero loss and zero gradient
    perfect = np.zeros((n, 32))
    perfect[:, 0] = np.log(np.expm1(t[:, 0]))
    perfect[:, 1:8] = t[:, 1:8] * np.r_[1, 1, 1, 2.5, 2.5, 2.5, 2.5]
    _, l0, g0 = oracle.mlp.heads(perfect, t)
    assert l0 == pytest.approx(0.0, abs=1e-14)
    assert np.abs(g0).max() < 1e-14


def test_canonical_target_defines_the_same_gaussian():
    rng = np.random.default_rng(13)
    n = 200
    ls = rng.normal(-3, 0.5, (3, n))
    ls[:, :5] = ls[0, :5]                     # fully tied scales
    ls[1, 5:10] = ls[0, 5:10]                 # partly tied
    q = rng.normal(0, 1, (4, n))
    rho = rng.uniform(0.1, 1, n)
    t = oracle.mlp.canonical_target(rho, ls, q)
    np.testing.assert_array_equal(t[:, 0], rho)
    assert np.all(np.diff(t[:, 1:4], axis=1) <= 0)
    assert np.all(t[:, 4] >= 0)
    np.testing.assert_allclose(np.linalg.norm(t[:, 4:8], axis=1), 1.0, atol=1e-13)
    for i in range(n):
        R0 = Rotation.from_quat(np.r_[q[1:, i], q[0, i]]).as_matrix()
        S0 = R0 @ np.diag(np.exp(2 * ls[:, i])) @ R0.T
        R1 = Rotation.from_quat(np.r_[t[i, 5:8], t[i, 4]]).as_matrix()
        S1 = R1 @ np.diag(np.exp(2 * t[i, 1:4])) @ R1.T
        np.testing.assert_allclose(S1, S0, rtol=1e-12, atol=1e-16)
    # sorted input with w >= 0 is returned unchanged
    ls_s = -np.sort(-ls, axis=0)
    qn = q / np.linalg.norm(q, axis=0)
    qn *= np.where(qn[0] < 0, -1.0, 1.0)
    t2 = oracle.mlp.canonical_target(rho, ls_s, qn)
    np.testing.assert_allclose(t2[:, 4:8], qn.T, atol=1e-12)
    # a permutation (with a sign flip to stay proper) of distinct axes maps back to the same target
    P = np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1.0]])
    for i in range(10, 30):
        R0 = Rotation.from_quat(np.r_[qn[1:, i], qn[0, i]]).as_matrix()
        Rp = R0 @ P.T
        qp = Rotation.from_matrix(Rp).as_quat()
        lp = (np.abs(P) @ ls_s[:, i])
        t3 = oracle.mlp.canonical_target(rho[i:i + 1], lp[:, None], np.r_[qp[3], qp[:3]][:, None])
        np.testing.assert_allclose(t3[0], t2[i], atol=1e-12)


def test_patch_features_sample_a_linear_field_at_the_stated_offsets():
    n = 32
    g = si.grid(n)
    o = np.asarray(g["origin"], dtype=np.float64)
    h = np.asarray(g["spacing"], dtype=np.float64)
    idx = np.stack(np.meshgrid(*(np.arange(n),) * 3, indexing="ij"), -1)  # [z][y][x] -> (z, y, x)
    cz, cy, cx = (o[::-1] + (idx + 0.5) * h[::-1]).transpose(3, 0, 1, 2)
    a = np.array([0.3, -1.1, 2.0])
    vol = (a[0] * cx + a[1] * cy + a[2] * cz + 0.25).astype(np.float32)
    rng = np.random.default_rng(14)
    mean = rng.uniform(-0.5 + 5 * h[0], 0.5 - 5 * h[0], (3, 16))
    f = oracle.mlp.patches(vol, g, mean, 2.0)
    offs = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    for m in range(16):
        for fi in rng.choice(512, 40, replace=False):
            iz, iy, ix = offs[fi]
            p = mean[:, m] + h * (np.array([ix, iy, iz]) - 3.5)
            vol_lin = a @ p + 0.25
            assert f[m, fi] == pytest.approx(2.0 * vol_lin, abs=2e-6)
    np.testing.assert_allclose(f[:, 512:515], 2 * mean.T)
    assert np.all(f[:, 515:] == 0)
    ex = rng.normal(0, 1, (2, 16))
    fe = oracle.mlp.patches(vol, g, mean, 2.0, extra=ex)
    np.testing.assert_array_equal(fe[:, :515], f[:, :515])
    np.testing.assert_array_equal(fe[:, 515:517], ex.T)
    assert np.all(fe[:, 517:] == 0)
    # a patch that leaves the grid reads zeros outside it
    corner = np.full((3, 1), -0.5 + 0.5 * h[0])
    fc = oracle.mlp.patches(np.ones_like(vol), g, corner, 1.0)
    np.testing.assert_allclose(fc[0, 0], 0.0)
    np.testing.assert_allclose(fc[0, 511], 1.0)


# ---------------------------------------------------------------------------
# 3D total variation (TV term of Eq. 5)

def test_tv_hand_values_invariances_and_finite_differences():
    # 1 x 2 x 3 volume (nz, ny, nx): x-differences 1, 3 / -2, 0; y-differences 1, -2, -5
    v = np.array([[[0.0, 1.0, 4.0], [1.0, -1.0, -1.0]]], dtype=np.float32)
    loss, g = oracle.tv_loss_grad(v, scale=2.0)
    assert loss == pytest.approx(2.0 * (1 + 3 + 2 + 0 + 1 + 2 + 5) / 6, rel=1e-15)
    # voxel (0,0,0): x-diff +1 -> -1, y-diff +1 -> -1; voxel (0,1,1): x-diffs -2 (in: -1), 0; y-diff -2 (in: -1)
    np.testing.assert_allclose(g[0, 0, 0], 2.0 * (-1 - 1) / 6)
    np.testing.assert_allclose(g[0, 1, 1], 2.0 * (-1 + 0 - 1) / 6)
    np.testing.assert_allclose(g.sum(), 0.0, atol=1e-15)  # translation invariance of TV
    assert oracle.tv_loss_grad(np.full((4, 5, 6), 3.5, np.float32))[0] == 0.0
    rng = np.random.default_rng(31)
    w = rng.normal(size=(5, 6, 7)).astype(np.float32)
    l0, g0 = oracle.tv_loss_grad(w)
    assert oracle.tv_loss_grad(w + np.float32(2.0))[0] == pytest.approx(l0, rel=1e-6)
    assert oracle.tv_loss_grad(-w)[0] == pytest.approx(l0, rel=1e-15)
    # TV is piecewise linear: central differences are exact away from ties
    w64 = w.astype(np.float64)
    for idx in [(0, 0, 0), (2, 3, 4), (4, 5, 6), (1, 0, 6)]:
        h = 1e-3
        wp = w64.copy(); wp[idx] += h
        wm = w64.copy(); wm[idx] -= h
        f = lambda a: sum(np.abs(np.diff(a, axis=ax)).sum() for ax in range(3)) / a.size
        assert (f(wp) - f(wm)) / (2 * h) == pytest.approx(g0[idx], abs=1e-9)


# ---------------------------------------------------------------------------
# SSIM term of Eq. 5

def test_ssim_window_identity_constants_and_brute_force():
    rng = np.random.default_rng(41)
    x = rng.uniform(0, 1, (2, 17, 23))
    loss, g = oracle.ssim_loss_grad(x, x)
    assert loss == pytest.approx(0.0, abs=1e-14)
    assert np.abs(g).max() < 1e-14
    w = oracle.ssim_window()
    assert w.sum() == pytest.approx(1.0, abs=1e-15) and np.argmax(w) == 5 and w[0] == pytest.approx(w[10])
    # brute force at a few pixels (zero padding), from the definition
    y = rng.uniform(0, 1, (2, 17, 23))
    c1, c2 = 1e-4, 9e-4
    W2 = np.outer(w, w)
    pad = lambda a: np.pad(a, ((0, 0), (5, 5), (5, 5)))
    xp, yp = pad(x), pad(y)
    vals = []
    for v in range(2):
        for i in range(17):
            for j in range(23):
                px, py = xp[v, i:i + 11, j:j + 11], yp[v, i:i + 11, j:j + 11]
                mx, my = (W2 * px).sum(), (W2 * py).sum()
                sx = (W2 * px * px).sum() - mx * mx
                sy = (W2 * py * py).sum() - my * my
                sxy = (W2 * px * py).sum() - mx * my
                vals.append((2 * mx * my + c1) * (2 * sxy + c2) / ((mx * mx + my * my + c1) * (sx + sy + c2)))
    loss, _ = oracle.ssim_loss_grad(x, y, scale=0.7)
    assert loss == pytest.approx(0.7 * (1 - np.mean(vals)), rel=1e-12)


def test_ssim_gradient_matches_finite_differences():
    rng = np.random.default_rng(42)
    x = rng.uniform(0, 1, (2, 13, 15))
    y = rng.uniform(0, 1, (2, 13, 15))
    _, g = oracle.ssim_loss_grad(x, y, scale=0.5)
    h = 1e-6
    for idx in [(0, 0, 0), (0, 6, 7), (1, 12, 14), (1, 3, 10), (0, 12, 0)]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (oracle.ssim_loss_grad(xp, y, scale=0.5)[0] - oracle.ssim_loss_grad(xm, y, scale=0.5)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-11)


def test_ssim3d_identity_brute_force_and_finite_differences():
    rng = np.random.default_rng(43)
    x = rng.uniform(0, 1, (7, 8, 9))
    y = rng.uniform(0, 1, (7, 8, 9))
    l0, g0 = oracle.ssim3d_loss_grad(x, x)
    assert l0 == pytest.approx(0.0, abs=1e-14) and np.abs(g0).max() < 1e-14
    w = oracle.ssim_window()
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    pad = lambda a: np.pad(a, 5)
    xp, yp = pad(x), pad(y)
    c1, c2 = 1e-4, 9e-4
    vals = []
    for i in range(7):
        for j in range(8):
            for k in range(9):
                px, py = xp[i:i + 11, j:j + 11, k:k + 11], yp[i:i + 11, j:j + 11, k:k + 11]
                mx, my = (W3 * px).sum(), (W3 * py).sum()
                sx = (W3 * px * px).sum() - mx * mx
                sy = (W3 * py * py).sum() - my * my
                sxy = (W3 * px * py).sum() - mx * my
                vals.append((2 * mx * my + c1) * (2 * sxy + c2) / ((mx * mx + my * my + c1) * (sx + sy + c2)))
    loss, g = oracle.ssim3d_loss_grad(x, y, scale=0.3)
    assert loss == pytest.approx(0.3 * (1 - np.mean(vals)), rel=1e-12)
    h = 1e-4   # the gradient entries are ~1e-5 of a loss ~0.3: a larger step keeps rounding below 1e-8
    for idx in [(0, 0, 0), (3, 4, 5), (6, 7, 8), (2, 0, 8)]:
        xp_ = x.copy(); xp_[idx] += h
        xm_ = x.copy(); xm_[idx] -= h
        fd = (oracle.ssim3d_loss_grad(xp_, y, scale=0.3)[0] - oracle.ssim3d_loss_grad(xm_, y, scale=0.3)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-5, abs=1e-12)


def test_scaling_workload_gradients_match_central_differences_64_gaussians():
    """The 64 Gaussians the scaling workload's gradient test samples (of
    500,000; 2048^2 detector, F ~ 1450 px), two views, support frozen (kappa
    = 8 puts the cutoff far below the step's effect): the analytic gradient
    of <c, M> against FP64 central differences with h = 1e-3, Richardson-
    extrapolated with h / 2. M is a sum over Gaussians, so each Gaussian's
    differences are taken with it alone in the scene."""
    full = si.gaussians(500000, 2)
    sel = np.random.default_rng(16).choice(500000, 64, replace=False)
    gs = {k: np.ascontiguousarray(v[..., sel], dtype=np.float64) for k, v in full.items()}
    geom = si.geometry(2048)
    ang = [0.0, 2.2]
    c = np.random.default_rng(9).normal(size=(2, 2048, 2048))
    ana = oracle.project_bwd(gs, geom, ang, c, kappa=8.0)
    h = 1e-3
    for key in ("mean", "log_scale", "quat", "density"):
        num = np.zeros_like(gs[key])
        for i in range(64):
            one = subset(gs, [i])
            # the weighted sum over the pixels the Gaussian reaches (its
            # footprint plus a margin far wider than a step can move it)
            nz = np.nonzero(oracle.project(one, geom, ang, kappa=8.0))
            box = tuple(slice(max(a.min() - 16, 0), a.max() + 17) for a in nz)
            cb = c.reshape(2, 2048, 2048)[box]
            for j in range(one[key].shape[0] if one[key].ndim == 2 else 1):
                def f(step):
                    g2 = {k: v.copy() for k, v in one.items()}
                    g2[key].reshape(-1)[j] += step
                    return float(np.sum(cb * oracle.project(g2, geom, ang, kappa=8.0)[box]))
                d1 = (f(h) - f(-h)) / (2 * h)
                d2 = (f(h / 2) - f(-h / 2)) / h
                if one[key].ndim == 2:
                    num[j, i] = (4 * d2 - d1) / 3
                else:
                    num[i] = (4 * d2 - d1) / 3
        err = np.linalg.norm(ana[key] - num) / np.linalg.norm(num)
        assert err < 1e-6, (key, err)
