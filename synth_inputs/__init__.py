"""Seeded synthetic inputs for the Gaussian X-ray rasterizer and voxelizer.

This module holds random draws and workload descriptions only. It contains
none of the method's arithmetic: no projection, no covariance, no kernel
evaluation. Both the FP64 oracle (``oracle/``) and the HIP path
(``paper_2604_01844_amd``) consume what it returns, and neither imports the
other.

Draws use NumPy's PCG64 generator, are made in float64 and rounded once to
float32 where the consumer is the FP32 GPU path, so that both sides see the
same bits.

Workloads (sizes follow the paper's experiments, Sec. 4.1 and Sec. 4.2, and
the Fig. 3 kernel evaluation; the paper's datasets are not available, so
these seeded scenes stand in for them):

* ``tiny``  -- 2,000 Gaussians, 24 cone-beam views of 64x64, 64^3 voxels.
* ``scan``  -- 50,000 Gaussians, 75 views of 512x512, 256^3 voxels
  (the paper's standard sparse-view setting, Sec. 4.1).
* ``scale`` -- 500,000 Gaussians, 50 views of 2048x2048, 512^3 voxels
  (the high-resolution setting of Sec. 4.2).
* ``fit``   -- 200,000 Gaussians fitted to a 256^3 phantom volume (Sec. 3.6).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "CONFIGS",
    "gaussians",
    "phantom",
    "random_phantom",
    "perturbed_phantom",
    "angles",
    "geometry",
    "grid",
    "uniforms",
    "normals",
]

# Circular cone-beam orbit: source-to-origin and source-to-detector distances
# in units of the reconstruction cube's edge.
SOD = 1.5
SDD = 2.0

CONFIGS = {
    "tiny": dict(n_gauss=2000, n_views=24, det=64, vol=64, n_ell=10,
                 seed=0, phantom_seed=100),
    "scan": dict(n_gauss=50000, n_views=75, det=512, vol=256, n_ell=40,
                 seed=1, phantom_seed=101),
    "scale": dict(n_gauss=500000, n_views=50, det=2048, vol=512, n_ell=40,
                  seed=2, phantom_seed=102),
    "fit": dict(n_gauss=200000, n_views=0, det=0, vol=256, n_ell=40,
                seed=3, phantom_seed=103),
}


def gaussians(n: int, seed: int, *, log_scale_mean: float = math.log(0.03),
              log_scale_sd: float = 0.3, lo: float = -0.5, hi: float = 0.5,
              density_lo: float = 0.1, density_hi: float = 1.0) -> dict:
    """Random anisotropic Gaussians in the unit cube [-1/2, 1/2]^3.

    Centres are uniform, log standard deviations i.i.d. normal per axis,
    quaternions are raw 4D standard-normal draws (their direction is a
    uniform rotation; the method normalises them), densities uniform.
    Returned arrays are float32, structure-of-arrays:
    ``mean[3][n]``, ``log_scale[3][n]``, ``quat[4][n]`` (w, x, y, z),
    ``density[n]``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = rng.uniform(lo, hi, size=(3, n))
    log_scale = rng.normal(log_scale_mean, log_scale_sd, size=(3, n))
    quat = rng.normal(size=(4, n))
    density = rng.uniform(density_lo, density_hi, size=n)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(mean=f(mean), log_scale=f(log_scale), quat=f(quat),
                density=f(density))


def phantom(n_ell: int, seed: int) -> dict:
    """Random additive ellipsoid phantom (float64 parameters).

    Ellipsoid 0 is the body: semi-axes U(0.30, 0.42), amplitude 0.5.
    The others have centres uniform in the ball of radius 0.22 (drawn by
    rejection from the enclosing cube), semi-axes U(0.02, 0.12) and
    amplitudes U(0.1, 0.5). Every ellipsoid has a raw 4D normal quaternion
    as its orientation. Amplitudes add where ellipsoids overlap.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = np.zeros((n_ell, 3))
    semi = np.zeros((n_ell, 3))
    amp = np.zeros(n_ell)
    quat = rng.normal(size=(n_ell, 4))
    semi[0] = rng.uniform(0.30, 0.42, size=3)
    amp[0] = 0.5
    for e in range(1, n_ell):
        while True:
            c = rng.uniform(-0.22, 0.22, size=3)
            if c @ c <= 0.22 * 0.22:
                break
        centre[e] = c
        semi[e] = rng.uniform(0.02, 0.12, size=3)
        amp[e] = rng.uniform(0.1, 0.5)
    return dict(centre=centre, semi=semi, quat=quat, amp=amp)


def random_phantom(seed: int, lo: int = 20, hi: int = 60) -> dict:
    """Phantom with a seeded ellipsoid count U{lo..hi} (the training-pair
    scenes of the learned initializer; seeds 1000+ for training, 2000+ held
    out, 1999 for calibrating the PSNR target)."""
    n_ell = int(np.random.Generator(np.random.PCG64(seed + 7_000_000)).integers(lo, hi + 1))
    return phantom(n_ell, seed)


def perturbed_phantom(ph: dict, seed: int, shift: float = 0.01, scale: float = 0.1, amp: float = 0.2) -> dict:
    """A prior scan of the same object: each ellipsoid's centre moved by up to
    `shift` per axis, semi-axes scaled by U(1 - scale, 1 + scale), amplitudes
    by U(1 - amp, 1 + amp); the body's amplitude is kept."""
    rng = np.random.Generator(np.random.PCG64(seed + 9_000_000))
    n = ph["amp"].shape[0]
    out = {k: np.array(v, dtype=np.float64, copy=True) for k, v in ph.items()}
    out["centre"] = out["centre"] + rng.uniform(-shift, shift, size=(n, 3))
    out["semi"] = out["semi"] * rng.uniform(1 - scale, 1 + scale, size=(n, 3))
    f = rng.uniform(1 - amp, 1 + amp, size=n)
    f[0] = 1.0
    out["amp"] = out["amp"] * f
    return out


def angles(n_views: int) -> np.ndarray:
    """View angles 2*pi*k/V, k = 0..V-1, as float32 (no duplicate at 360)."""
    k = np.arange(n_views, dtype=np.float64)
    return (2.0 * math.pi * k / n_views).astype(np.float32)


def geometry(det_w: int, det_h: int | None = None, *, mode: str = "cone",
             sod: float = SOD, sdd: float = SDD) -> dict:
    """Flat-detector geometry description.

    The detector is sqrt(2)*SDD wide (it covers the cone tangent to the unit
    cube's circumsphere at SOD 1.5); pitches are float32-rounded.
    ``mode`` is "cone" or "parallel".
    """
    det_h = det_w if det_h is None else det_h
    width = math.sqrt(2.0) * sdd
    return dict(mode=mode, sod=float(np.float32(sod)), sdd=float(np.float32(sdd)),
                det_w=int(det_w), det_h=int(det_h),
                pitch_u=float(np.float32(width / det_w)),
                pitch_v=float(np.float32(width / det_h)),
                off_u=0.0, off_v=0.0, near=float(np.float32(1e-2)))


def grid(n: int | tuple, lo: float = -0.5, hi: float = 0.5) -> dict:
    """Axis-aligned voxel grid covering [lo, hi]^3 with n^3 voxels.

    ``origin`` is the outer corner of voxel (0, 0, 0); voxel (i, j, k) has
    its centre at origin + (index + 1/2) * spacing. Values are float32-exact.
    """
    dims = (n, n, n) if isinstance(n, int) else tuple(int(d) for d in n)
    spacing = tuple(float(np.float32((hi - lo) / d)) for d in dims)
    return dict(origin=(float(np.float32(lo)),) * 3, spacing=spacing, dims=dims)


def uniforms(n: int, seed: int) -> np.ndarray:
    """n float64 variates U[0, 1)."""
    return np.random.Generator(np.random.PCG64(seed)).random(n)


def normals(shape, seed: int) -> np.ndarray:
    """Standard-normal float32 array, e.g. weights of a random linear loss."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=shape).astype(np.float32)
