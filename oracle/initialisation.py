"""FP64 oracle of the initialisation path (Sec. 3.1): FDK reconstruction and
FDK-gradient sampling. TEST INFRASTRUCTURE ONLY (see the package docstring).

FDK follows Feldkamp, Davis and Kress for a full circular scan on a flat
detector, written out plainly: cosine pre-weight on the detector rescaled to
the rotation axis, a Ram-Lak ramp filter by direct linear convolution along
each row, distance-weighted backprojection with bilinear interpolation, and a
factor 1/2 because a full scan measures every ray twice.

Gradient sampling takes the paper's steps in order: threshold the
background, take the gradient magnitude, draw means with probability
proportional to it, set densities to k times the reconstruction at the
means, zero rotation, scale = nearest-neighbour distance. The integer
decision (which voxel a draw picks) is taken in FP32 with the same operations
as the kernels: the gradient magnitude in float32, quantised to 24 bits of its
maximum, summed exactly in 64-bit integers.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree


def _frame(theta, sod):
    c, s = math.cos(theta), math.sin(theta)
    W = np.array([[-s, c, 0.0], [0.0, 0.0, -1.0], [-c, -s, 0.0]])
    src = np.array([sod * c, sod * s, 0.0])
    return W, src


def _centres(grid):
    nx, ny, nz = grid["dims"]
    o = np.asarray(grid["origin"], dtype=np.float64)
    h = np.asarray(grid["spacing"], dtype=np.float64)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([o[0] + (x + 0.5) * h[0], o[1] + (y + 0.5) * h[1], o[2] + (z + 0.5) * h[2]], -1).reshape(-1, 3)


def ramp_filter_rows(pw, pitch):
    """q[n] = pitch * sum_k h[n - k] pw[k] along the last axis (linear
    convolution, zero outside), Ram-Lak h for sample spacing `pitch`."""
    W = pw.shape[-1]
    m = np.arange(-(W - 1), W)
    h = np.zeros(m.shape)
    h[m == 0] = 1.0 / (4.0 * pitch ** 2)
    odd = (m % 2) != 0
    h[odd] = -1.0 / (math.pi ** 2 * m[odd].astype(np.float64) ** 2 * pitch ** 2)
    flat = pw.reshape(-1, W)
    out = np.empty_like(flat)
    for r in range(flat.shape[0]):
        out[r] = np.convolve(flat[r], h)[W - 1:2 * W - 1]
    return pitch * out.reshape(pw.shape)


def fdk(img, geom: dict, angles, grid: dict) -> np.ndarray:
    """FDK of cone-beam projections img[V][H][W] (views covering 360 degrees
    uniformly) on `grid`; returns [nz][ny][nx] float64."""
    img = np.asarray(img, dtype=np.float64)
    V, H, W = img.shape
    sod, sdd = geom["sod"], geom["sdd"]
    ratio = sod / sdd
    pu, pv = geom["pitch_u"] * ratio, geom["pitch_v"] * ratio
    cu, cv = 0.5 * W + geom["off_u"], 0.5 * H + geom["off_v"]
    a = (np.arange(W) + 0.5 - cu) * pu
    b = (np.arange(H) + 0.5 - cv) * pv
    wgt = sod / np.sqrt(sod ** 2 + a[None, :] ** 2 + b[:, None] ** 2)
    q = ramp_filter_rows(img * wgt[None], pu)
    x = _centres(grid)
    fu, fv = sdd / geom["pitch_u"], sdd / geom["pitch_v"]
    acc = np.zeros(x.shape[0])
    for v in range(V):
        Wm, src = _frame(float(angles[v]), sod)
        t = (x - src) @ Wm.T
        ok = t[:, 2] > 0
        uu = fu * t[:, 0] / t[:, 2] + cu - 0.5
        ww = fv * t[:, 1] / t[:, 2] + cv - 0.5
        u0 = np.floor(uu).astype(np.int64)
        w0 = np.floor(ww).astype(np.int64)
        fuv, fwv = uu - u0, ww - w0
        val = np.zeros(x.shape[0])
        for du, dw, wt in ((0, 0, (1 - fuv) * (1 - fwv)), (1, 0, fuv * (1 - fwv)), (0, 1, (1 - fuv) * fwv),
                           (1, 1, fuv * fwv)):
            iu, iw = u0 + du, w0 + dw
            inside = (iu >= 0) & (iu < W) & (iw >= 0) & (iw < H)
            vals = np.zeros(x.shape[0])
            vals[inside] = q[v, iw[inside], iu[inside]]
            val += wt * vals
        acc += np.where(ok, (sod / np.where(ok, t[:, 2], 1.0)) ** 2 * val, 0.0)
    nx, ny, nz = grid["dims"]
    return (0.5 * 2.0 * math.pi / V * acc).reshape(nz, ny, nx)


def sampling_weights(vol32, background_fraction: float = 0.05, weighting: str = "gradient"):
    """Integer sampling weights: the float32 gradient magnitude of the
    background-thresholded volume (Sec. 3.1), or for the intensity-sampling
    baseline the thresholded, non-negative value itself, quantised to 24 bits
    of its maximum."""
    v = np.asarray(vol32, dtype=np.float32)
    thr = np.float32(background_fraction) * np.float32(v.max())
    vt = np.where(v >= thr, v, np.float32(0)).astype(np.float32)
    if weighting == "intensity":
        g = np.maximum(vt, np.float32(0))
        scale = np.float32(16777216.0) / np.float32(g.max())
        return np.floor(g * scale).astype(np.uint64)
    if weighting != "gradient":
        raise ValueError(weighting)
    p = np.pad(vt, 1)
    half = np.float32(0.5)
    gx = half * (p[1:-1, 1:-1, 2:] - p[1:-1, 1:-1, :-2])
    gy = half * (p[1:-1, 2:, 1:-1] - p[1:-1, :-2, 1:-1])
    gz = half * (p[2:, 1:-1, 1:-1] - p[:-2, 1:-1, 1:-1])
    sq = gx * gx + gy * gy
    g = np.sqrt(sq + gz * gz).astype(np.float32)
    scale = np.float32(16777216.0) / np.float32(g.max())
    return np.floor(g * scale).astype(np.uint64)


def trilinear(vol, c):
    """Trilinear interpolation of vol[nz][ny][nx] at continuous voxel-index
    coordinates c[m][3] = (x, y, z), zero outside the grid."""
    vol = np.asarray(vol, dtype=np.float64)
    nz, ny, nx = vol.shape
    f = np.floor(c)
    i0 = f.astype(np.int64)
    fr = c - f
    out = np.zeros(c.shape[0])
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                x, y, z = i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz
                w = ((fr[:, 0] if dx else 1 - fr[:, 0]) * (fr[:, 1] if dy else 1 - fr[:, 1]) *
                     (fr[:, 2] if dz else 1 - fr[:, 2]))
                ok = (x >= 0) & (x < nx) & (y >= 0) & (y < ny) & (z >= 0) & (z < nz)
                vals = np.zeros(c.shape[0])
                vals[ok] = vol[z[ok], y[ok], x[ok]]
                out += w * vals
    return out


def gradient_init(vol32, grid: dict, uniforms, background_fraction: float = 0.05, density_scale: float = 0.15,
                  min_scale: float = 1e-4, weighting: str = "gradient") -> dict:
    """FDK-gradient sampling initialisation (Sec. 3.1) of n = uniforms.shape[1]
    Gaussians; uniforms[4][n]: voxel choice, then position inside the voxel.
    weighting="intensity": the intensity-sampling baseline of the
    initialisation comparison (Sec. 4), which differs only in the weights."""
    u = np.asarray(uniforms, dtype=np.float64)
    n = u.shape[1]
    vol32 = np.asarray(vol32, dtype=np.float32)
    nz, ny, nx = vol32.shape
    w = sampling_weights(vol32, background_fraction, weighting).reshape(-1)
    cdf = np.zeros(w.size + 1, dtype=np.uint64)
    np.cumsum(w, out=cdf[1:])
    total = int(cdf[-1])
    target = np.floor(u[0] * float(total)).astype(np.uint64)
    target = np.minimum(target, np.uint64(total - 1))
    k = np.searchsorted(cdf, target, side="right") - 1
    idx = np.stack([k % nx, (k // nx) % ny, k // (nx * ny)], axis=1).astype(np.float64)
    o = np.asarray(grid["origin"], dtype=np.float64)
    h = np.asarray(grid["spacing"], dtype=np.float64)
    mean = o[None, :] + (idx + u[1:4].T) * h[None, :]
    density = density_scale * trilinear(vol32, idx + u[1:4].T - 0.5)
    d, _ = cKDTree(mean).query(mean, k=2)
    ls = np.log(np.maximum(d[:, 1], min_scale))
    quat = np.zeros((4, n))
    quat[0] = 1.0
    return dict(mean=mean.T.copy(), log_scale=np.tile(ls, (3, 1)), quat=quat, density=density,
                voxel=k.astype(np.int64))
