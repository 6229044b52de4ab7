"""FP64 oracle of the learned initializer's MLP. TEST INFRASTRUCTURE ONLY.

The network is 544 -> 128 (ReLU) -> 128 (ReLU) -> 32, of which 8 outputs are
used: softplus density, three log-scales (optionally offsets from a given
per-sample base), and a quaternion normalised to unit length. Operands are
BF16 (round to nearest even from FP32); products and sums are taken in FP64
here; activations and the output gradient are rounded to BF16 between
layers, as the kernels store them. The loss per sample is
(rho - rho_t)^2 + live * (|s - s_t|^2 + (1 - (q . q_t)^2)), live =
[rho_t > 1e-3] (a fitted Gaussian without density has no meaningful shape),
averaged over samples.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 (ties to even) via FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(x, w1, b1, w2, b2, w3, b3, round_between=True):
    """x [m][544] (BF16 values), w1 [128][544], ... -> dict of z1, h1, z2, h2, z3."""
    r = bf16_round if round_between else (lambda a: np.asarray(a, dtype=np.float64))
    z1 = x @ w1.T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ w2.T + b2
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ w3.T + b3
    return dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3)


LIVE_DENSITY = 1e-3


def heads(z3, target=None, base_log_scale=None):
    """Predicted parameters [8][n] and, with a target [n][8], the mean loss and
    its gradient with respect to z3 (columns beyond 8 get zero)."""
    y = np.asarray(z3, dtype=np.float64)
    n = y.shape[0]
    rho = np.logaddexp(0.0, y[:, 0])
    base = np.zeros(n) if base_log_scale is None else np.asarray(base_log_scale, dtype=np.float64)
    ls = base[:, None] + y[:, 1:4]
    q = y[:, 4:8]
    qn = np.maximum(np.linalg.norm(q, axis=1), 1e-12)
    qh = q / qn[:, None]
    params = np.concatenate([rho[None], ls.T, qh.T], axis=0)
    if target is None:
        return params, None, None
    t = np.asarray(target, dtype=np.float64)
    live = (t[:, 0] > LIVE_DENSITY).astype(np.float64)
    dot = np.sum(qh * t[:, 4:8], axis=1)
    loss = np.mean((rho - t[:, 0]) ** 2 + live * (np.sum((ls - t[:, 1:4]) ** 2, axis=1) + (1.0 - dot ** 2)))
    g = np.zeros_like(y)
    g[:, 0] = 2.0 * (rho - t[:, 0]) / (1.0 + np.exp(-y[:, 0])) / n
    g[:, 1:4] = live[:, None] * 2.0 * (ls - t[:, 1:4]) / n
    gh = -2.0 * dot[:, None] * t[:, 4:8]
    proj = np.sum(gh * qh, axis=1)
    g[:, 4:8] = live[:, None] * (gh - qh * proj[:, None]) / qn[:, None] / n
    return params, loss, g


def backward(x, acts, w2, w3, dz3, round_between=True):
    """Weight and bias gradients given the (BF16) output gradient dz3."""
    r = bf16_round if round_between else (lambda a: np.asarray(a, dtype=np.float64))
    dz3 = r(dz3)
    dw3 = dz3.T @ acts["h2"]
    db3 = dz3.sum(0)
    dz2 = r(np.where(acts["z2"] > 0, dz3 @ w3, 0.0))
    dw2 = dz2.T @ acts["h1"]
    db2 = dz2.sum(0)
    dz1 = r(np.where(acts["z1"] > 0, dz2 @ w2, 0.0))
    dw1 = dz1.T @ x
    db1 = dz1.sum(0)
    return dict(dw1=dw1, db1=db1, dw2=dw2, db2=db2, dw3=dw3, db3=db3)


def patches(vol32, grid: dict, mean, inv_norm: float, extra=None) -> np.ndarray:
    """Features [n][544]: 8^3 trilinear samples one voxel apart centred on each
    mean (zero outside), times inv_norm; then 2 * mean; then the rows of
    extra [k][n]; zeros. FP64."""
    from .initialisation import trilinear
    mean = np.asarray(mean, dtype=np.float64)
    n = mean.shape[1]
    o = np.asarray(grid["origin"], dtype=np.float64)
    h = np.asarray(grid["spacing"], dtype=np.float64)
    c = (mean.T - o) / h - 0.5
    offs = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    offs = offs[:, ::-1] - 3.5  # feature f = ((iz * 8) + iy) * 8 + ix -> offsets (ix, iy, iz)
    feats = np.zeros((n, 544))
    pts = (c[:, None, :] + offs[None, :, :]).reshape(-1, 3)
    feats[:, :512] = inv_norm * trilinear(vol32, pts).reshape(n, 512)
    feats[:, 512:515] = 2.0 * mean.T
    if extra is not None:
        e = np.asarray(extra, dtype=np.float64)
        feats[:, 515:515 + e.shape[0]] = e.T
    return feats


def canonical_target(density, log_scale, quat) -> np.ndarray:
    """Targets [n][8] from Gaussian parameters: log-scales in descending order
    with the rotation's columns permuted to match (and made proper), the
    quaternion of that rotation with w >= 0."""
    from scipy.spatial.transform import Rotation
    ls = np.asarray(log_scale, dtype=np.float64)
    q = np.asarray(quat, dtype=np.float64)
    n = ls.shape[1]
    order = np.argsort(-ls, axis=0, kind="stable")
    R = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=1)).as_matrix()
    Rp = np.take_along_axis(R, order.T[:, None, :], axis=2)
    det = np.linalg.det(Rp)
    Rp[:, :, 2] *= np.sign(det)[:, None]
    qc = Rotation.from_matrix(Rp).as_quat()  # x, y, z, w
    qc = np.stack([qc[:, 3], qc[:, 0], qc[:, 1], qc[:, 2]], axis=1)
    qc *= np.where(qc[:, :1] < 0, -1.0, 1.0)
    out = np.zeros((n, 8))
    out[:, 0] = density
    out[:, 1:4] = np.take_along_axis(ls, order, axis=0).T
    out[:, 4:8] = qc
    return out
