"""Adaptive density control: plain NumPy reference.

TEST INFRASTRUCTURE ONLY: used by the test suite; the product path never
imports it, and it imports nothing from the product.

Sec. 3.4 states that the loss gradient is used to prune, clone or split
Gaussians, and Suppl. C caps the count 10% above the initial one. The paper
gives no criteria or thresholds; the readings written out here:

* statistic: per Gaussian, the Euclidean norm of dL/dmean summed over the
  optimiser steps since the last densification, and the number of those
  steps in which it was non-zero; the score is their ratio (the count
  floored at 1);
* prune when the density is below a threshold or the largest standard
  deviation above one (NaNs prune);
* densify the survivors whose score exceeds a threshold: split those whose
  largest standard deviation exceeds a size threshold into two children
  drawn from the parent (mean + R diag(s) z, z standard normal), with
  standard deviations divided by a shrink factor and the density scaled by
  shrink^3 / 2, and clone the others (two copies at half the density); both
  keep the total mass rho (2 pi)^(3/2) s1 s2 s3;
* when the candidates do not fit under the cap, the largest scores are
  densified (ties: lower index), the rest kept;
* output order: survivors in input order, a clone's copy right after it, a
  split parent replaced by its two children; every output Gaussian carries
  its source's Adam moments (fresh zero moments late in a run make Adam's
  first updates of the new Gaussians several times the learning rate, since
  the bias correction follows the global step count).

Decisions are comparisons of FP32 values in FP32 (the score by correctly
rounded FP32 division, sizes in the log domain), as the GPU takes them.
"""
from __future__ import annotations

import math

import numpy as np

PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3
F32 = np.float32


def rotation(quat) -> np.ndarray:
    """R[3][3][n] of the normalised quaternions quat[4][n] (w, x, y, z)."""
    q = np.asarray(quat, dtype=np.float64)
    w, x, y, z = q / np.linalg.norm(q, axis=0)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def accumulate(grad_mean, stat) -> np.ndarray:
    """stat[2][n] plus (|dL/dmean|, [|dL/dmean| > 0]), in FP64."""
    norm = np.sqrt(np.sum(np.asarray(grad_mean, dtype=np.float64) ** 2, axis=0))
    out = np.array(stat, dtype=np.float64, copy=True)
    out[0] += norm
    out[1] += norm > 0
    return out


def classify(gs: dict, stat, *, grad_threshold, split_scale, prune_density, prune_scale):
    """(code[n], score[n]) with the decisions taken in FP32."""
    ls = np.max(np.asarray(gs["log_scale"], dtype=F32), axis=0)
    rho = np.asarray(gs["density"], dtype=F32)
    st = np.asarray(stat, dtype=F32)
    with np.errstate(invalid="ignore"):
        prune = ~(rho >= F32(prune_density)) | ~(ls <= F32(math.log(prune_scale)))
        score = (st[0] / np.maximum(st[1], F32(1.0))).astype(F32)
        cand = ~prune & (score > F32(grad_threshold))
        split = ls > F32(math.log(split_scale))
    code = np.where(prune, PRUNE, np.where(cand, np.where(split, SPLIT, CLONE), KEEP))
    return code, score


def densify(gs: dict, m: dict, v: dict, stat, normals, *, grad_threshold, split_scale, prune_density,
            prune_scale, split_shrink=1.6, n_max: int):
    """One densification step. gs, m, v: dicts of SoA arrays (mean [3][n],
    log_scale [3][n], quat [4][n], density [n]); normals [6][n]. Returns
    (gs_out, m_out, v_out, code) in FP64."""
    code, score = classify(gs, stat, grad_threshold=grad_threshold, split_scale=split_scale,
                           prune_density=prune_density, prune_scale=prune_scale)
    n = code.shape[0]
    n_surv = int(np.sum(code != PRUNE))
    if n_surv > n_max:
        raise ValueError("n_max is below the number of surviving Gaussians")
    room = n_max - n_surv
    cand = [i for i in range(n) if code[i] >= CLONE]
    if len(cand) > room:
        ranked = sorted(cand, key=lambda i: (-float(score[i]), i))
        for i in ranked[room:]:
            code[i] = KEEP
    keys = ("mean", "log_scale", "quat", "density")
    P = {k: np.asarray(gs[k], dtype=np.float64) for k in keys}
    Mi = {k: np.asarray(m[k], dtype=np.float64) for k in keys}
    Vi = {k: np.asarray(v[k], dtype=np.float64) for k in keys}
    z = np.asarray(normals, dtype=np.float64)
    R = rotation(P["quat"])
    cols = {k: [] for k in keys}
    mcols = {k: [] for k in keys}
    vcols = {k: [] for k in keys}

    def put(mean, ls, q, rho, mom_of):
        for k, val in zip(keys, (mean, ls, q, rho)):
            cols[k].append(val)
        for k in keys:
            mcols[k].append(Mi[k][..., mom_of])
            vcols[k].append(Vi[k][..., mom_of])

    for i in range(n):
        c = code[i]
        mean, ls, q, rho = P["mean"][:, i], P["log_scale"][:, i], P["quat"][:, i], P["density"][i]
        if c == PRUNE:
            continue
        if c == KEEP:
            put(mean, ls, q, rho, i)
        elif c == CLONE:
            put(mean, ls, q, 0.5 * rho, i)
            put(mean, ls, q, 0.5 * rho, i)
        else:
            s = np.exp(ls)
            for child in range(2):
                put(mean + R[:, :, i] @ (s * z[3 * child:3 * child + 3, i]), ls - math.log(split_shrink), q,
                    rho * split_shrink ** 3 / 2.0, i)

    def pack(c):
        out = {}
        for k in keys:
            arr = np.array(c[k])
            out[k] = arr if k == "density" else arr.T.copy()
        return out
    return pack(cols), pack(mcols), pack(vcols), code


def mass(gs: dict) -> float:
    """Total mass sum rho (2 pi)^(3/2) s1 s2 s3 of the Gaussians."""
    ls = np.asarray(gs["log_scale"], dtype=np.float64)
    return float(np.sum(np.asarray(gs["density"], dtype=np.float64) * (2 * math.pi) ** 1.5 * np.exp(ls.sum(0))))
