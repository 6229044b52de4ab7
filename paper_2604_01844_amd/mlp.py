"""Learned initializer network (bindings over libfactgs' BF16 matrix-core
kernels): 544 -> 128 -> 128 -> 32 (8 used), FP32 master weights updated by
the library's Adam, BF16 copies repacked after every step."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi as A
from . import ops

K_IN, HIDDEN, N_OUT = 544, 128, 32


def _i16(shape, device):
    return torch.empty(shape, dtype=torch.int16, device=device)


def pad_rows(n: int) -> int:
    return (n + 31) // 32 * 32


class InitMLP:
    """Weights are drawn by the caller (seeded NumPy arrays) and passed in."""

    def __init__(self, weights: dict, device="cuda"):
        self.device = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)
        self.w = [t(weights["w1"]), t(weights["w2"]), t(weights["w3"])]
        self.b = [t(weights["b1"]), t(weights["b2"]), t(weights["b3"])]
        shapes = [(HIDDEN, K_IN), (HIDDEN, HIDDEN), (N_OUT, HIDDEN)]
        self.wb = [_i16(s, self.device) for s in shapes]
        self.wbt = [_i16(s[::-1], self.device) for s in shapes]
        self.params = self.w + self.b
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.grads = [torch.empty_like(p) for p in self.params]
        self.step = 0
        self.ws = ops.Workspace(self.device, 1 << 20)
        self.pack()

    @staticmethod
    def init_weights(seed: int) -> dict:
        """He-normal weights, zero biases (density bias -2: softplus ~ 0.13)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        b3 = np.zeros(N_OUT)
        b3[0] = -2.0
        b3[4] = 1.0  # identity rotation
        return dict(w1=rng.normal(0, np.sqrt(2.0 / K_IN), (HIDDEN, K_IN)),
                    w2=rng.normal(0, np.sqrt(2.0 / HIDDEN), (HIDDEN, HIDDEN)),
                    w3=rng.normal(0, np.sqrt(1.0 / HIDDEN), (N_OUT, HIDDEN)) * 0.1,
                    b1=np.zeros(HIDDEN), b2=np.zeros(HIDDEN), b3=b3)

    def pack(self):
        L = A.lib()
        s = A.stream_ptr(self.device)
        for w, wb, wbt in zip(self.w, self.wb, self.wbt):
            A.check(L.fgs_mlp_pack(A.ptr(w), w.shape[0], w.shape[1], A.ptr(wb), A.ptr(wbt), s))

    def struct(self) -> A.fgs_mlp:
        return A.fgs_mlp(K_IN, HIDDEN, N_OUT, A.ptr(self.wb[0]), A.ptr(self.wbt[0]), A.ptr(self.wb[1]),
                         A.ptr(self.wbt[1]), A.ptr(self.wb[2]), A.ptr(self.wbt[2]), A.ptr(self.b[0]),
                         A.ptr(self.b[1]), A.ptr(self.b[2]))

    def features(self, vol, grid: ops.Grid, inv_norm: float, mean, transposed: bool = False, norm_max=None,
                 extra=None):
        """bf16 features [rows][544] (and [544][rows]) of the Gaussians at
        mean [3][n]; samples scaled by inv_norm / norm_max[0] (norm_max a
        device scalar, optional); extra [k][n] per-sample inputs (optional)."""
        n = mean.shape[1]
        rows = pad_rows(n)
        x = _i16((rows, K_IN), self.device)
        xt = _i16((K_IN, rows), self.device) if transposed else None
        gd = grid.struct()
        n_extra = 0 if extra is None else extra.shape[0]
        A.check(A.lib().fgs_gather_patches(A.ptr(vol), ctypes.byref(gd), float(inv_norm), A.ptr(norm_max),
                                           A.ptr(mean.contiguous()),
                                           A.ptr(None if extra is None else extra.contiguous()), n_extra, n,
                                           rows, A.ptr(x), A.ptr(xt), A.stream_ptr(self.device)))
        return x, xt, rows

    def forward(self, x, rows: int, keep_transposes: bool = False) -> dict:
        f32 = lambda c: torch.empty((rows, c), device=self.device)
        acts = dict(z1=f32(HIDDEN), z2=f32(HIDDEN), z3=f32(N_OUT), h1=_i16((rows, HIDDEN), self.device),
                    h2=_i16((rows, HIDDEN), self.device))
        acts["h1t"] = _i16((HIDDEN, rows), self.device) if keep_transposes else None
        acts["h2t"] = _i16((HIDDEN, rows), self.device) if keep_transposes else None
        s = A.fgs_mlp_acts(*(A.ptr(acts[k]) for k in ("z1", "z2", "z3", "h1", "h1t", "h2", "h2t")))
        net = self.struct()
        A.check(A.lib().fgs_mlp_fwd(ctypes.byref(net), A.ptr(x), rows, ctypes.byref(s), A.stream_ptr(self.device)))
        return acts

    def heads(self, acts: dict, n: int, target=None, base_log_scale=None):
        """Predicted [8][n]; with target [n][8] also (loss, dz3, dz3t).
        Log-scales are base_log_scale [n] (optional) plus the network's."""
        rows = acts["z3"].shape[0]
        out = torch.empty((8, n), device=self.device)
        base = A.ptr(None if base_log_scale is None else base_log_scale.contiguous())
        if target is None:
            A.check(A.lib().fgs_mlp_heads(A.ptr(acts["z3"]), rows, n, base, None, A.ptr(out), None, None, None,
                                          None, A.stream_ptr(self.device)))
            return out, None, None, None
        loss = torch.empty(1, device=self.device)
        dz3 = _i16((rows, N_OUT), self.device)
        dz3t = _i16((N_OUT, rows), self.device)
        self.ws.call(A.lib().fgs_mlp_heads, A.ptr(acts["z3"]), rows, n, base, A.ptr(target.contiguous()),
                     A.ptr(out), A.ptr(dz3), A.ptr(dz3t), A.ptr(loss))
        return out, loss, dz3, dz3t

    def backward(self, xt, rows: int, acts: dict, dz3, dz3t):
        s = A.fgs_mlp_acts(*(A.ptr(acts[k]) for k in ("z1", "z2", "z3", "h1", "h1t", "h2", "h2t")))
        g = A.fgs_mlp_grads(A.ptr(self.grads[0]), A.ptr(self.grads[3]), A.ptr(self.grads[1]), A.ptr(self.grads[4]),
                            A.ptr(self.grads[2]), A.ptr(self.grads[5]))
        net = self.struct()
        self.ws.call(A.lib().fgs_mlp_bwd, ctypes.byref(net), A.ptr(xt), rows, ctypes.byref(s), A.ptr(dz3),
                     A.ptr(dz3t), ctypes.byref(g))
        return dict(dw1=self.grads[0], dw2=self.grads[1], dw3=self.grads[2], db1=self.grads[3], db2=self.grads[4],
                    db3=self.grads[5])

    def adam(self, lr: float):
        self.step += 1
        for p, g, m, v in zip(self.params, self.grads, self.m, self.v):
            ops.adam_step(p, g, m, v, self.step, lr, eps=1e-8)
        self.pack()

    def train_step(self, vol, grid, inv_norm, mean, target, lr: float, norm_max=None, base_log_scale=None):
        """One Adam step on the batch of Gaussians at mean [3][n] with
        targets [n][8]; returns the batch loss (device scalar). With
        base_log_scale [n] the network sees it as an input and predicts
        log-scales relative to it."""
        n = mean.shape[1]
        extra = None if base_log_scale is None else base_log_scale.reshape(1, n)
        x, xt, rows = self.features(vol, grid, inv_norm, mean, transposed=True, norm_max=norm_max, extra=extra)
        acts = self.forward(x, rows, keep_transposes=True)
        _, loss, dz3, dz3t = self.heads(acts, n, target, base_log_scale)
        self.backward(xt, rows, acts, dz3, dz3t)
        self.adam(lr)
        return loss

    def predict(self, vol, grid, inv_norm, mean, norm_max=None, base_log_scale=None):
        """(density [n], log_scale [3][n], quat [4][n]) for Gaussians at mean."""
        n = mean.shape[1]
        extra = None if base_log_scale is None else base_log_scale.reshape(1, n)
        x, _, rows = self.features(vol, grid, inv_norm, mean, norm_max=norm_max, extra=extra)
        acts = self.forward(x, rows)
        out, *_ = self.heads(acts, n, None, base_log_scale)
        return out[0].contiguous(), out[1:4].contiguous(), out[4:8].contiguous()


def canonical_targets(mean, log_scale, quat, density):
    """[n][8] training targets (see fgs_canonical_targets)."""
    n = density.numel()
    out = torch.empty((n, 8), device=density.device)
    g = A.fgs_gaussians(n, A.ptr(mean), A.ptr(log_scale), A.ptr(quat), A.ptr(density))
    A.check(A.lib().fgs_canonical_targets(ctypes.byref(g), A.ptr(out), A.stream_ptr(density.device)))
    return out
