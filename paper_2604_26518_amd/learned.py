"""Learned initializer: training loop and the learned solve path.

Sequencing only: the network forward/backward, the V-cycle, the physics loss
and its adjoint, AdamW and the solver all run in libgmt (gmt_nn_*,
gmt_vcycle_loss, gmt_vcycle, gmt_solve).

Learned solve (Alg. 2 + fallback): predictions u_hat^1, e_hat^l -> one V-cycle
-> FP64 residual check -> if above tol, warm-started GMG-PCG from the
V-cycle result (never a restart from zero).
"""

from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import binding as B

DEFAULT_CHANNELS = (16, 32, 64, 64, 64, 64, 64, 64)


def channels_for(levels: int):
    return list(DEFAULT_CHANNELS[:levels])


def init_params(n_params: int, levels: int, physics: str = "elastic", seed: int = 0, device="cuda",
                attention: bool = False):
    """He-style uniform initialisation with the oracle's parameter order (small last head layer and,
    with attention blocks, small output projections Wo, so every block starts near the identity)."""
    from math import sqrt
    q = 18 if physics == "elastic" else 3
    C = channels_for(levels)
    H = 32
    shapes = [("E", (256, C[0]))]
    for l in range(levels):
        shapes += [("We", (27, C[l], C[l])), ("b", (C[l],))]
    for l in range(levels - 1):
        shapes += [("Wp", (27, C[l], C[l + 1])), ("b", (C[l + 1],)), ("Wu", (27, C[l + 1], C[l])), ("b", (C[l],)),
                   ("Wd", (27, C[l], C[l])), ("b", (C[l],)), ("W1", (C[l], H)), ("b", (H,)), ("W2", (H, H)),
                   ("b", (H,)), ("W3", (H, q)), ("b", (q,))]
    if attention:
        for l in range(levels):
            shapes += [("Wq", (C[l], C[l])), ("Wk", (C[l], C[l])), ("Wv", (C[l], C[l])), ("Wo", (C[l], C[l]))]
    g = torch.Generator().manual_seed(seed)
    parts = []
    for name, sh in shapes:
        n = int(np.prod(sh))
        if name == "b":
            parts.append(torch.zeros(n))
            continue
        fan_in = 1 if name == "E" else (sh[0] * sh[1] if len(sh) == 3 else sh[0])
        bound = sqrt(3.0 / fan_in) * (0.1 if name in ("W3", "Wo") else 1.0)
        parts.append((torch.rand(n, generator=g) * 2 - 1) * bound)
    flat = torch.cat(parts)
    assert flat.numel() == n_params, (flat.numel(), n_params)
    return flat.to(device=device, dtype=torch.float32).contiguous()


class Trainer:
    """AdamW on FP32 master weights with a cosine schedule, global-norm clipping and an EMA copy."""

    def __init__(self, n_params, levels, physics="elastic", lr=1e-3, wd=1e-2, clip=1.0, ema=0.999, seed=0,
                 lam=0.0, device="cuda", warmup=300, attention=False):
        self.params = init_params(n_params, levels, physics, seed, device, attention)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.ema = self.params.clone()
        self.lr, self.wd, self.clip, self.ema_decay = lr, wd, clip, ema
        self.lam = lam
        self.warmup = warmup
        self.step = 0

    def save(self, path):
        torch.save({"params": self.params.cpu(), "m": self.m.cpu(), "v": self.v.cpu(), "ema": self.ema.cpu(),
                    "step": self.step}, path)

    def load(self, path):
        ck = torch.load(path, map_location="cpu", weights_only=True)
        for name in ("params", "m", "v", "ema"):
            getattr(self, name).copy_(ck[name].to(self.params.device))
        self.step = int(ck["step"])

    def lr_at(self, k, total):
        """Linear warm-up over the first `warmup` steps, then cosine decay to zero at `total`."""
        warmup = self.warmup
        w = min(1.0, (k + 1) / warmup) if warmup > 0 else 1.0
        return self.lr * w * 0.5 * (1 + math.cos(math.pi * min(k, total) / max(total, 1)))

    def train_cell(self, H: B.Hierarchy, total_steps: int, inject: bool = True, target=None, alpha=0.0):
        """One optimisation step on one cell; returns (loss, ||r||, max relative residual).
        With a target (the plain solver's FP32 solution) and alpha > 0 the loss adds the
        supervised term alpha |u_hat^1 - target_c|^2 / |target_c|^2."""
        preds = H.nn_forward(self.params)
        if not inject:
            preds = preds[:1]
        lr = self.lr_at(self.step, total_steps)
        # gauge penalty lambda (sum_i u_i)^2 with lambda = lam / n^2: lam times the squared
        # per-component mean of u^1 (the residual does not see rigid translations)
        loss, rn, rel, _, grads = H.vcycle_loss(preds, lam=self.lam / float(H.n_n(1)) ** 2)
        if target is not None and alpha > 0:
            loss += H.nn_supervised_loss(preds[0], target, alpha, grad=grads[0])
        self.grad.zero_()  # memory fill
        H.nn_backward(grads, self.grad)
        gn = math.sqrt(B.norm2(self.grad))
        scale = min(1.0, self.clip / gn) if gn > 0 and math.isfinite(gn) else 0.0
        self.step += 1
        B.adamw(self.params, self.grad, self.m, self.v, lr, self.step, wd=self.wd, grad_scale=scale)
        B.ema(self.ema, self.params, self.ema_decay)
        return loss, rn, float(np.max(rel))


def save_weights(path, flat, levels, N, physics, meta=None, attention=False):
    """Inference weights: the BF16 rounding of `flat` (the network only ever uses BF16 weights)."""
    x = flat.detach().to("cpu", torch.float32).contiguous()
    bits = x.view(torch.int32).numpy().astype(np.uint32)
    bf = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)
    info = {"levels": int(levels), "N": int(N), "physics": physics, "channels": channels_for(levels), "head": 32,
            "attention": bool(attention)}
    if meta:
        info.update(meta)
    np.savez(path, bf16=bf, info=np.frombuffer(json.dumps(info).encode(), dtype=np.uint8))


def load_weights(path, device="cuda"):
    """(flat FP32 tensor holding BF16 values, info dict) from save_weights' file."""
    with np.load(path, allow_pickle=False) as z:
        bf = z["bf16"].astype(np.uint32) << 16
        info = json.loads(bytes(z["info"]).decode())
    flat = torch.from_numpy(bf.view(np.float32).copy()).to(device)
    return flat, info


def injection(H: B.Hierarchy, preds, inject=True):
    """The e_init list of a cycle (one entry per hierarchy level) from the network's predictions
    [u_hat^1, e_hat^2, ..., e_hat^{L'-1}]: no entry for level 1 (u_hat^1 is the iterate) nor for
    the levels at and below the network's coarsest, L' (there the cycle starts from zero)."""
    e = [None] * H.L
    if inject:
        for l, p in enumerate(preds[1:], start=2):
            e[l - 1] = p
    return e


def learned_solve(H: B.Hierarchy, params, tol=1e-5, inject=True, max_iter=3000, f64=None):
    """u_hat -> one Alg. 2 V-cycle -> FP64 check -> warm GMG-PCG fallback. Returns (u, info)."""
    f64 = H.load_vector() if f64 is None else f64
    f32 = f64.to(torch.float32)
    preds = H.nn_forward(params)
    u = preds[0]
    H.vcycle(f32, u, e_init=injection(H, preds, inject))
    u64 = u.to(torch.float64)
    u64, rep = H.solve(f64, u=u64, tol=tol, precision="f32", max_iter=max_iter)
    return u64, {"rel_after_vcycle": max(rep["rel_res_init"]), "iterations": rep["iterations"],
                 "converged": rep["converged"], "fallback": rep["iterations"] > 0}


def timed(fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t
