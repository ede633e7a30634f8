"""Serialized window attention with Ra-RoPE (Sec. 4.2-4.3), by definition, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Serialization (Sec. 4.2, homogenization-aware serialization): the active nodes
  of a level are ordered by the Morton (Z-order) code of their coordinates under
  one of three cyclic permutations -- view 0 (x, y, z), view 1 (y, z, x),
  view 2 (z, x, y) -- with bit b of the first, second and third coordinate at
  code bits 3b, 3b + 1, 3b + 2.  Consecutive runs of W tokens of that order
  are the attention windows (the last one partial).
* Ra-RoPE (Sec. 4.3, eq. rarope_theta): the channels of a head form pairs
  (2k, 2k + 1); pair k rotates by theta = 2 pi (m + 1) p_i / Upsilon_i with
  axis i = k mod 3 and harmonic m = k div 3 (reading: the paper splits the
  channels over the axes without fixing the split), p the node's coordinate on
  its level and Upsilon = N_l the level's period.  A shift by Upsilon changes
  theta by a multiple of 2 pi, so the encoding is exactly periodic.
* Attention per window and head: o_i = sum_j softmax_j(q~_i . k~_j / sqrt(dh)) v_j
  with q~, k~ the rotated queries and keys.

The block that uses it (``nn.UNet(..., attention=True)``):
  q = bf16(a Wq), k = bf16(a Wk), v = bf16(a Wv);  o = bf16(Attn(q, k, v));
  s = bf16(a + o Wo)
"""

from __future__ import annotations

import numpy as np

HEAD_DIM = 8


def window_size(level: int) -> int:
    """Attention window of a level (0-based): 256, 512, then 1024 tokens."""
    return min(256 << level, 1024)


def morton(coords: np.ndarray, view: int, bits: int = 11) -> np.ndarray:
    """Morton codes of integer coordinates [n, 3] (x, y, z) under cyclic view 0, 1 or 2."""
    c = np.asarray(coords, dtype=np.int64)
    perm = [(0, 1, 2), (1, 2, 0), (2, 0, 1)][view]
    code = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(bits):
        for slot, axis in enumerate(perm):
            code |= ((c[:, axis] >> b) & 1) << (3 * b + slot)
    return code


def serialize(lv, view: int) -> np.ndarray:
    """Node ids of a level in the serialization order of `view`."""
    N = lv.N
    lin = lv.node_lin
    coords = np.stack([lin % N, (lin // N) % N, lin // (N * N)], axis=1)
    return np.argsort(morton(coords, view), kind="stable")


def rope_angles(lv, heads: int) -> np.ndarray:
    """theta [n, heads, dh/2] of every node (identical for every head)."""
    N = lv.N
    lin = lv.node_lin
    p = np.stack([lin % N, (lin // N) % N, lin // (N * N)], axis=1).astype(np.float64)
    npair = HEAD_DIM // 2
    th = np.empty((lv.n_n, npair))
    for k in range(npair):
        axis, m = k % 3, k // 3
        th[:, k] = 2.0 * np.pi * (m + 1) * p[:, axis] / N
    return np.repeat(th[:, None, :], heads, axis=1)


def rotate(x: np.ndarray, theta: np.ndarray, sign: float = 1.0) -> np.ndarray:
    """Rotates the channel pairs of x [n, heads * dh] by sign * theta [n, heads, dh/2]."""
    n = x.shape[0]
    heads = theta.shape[1]
    xr = x.reshape(n, heads, HEAD_DIM // 2, 2)
    c, s = np.cos(theta), sign * np.sin(theta)
    out = np.empty_like(xr)
    out[..., 0] = c * xr[..., 0] - s * xr[..., 1]
    out[..., 1] = s * xr[..., 0] + c * xr[..., 1]
    return out.reshape(n, heads * HEAD_DIM)


def attention(q, k, v, order, W, theta):
    """Window attention of every head over the windows of `order`; returns (o, cache)."""
    n, C = q.shape
    heads = C // HEAD_DIM
    qt, kt = rotate(q, theta), rotate(k, theta)
    o = np.zeros((n, C))
    probs = []
    for w0 in range(0, n, W):
        ids = order[w0:w0 + W]
        for h in range(heads):
            sl = slice(h * HEAD_DIM, (h + 1) * HEAD_DIM)
            S = qt[ids, sl] @ kt[ids, sl].T / np.sqrt(HEAD_DIM)
            S -= S.max(axis=1, keepdims=True)
            P = np.exp(S)
            P /= P.sum(axis=1, keepdims=True)
            o[ids, sl] = P @ v[ids, sl]
            probs.append(P)
    return o, {"qt": qt, "kt": kt, "P": probs}


def attention_backward(go, q, k, v, order, W, theta, cache):
    """Gradients (gq, gk, gv) of sum <go, o> through the windows and the rotations."""
    n, C = q.shape
    heads = C // HEAD_DIM
    qt, kt = cache["qt"], cache["kt"]
    gqt, gkt, gv = np.zeros((n, C)), np.zeros((n, C)), np.zeros((n, C))
    it = iter(cache["P"])
    for w0 in range(0, n, W):
        ids = order[w0:w0 + W]
        for h in range(heads):
            sl = slice(h * HEAD_DIM, (h + 1) * HEAD_DIM)
            P = next(it)
            g = go[ids, sl]
            gv[ids, sl] += P.T @ g
            dP = g @ v[ids, sl].T
            dS = P * (dP - (P * dP).sum(axis=1, keepdims=True)) / np.sqrt(HEAD_DIM)
            gqt[ids, sl] += dS @ kt[ids, sl]
            gkt[ids, sl] += dS.T @ qt[ids, sl]
    # the rotation is orthogonal: its adjoint rotates back
    return rotate(gqt, theta, -1.0), rotate(gkt, theta, -1.0), gv
