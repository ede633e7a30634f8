"""FP64 reference of the learned initializer: a sparse 3D conv U-Net on the GMG hierarchy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network follows the structure of Sec. 4.2-4.4 with convolutions in place of
the serialized attention: it runs on the active node sets P_1..P_L of the
solver hierarchy, embeds the 8-bit occupancy of each fine node (Sec. 4.2,
network input), pools with a learned 27-tap map from the fine nodes 2x + k
(k in {-1,0,1}^3) to the coarse node x (GMG-aware pooling, Sec. 4.2.2),
unpools along the same connectivity, and attaches a three-layer head zeta_l to
the decoder at every level but the coarsest: level 1 predicts u_hat^1 and
level l > 1 the correction e_hat^l (Sec. 4.4).  Neighbour maps wrap
periodically, which makes the network exactly periodic.

Precision emulation: every parameter (weights and biases) and every stored
activation are rounded to BF16 (round to nearest even) exactly where the GPU
stores BF16; sums are in FP64.

Definition (0-based level index l, channels C[l], head width H, q = c*d):
  h_0 = E[occ8]
  a_l = act(conv_l(h_l; We_l) + be_l)                       l = 0..L-1
  h_{l+1} = act(pool_l(a_l; Wp_l) + bp_l)                   l = 0..L-2
  d_{L-1} = a_{L-1}
  t_l = act(unpool_l(d_{l+1}; Wu_l) + bu_l + a_l)           l = L-2..0
  d_l = act(conv_l(t_l; Wd_l) + bd_l)
  z1 = act(d_l W1_l + b1_l); z2 = act(z1 W2_l + b2_l); out_l = center(scale * (z2 W3_l + b3_l))
with act = leaky ReLU (slope 0.1), conv_l(x)(i) = sum_j x(nb_j(i)) W[j] over the
27 periodic neighbours (absent nodes contribute 0), pool_l(x)(X) = sum_j
x(2X + o_j) W[j], unpool_l(y)(i) = sum over parents X with i = 2X + o_j of
y(X) W[j], and scale = N (displacements are measured in voxels).  center()
removes the mean over the level's nodes from every output column: the
periodic problem fixes displacements only up to a translation, and the
zero-mean gauge (Sec. 4.5) is imposed on every prediction exactly instead of
through the penalty alone.
"""

from __future__ import annotations

import numpy as np

SLOPE = 0.1


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def act(x):
    return np.where(x > 0, x, SLOPE * x)


def act_grad(y):
    """Derivative of the activation from its output (the sign is preserved)."""
    return np.where(y > 0, 1.0, SLOPE)


OFFS = np.array([(j % 3 - 1, (j // 3) % 3 - 1, j // 9 - 1) for j in range(27)], dtype=np.int64)


def _coords(lv):
    N = lv.N
    lin = lv.node_lin
    return lin % N, (lin // N) % N, lin // (N * N)


def conv_map(lv) -> np.ndarray:
    """[n_n, 27] ids of the periodic neighbours x + o_j on the same level (-1 if inactive)."""
    N = lv.N
    x, y, z = _coords(lv)
    out = np.empty((lv.n_n, 27), dtype=np.int64)
    for j, (ox, oy, oz) in enumerate(OFFS):
        out[:, j] = lv.node_id[(z + oz) % N, (y + oy) % N, (x + ox) % N]
    return out


def pool_map(fine, coarse) -> np.ndarray:
    """[n_coarse, 27] ids of the fine nodes 2X + o_j (-1 if inactive)."""
    Nf = fine.N
    X, Y, Z = _coords(coarse)
    out = np.empty((coarse.n_n, 27), dtype=np.int64)
    for j, (ox, oy, oz) in enumerate(OFFS):
        out[:, j] = fine.node_id[(2 * Z + oz) % Nf, (2 * Y + oy) % Nf, (2 * X + ox) % Nf]
    return out


class UNet:
    def __init__(self, channels, head: int, q: int, attention: bool = False):
        self.C = list(channels)
        self.L = len(channels)
        self.H = head
        self.q = q
        self.attention = attention

    def shapes(self):
        """Ordered (name, shape) of every parameter (the flat layout shared with the GPU)."""
        C, L, H, q = self.C, self.L, self.H, self.q
        s = [("E", (256, C[0]))]
        for l in range(L):
            s += [(f"We{l}", (27, C[l], C[l])), (f"be{l}", (C[l],))]
        for l in range(L - 1):
            s += [(f"Wp{l}", (27, C[l], C[l + 1])), (f"bp{l}", (C[l + 1],))]
            s += [(f"Wu{l}", (27, C[l + 1], C[l])), (f"bu{l}", (C[l],))]
            s += [(f"Wd{l}", (27, C[l], C[l])), (f"bd{l}", (C[l],))]
            s += [(f"W1_{l}", (C[l], H)), (f"b1_{l}", (H,)), (f"W2_{l}", (H, H)), (f"b2_{l}", (H,)),
                  (f"W3_{l}", (H, q)), (f"b3_{l}", (q,))]
        if self.attention:  # after every convolutional parameter: the layout without attention is unchanged
            for l in range(L):
                s += [(f"Wq{l}", (C[l], C[l])), (f"Wk{l}", (C[l], C[l])), (f"Wv{l}", (C[l], C[l])),
                      (f"Wo{l}", (C[l], C[l]))]
        return s

    def n_params(self):
        return int(sum(np.prod(sh) for _, sh in self.shapes()))

    def unflatten(self, flat):
        out = {}
        k = 0
        for name, sh in self.shapes():
            n = int(np.prod(sh))
            out[name] = np.asarray(flat[k:k + n], dtype=np.float64).reshape(sh)
            k += n
        return out

    def flatten(self, params):
        return np.concatenate([params[name].ravel() for name, _ in self.shapes()])

    def init(self, seed: int = 0):
        """He-style initialisation (uniform), seeded; final head layers scaled small."""
        rng = np.random.default_rng(seed)
        p = {}
        for name, sh in self.shapes():
            if name.startswith("b"):
                p[name] = np.zeros(sh)
                continue
            fan_in = sh[0] * sh[1] if len(sh) == 3 else sh[0]
            if name == "E":
                fan_in = 1
            bound = np.sqrt(3.0 / fan_in)
            if name.startswith("W3") or name.startswith("Wo"):
                bound *= 0.1
            p[name] = rng.uniform(-bound, bound, size=sh)
        return self.flatten(p)


def center(y):
    """Removes the mean over nodes of every output column (the zero-mean gauge of Sec. 4.5)."""
    return y - y.mean(axis=0, keepdims=True)


def _conv(x, nbmap, W):
    """sum_j x[nb_j] @ W[j] with absent neighbours contributing zero."""
    n = nbmap.shape[0]
    y = np.zeros((n, W.shape[2]))
    for j in range(27):
        idx = nbmap[:, j]
        m = idx >= 0
        y[m] += x[idx[m]] @ W[j]
    return y


def _conv_T(gy, nbmap, W, n_in):
    """Adjoint of _conv with respect to x."""
    gx = np.zeros((n_in, W.shape[1]))
    for j in range(27):
        idx = nbmap[:, j]
        m = idx >= 0
        np.add.at(gx, idx[m], gy[m] @ W[j].T)
    return gx


def _conv_W(x, nbmap, gy):
    """Gradient of _conv with respect to W."""
    gW = np.zeros((27, x.shape[1], gy.shape[1]))
    for j in range(27):
        idx = nbmap[:, j]
        m = idx >= 0
        gW[j] = x[idx[m]].T @ gy[m]
    return gW


class Graph:
    """Neighbour maps of one cell's hierarchy for the network (and, for the attention
    blocks, every level's serialization order -- view l mod 3 -- and Ra-RoPE angles)."""

    def __init__(self, levels):
        from . import attention as att
        self.levels = levels
        self.L = len(levels)
        self.conv = [conv_map(lv) for lv in levels]
        self.pool = [pool_map(levels[l], levels[l + 1]) for l in range(self.L - 1)]
        self.occ8 = levels[0].occ8.astype(np.int64)
        self.N = levels[0].N
        self.order = [att.serialize(lv, l % 3) for l, lv in enumerate(levels)]
        self.window = [att.window_size(l) for l in range(self.L)]
        self._theta = {}

    def theta(self, l, heads):
        from . import attention as att
        if (l, heads) not in self._theta:
            self._theta[(l, heads)] = att.rope_angles(self.levels[l], heads)
        return self._theta[(l, heads)]


def forward(net: UNet, flat, g: Graph, emulate_bf16: bool = True):
    """Returns (outputs list [u_hat^1, e_hat^2, ..., e_hat^{L-1}] as [n_l, q], cache)."""
    P = net.unflatten(flat)
    rb = bf16 if emulate_bf16 else (lambda v: v)
    W = {k: rb(v) for k, v in P.items()}  # every parameter is stored in BF16
    L = net.L
    cache = {"W": W}
    h = [None] * L
    a = [None] * L
    h[0] = rb(W["E"][g.occ8])
    s = [None] * L  # a_l after the attention block (a_l itself without attention)
    att_cache = [None] * L
    for l in range(L):
        a[l] = rb(act(_conv(h[l], g.conv[l], W[f"We{l}"]) + W[f"be{l}"]))
        if net.attention:
            from . import attention as att
            q = rb(a[l] @ W[f"Wq{l}"])
            k = rb(a[l] @ W[f"Wk{l}"])
            v = rb(a[l] @ W[f"Wv{l}"])
            th = g.theta(l, net.C[l] // att.HEAD_DIM)
            o_raw, ac = att.attention(q, k, v, g.order[l], g.window[l], th)
            o = rb(o_raw)
            s[l] = rb(a[l] + o @ W[f"Wo{l}"])
            att_cache[l] = dict(q=q, k=k, v=v, o=o, theta=th, cache=ac)
        else:
            s[l] = a[l]
        if l < L - 1:
            h[l + 1] = rb(act(_conv(s[l], g.pool[l], W[f"Wp{l}"]) + W[f"bp{l}"]))
    d = [None] * L
    t = [None] * L
    d[L - 1] = s[L - 1]
    for l in range(L - 2, -1, -1):
        up = _conv_T(d[l + 1], g.pool[l], np.transpose(W[f"Wu{l}"], (0, 2, 1)), g.levels[l].n_n)
        t[l] = rb(act(up + W[f"bu{l}"] + s[l]))
        d[l] = rb(act(_conv(t[l], g.conv[l], W[f"Wd{l}"]) + W[f"bd{l}"]))
    outs, z1s, z2s = [], [], []
    for l in range(L - 1):
        z1 = rb(act(d[l] @ W[f"W1_{l}"] + W[f"b1_{l}"]))
        z2 = rb(act(z1 @ W[f"W2_{l}"] + W[f"b2_{l}"]))
        outs.append(center(g.N * (z2 @ W[f"W3_{l}"] + W[f"b3_{l}"])))
        z1s.append(z1)
        z2s.append(z2)
    cache.update(h=h, a=a, s=s, d=d, t=t, z1=z1s, z2=z2s, att=att_cache)
    return outs, cache


def backward(net: UNet, g: Graph, cache, gouts):
    """Gradient of sum_l <gouts[l], outs[l]> with respect to the flat parameters."""
    W = cache["W"]
    h, a, d, t, z1s, z2s = (cache[k] for k in ("h", "a", "d", "t", "z1", "z2"))
    L = net.L
    G = {k: np.zeros_like(v) for k, v in W.items()}
    gd = [np.zeros_like(x) if x is not None else None for x in d]
    for l in range(L - 1):
        go = g.N * center(gouts[l])  # the centring is symmetric: its adjoint is itself
        G[f"W3_{l}"] += z2s[l].T @ go
        G[f"b3_{l}"] += go.sum(0)
        gz2 = (go @ W[f"W3_{l}"].T) * act_grad(z2s[l])
        G[f"W2_{l}"] += z1s[l].T @ gz2
        G[f"b2_{l}"] += gz2.sum(0)
        gz1 = (gz2 @ W[f"W2_{l}"].T) * act_grad(z1s[l])
        G[f"W1_{l}"] += d[l].T @ gz1
        G[f"b1_{l}"] += gz1.sum(0)
        gd[l] = gd[l] + gz1 @ W[f"W1_{l}"].T
    s_ = cache.get("s") or a
    gs = [np.zeros_like(x) for x in a]  # gradients of the attention blocks' outputs s_l
    for l in range(0, L - 1):
        gpre = gd[l] * act_grad(d[l])
        G[f"Wd{l}"] += _conv_W(t[l], g.conv[l], gpre)
        G[f"bd{l}"] += gpre.sum(0)
        gt = _conv_T(gpre, g.conv[l], W[f"Wd{l}"], g.levels[l].n_n)
        gpre_t = gt * act_grad(t[l])
        gs[l] += gpre_t
        G[f"bu{l}"] += gpre_t.sum(0)
        # up = unpool(d[l+1]; Wu) = _conv_T(d[l+1], pool, Wu^T)
        G[f"Wu{l}"] += np.transpose(_conv_W(gpre_t, g.pool[l], d[l + 1]), (0, 2, 1))
        gd[l + 1] = gd[l + 1] + _conv(gpre_t, g.pool[l], np.transpose(W[f"Wu{l}"], (0, 2, 1)))
    gs[L - 1] = gs[L - 1] + gd[L - 1]
    gh = [None] * L
    for l in range(L - 1, -1, -1):
        ga_l = gs[l].copy()  # residual branch of s = a + o Wo
        if net.attention:
            from . import attention as att
            ac = cache["att"][l]
            G[f"Wo{l}"] += ac["o"].T @ gs[l]
            go = gs[l] @ W[f"Wo{l}"].T
            gq, gk, gv = att.attention_backward(go, ac["q"], ac["k"], ac["v"], g.order[l], g.window[l],
                                                ac["theta"], ac["cache"])
            for name, gx in (("Wq", gq), ("Wk", gk), ("Wv", gv)):
                G[f"{name}{l}"] += a[l].T @ gx
                ga_l += gx @ W[f"{name}{l}"].T
        gpre = ga_l * act_grad(a[l])
        G[f"We{l}"] += _conv_W(h[l], g.conv[l], gpre)
        G[f"be{l}"] += gpre.sum(0)
        gh[l] = _conv_T(gpre, g.conv[l], W[f"We{l}"], g.levels[l].n_n)
        if l > 0:
            gpre_h = gh[l] * act_grad(h[l])
            G[f"Wp{l - 1}"] += _conv_W(s_[l - 1], g.pool[l - 1], gpre_h)
            G[f"bp{l - 1}"] += gpre_h.sum(0)
            gs[l - 1] += _conv_T(gpre_h, g.pool[l - 1], W[f"Wp{l - 1}"], g.levels[l - 1].n_n)
    np.add.at(G["E"], g.occ8, gh[0])
    return net.flatten(G)


def physics_loss(prob, u_hat, e_hat, sm, nu1=2, nu2=2, lam=0.0):
    """Loss of Sec. 4.5 after one V-cycle of Alg. 2 started from the predictions.

    L = log10(||f - K u^1||_2 + 1e-12) + lam * sum_{case,dof} (sum_i u^1_i)^2,
    u^1 = Vcycle(f; u_hat, e_hat) (norm over all cases and DOFs of the cell).
    Returns (L, u^1).
    """
    from .solve import vcycle

    u1 = vcycle(prob, prob.f, np.asarray(u_hat, dtype=np.float64), sm, nu1, nu2, e_init=e_hat)
    r = prob.f - prob.Kmul(0, u1)
    rn = float(np.sqrt((r ** 2).sum()))
    sums = u1.sum(axis=0)
    return np.log10(rn + 1e-12) + lam * float((sums ** 2).sum()), u1
