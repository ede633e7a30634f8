"""Pins of the serialized window attention with Ra-RoPE (Sec. 4.2-4.3) and of the U-Net with
attention blocks: a worked Morton order, exact periodicity of the rotary encoding, scores that
depend only on the periodic coordinate difference, window locality, and the whole network's
backward against central finite differences."""

import numpy as np

from gmt_inputs import gyroid_sheet
from oracle import attention as att
from oracle import hierarchy, nn


def test_morton_order_worked_example():
    # the 8 corners of a 2x2x2 block: view 0 orders by x + 2y + 4z, view 1 (y, z, x) by
    # y + 2z + 4x, view 2 (z, x, y) by z + 2x + 4y
    c = np.array([(x, y, z) for z in range(2) for y in range(2) for x in range(2)])
    assert list(att.morton(c, 0)) == [0, 1, 2, 3, 4, 5, 6, 7]
    assert list(att.morton(c, 1)) == [0, 4, 1, 5, 2, 6, 3, 7]
    assert list(att.morton(c, 2)) == [0, 2, 4, 6, 1, 3, 5, 7]
    # a finer bit: (2, 0, 0) follows the whole first 2x2x2 octant
    assert att.morton(np.array([[2, 0, 0]]), 0)[0] == 8
    assert att.morton(np.array([[1, 1, 1]]), 0)[0] == 7


class _Lv:
    def __init__(self, lin, N):
        self.node_lin = np.asarray(lin)
        self.N = N
        self.n_n = len(lin)


def test_rope_is_exactly_periodic_and_relative():
    rng = np.random.default_rng(0)
    N, heads = 12, 2
    p = rng.integers(0, N, (50, 3))
    lin = p[:, 0] + N * (p[:, 1] + N * p[:, 2])
    th = att.rope_angles(_Lv(lin, N), heads)
    # a shift by one period changes every angle by a multiple of 2 pi: identical rotations
    th_shift = th.copy()
    for k in range(att.HEAD_DIM // 2):
        axis, m = k % 3, k // 3
        th_shift[:, :, k] += 2 * np.pi * (m + 1) * N / N
    x = rng.standard_normal((50, heads * att.HEAD_DIM))
    assert np.allclose(att.rotate(x, th), att.rotate(x, th_shift), atol=1e-12)
    # scores between a rotated query and key depend only on the coordinate difference mod N
    q = rng.standard_normal((1, heads * att.HEAD_DIM))
    k = rng.standard_normal((1, heads * att.HEAD_DIM))

    def score(pa, pb):
        la = np.array([pa[0] + N * (pa[1] + N * pa[2])])
        lb = np.array([pb[0] + N * (pb[1] + N * pb[2])])
        ta, tb = att.rope_angles(_Lv(la, N), heads), att.rope_angles(_Lv(lb, N), heads)
        return float((att.rotate(q, ta) * att.rotate(k, tb)).sum())

    for _ in range(10):
        pa, pb, t = rng.integers(0, N, 3), rng.integers(0, N, 3), rng.integers(0, N, 3)
        assert abs(score(pa, pb) - score((pa + t) % N, (pb + t) % N)) < 1e-10


def test_window_locality():
    vox = gyroid_sheet(16, 1, 0.35)
    lv = hierarchy.build(vox, 1)[0]
    rng = np.random.default_rng(1)
    n, C = lv.n_n, 16
    q, k, v = (rng.standard_normal((n, C)) for _ in range(3))
    order = att.serialize(lv, 1)
    th = att.rope_angles(lv, C // att.HEAD_DIM)
    W = 256
    o, _ = att.attention(q, k, v, order, W, th)
    j = order[300]  # a node of the second window
    v2 = v.copy()
    v2[j] += 1.0
    o2, _ = att.attention(q, k, v2, order, W, th)
    changed = np.nonzero(np.abs(o2 - o).max(axis=1) > 0)[0]
    assert set(changed) <= set(order[256:512]) and len(changed) > 0
    # every output row is a convex combination of the window's value rows
    win = order[:256]
    assert (o[win] <= v[win].max(axis=0) + 1e-12).all() and (o[win] >= v[win].min(axis=0) - 1e-12).all()


def test_attention_unet_backward_matches_finite_differences():
    vox = gyroid_sheet(8, 2, 0.45)
    levels = hierarchy.build(vox, 2)
    g = nn.Graph(levels)
    net = nn.UNet([8, 16], 8, 18, attention=True)
    rng = np.random.default_rng(3)
    flat = net.init(5) + 0.05 * rng.standard_normal(net.n_params())
    outs, cache = nn.forward(net, flat, g, emulate_bf16=False)
    gouts = [rng.standard_normal(o.shape) for o in outs]
    grad = nn.backward(net, g, cache, gouts)

    def loss(p):
        o, _ = nn.forward(net, p, g, emulate_bf16=False)
        return sum(float((a * b).sum()) for a, b in zip(o, gouts))

    names = [name for name, _ in net.shapes()]
    offs = np.cumsum([0] + [int(np.prod(sh)) for _, sh in net.shapes()])
    idx = list(rng.choice(net.n_params(), 30, replace=False))
    for name in ("Wq0", "Wk0", "Wv0", "Wo0", "Wq1", "Wk1", "Wo1", "We0", "Wp0"):
        k = names.index(name)
        idx += list(rng.integers(offs[k], offs[k + 1], 3))
    eps = 1e-6
    for kk in idx:
        e = np.zeros_like(flat)
        e[kk] = eps
        fd = (loss(flat + e) - loss(flat - e)) / (2 * eps)
        assert abs(fd - grad[kk]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (kk, fd, grad[kk])


def test_attention_off_keeps_the_layout():
    net0 = nn.UNet([8, 16, 16], 8, 18)
    net1 = nn.UNet([8, 16, 16], 8, 18, attention=True)
    s0, s1 = net0.shapes(), net1.shapes()
    assert s1[:len(s0)] == s0
    assert net1.n_params() - net0.n_params() == 4 * (64 + 256 + 256)
