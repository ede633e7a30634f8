"""Pins of the oracle's network reference (learned initializer)."""

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet
from oracle import hierarchy, nn


def _net_graph(N=8, L=3, ch=(4, 5, 6), head=4, seed=0):
    vox = gyroid_sheet(N, seed, 0.45)
    lv = hierarchy.build(vox, L)
    net = nn.UNet(ch, head, 18)
    return net, nn.Graph(lv), vox


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.14159265, 0.0, 65504.0, 1e-40])
    r = nn.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: round to even (1.0)
    assert r[0] == 1.0 and r[1] == 1.0
    assert r[2] == 1.0078125  # above the tie
    assert r[3] == 1.0078125  # representable
    assert r[4] == -3.140625
    assert r[5] == 0.0 and r[6] == 65536.0


def test_parameter_count_and_layout():
    net = nn.UNet([16, 32, 64, 64, 64, 64], 32, 18)
    assert net.n_params() == sum(int(np.prod(s)) for _, s in net.shapes())
    flat = net.init(1)
    assert flat.size == net.n_params()
    assert np.array_equal(net.flatten(net.unflatten(flat)), flat)


def test_backward_matches_finite_differences():
    net, g, _ = _net_graph()
    rng = np.random.default_rng(3)
    flat = net.init(7) + 0.05 * rng.standard_normal(net.n_params())  # nonzero biases too
    outs, cache = nn.forward(net, flat, g, emulate_bf16=False)
    gouts = [rng.standard_normal(o.shape) for o in outs]
    grad = nn.backward(net, g, cache, gouts)

    def loss(p):
        o, _ = nn.forward(net, p, g, emulate_bf16=False)
        return sum(float((a * b).sum()) for a, b in zip(o, gouts))

    idx = rng.choice(net.n_params(), 60, replace=False)
    eps = 1e-6
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = eps
        fd = (loss(flat + e) - loss(flat - e)) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (k, fd, grad[k])


def test_periodic_translation_equivariance():
    # a shift by a multiple of 2^(L-1) voxels maps the hierarchy onto itself,
    # so the outputs are the same values attached to the shifted nodes
    net, g, vox = _net_graph(N=16, L=3, ch=(4, 4, 4))
    flat = net.init(2)
    outs, _ = nn.forward(net, flat, g)
    sh = (4, 8, 12)
    lv2 = hierarchy.build(np.roll(vox, shift=sh, axis=(0, 1, 2)), 3)
    outs2, _ = nn.forward(net, flat, nn.Graph(lv2))
    for l in range(len(outs)):
        lv, lvs = g.levels[l], lv2[l]
        s = [v // (2 ** l) for v in sh]
        N = lv.N
        x, y, z = lv.node_lin % N, (lv.node_lin // N) % N, lv.node_lin // (N * N)
        moved = ((x + s[2]) % N) + N * (((y + s[1]) % N) + N * ((z + s[0]) % N))
        pos = np.searchsorted(lvs.node_lin, moved)
        assert np.array_equal(lvs.node_lin[pos], moved)
        assert np.abs(outs2[l][pos] - outs[l]).max() <= 1e-12 * max(1.0, np.abs(outs[l]).max())


def test_unpool_is_adjoint_of_pool_connectivity():
    net, g, _ = _net_graph()
    rng = np.random.default_rng(0)
    W = rng.standard_normal((27, 3, 2))
    x = rng.standard_normal((g.levels[0].n_n, 3))
    y = rng.standard_normal((g.levels[1].n_n, 2))
    lhs = (nn._conv(x, g.pool[0], W) * y).sum()
    rhs = (x * nn._conv_T(y, g.pool[0], W, g.levels[0].n_n)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_predictions_are_zero_mean_and_bias_free():
    # every prediction is centred over its level's nodes (zero-mean gauge), so a
    # constant shift of the head's last bias changes nothing and gets no gradient
    net, g, _ = _net_graph()
    rng = np.random.default_rng(5)
    flat = net.init(3) + 0.05 * rng.standard_normal(net.n_params())
    outs, cache = nn.forward(net, flat, g, emulate_bf16=False)
    for o in outs:
        assert np.abs(o.mean(axis=0)).max() <= 1e-12 * max(1.0, np.abs(o).max())
    P = net.unflatten(flat)
    P["b3_0"] = P["b3_0"] + 0.7
    outs2, _ = nn.forward(net, net.flatten(P), g, emulate_bf16=False)
    assert np.abs(outs2[0] - outs[0]).max() <= 1e-12 * np.abs(outs[0]).max()
    grad = net.unflatten(nn.backward(net, g, cache, [rng.standard_normal(o.shape) for o in outs]))
    for l in range(len(outs)):
        assert np.abs(grad[f"b3_{l}"]).max() <= 1e-10
