"""GPU parity of the learned initializer's attention blocks (Sec. 4.2-4.3: Morton
serialization under cyclic views, windowed multi-head attention with Ra-RoPE) against
the oracle: the serialization exactly, every layer of the block element by element on
the GPU's own inputs within bounds derived from the arithmetic, the gradients on the
GPU's stored activations, the whole network in a sign-definite regime, and determinism."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gmt_inputs import gyroid_sheet  # noqa: E402
from oracle import attention as oatt  # noqa: E402
from oracle import hierarchy as ohier  # noqa: E402
from oracle import nn as onn  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"
U32 = 2.0 ** -24


def _gmt():
    from paper_2604_26518_amd import binding
    return binding


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _make(N, L, chs, seed=7, vf=0.4, params_seed=3, sign=0):
    vox = gyroid_sheet(N, seed, vf)
    H = _gmt().Hierarchy(vox, L)
    H.nn_setup(chs, attention=True)
    lv = ohier.build(vox, L)
    net = onn.UNet(chs, 32, 18, attention=True)
    g = onn.Graph(lv)
    assert H.n_params == net.n_params()
    if sign:
        from test_gpu_nn import regime_params
        flat = regime_params(net, 5, sign)
    else:
        flat = net.init(params_seed)
        flat += 0.02 * np.random.default_rng(params_seed + 1).standard_normal(flat.size)
    print(f"[att] N={N} L={L} channels={chs} sign={sign} n_params={net.n_params()} "
          f"n_n={[x.n_n for x in lv]} windows={[-(-x.n_n // oatt.window_size(l)) for l, x in enumerate(lv)]}",
          flush=True)
    return vox, H, net, g, flat


def _bf16_bound(x, S, nterms):
    """|bf16(fl(x)) - x| for an FP32 sum x of nterms products with absolute sum S."""
    delta = (nterms + 3) * U32 * S
    return 2.0 ** -8 * (np.abs(x) + delta) + delta


def _ser_to_node(x_ser, order):
    out = np.empty_like(x_ser)
    out[order] = x_ser
    return out


@pytest.mark.parametrize("N,L", [(16, 3), (24, 3), (32, 4)])
def test_serialization_matches_oracle(N, L):
    """Every level's order (view l mod 3) equals the oracle's Morton order exactly; N = 24
    has levels of 24, 12 and 6 nodes per side, none a power of two."""
    vox = gyroid_sheet(N, 5, 0.35)
    H = _gmt().Hierarchy(vox, L)
    H.nn_setup([16] + [32] * (L - 1), attention=True)
    lv = ohier.build(vox, L)
    for l in range(L):
        got = H.nn_serialization(l + 1).cpu().numpy()
        ref = oatt.serialize(lv[l], l % 3)
        print(f"[att] serialization N={N} level {l + 1}: {lv[l].n_n} nodes, view {l % 3}", flush=True)
        assert np.array_equal(got, ref), l
    H.close()


def test_serialization_requires_attention():
    vox = gyroid_sheet(16, 5, 0.35)
    H = _gmt().Hierarchy(vox, 3)
    H.nn_setup([16, 32, 64])
    with pytest.raises(_gmt().GmtError):
        H.nn_serialization(1)
    with pytest.raises(_gmt().GmtError):
        H.nn_activation(1, 7)
    H.close()


@pytest.mark.parametrize("N,L,chs", [(16, 3, [16, 32, 64]), (32, 4, [16, 32, 64, 64])])
def test_block_layers_element_wise(N, L, chs):
    """q, k, v, the attention output and the block output s of every level, each against
    the oracle evaluated on the GPU's own inputs of that layer.

    * q, k, v = bf16(a W): FP32 sums of C products, then BF16 rounding (bound as for the
      convolutions: (C + 3) u S_abs for the sum, 2^-8 relative for the rounding).
    * o (FP32, before rounding): scores are sums of 8 products of rotated values (each
      rotation two products with FP32 cos / sin of ~1 ulp), so every score carries an
      error of at most c u sum_d |q~_d k~_d| / sqrt 8 with c = 64 a generous constant;
      to first order a score error e moves o by at most 2 max|e| max|v|, and the sum
      over W keys adds at most (W + 16) u max|v|.
    * s = bf16(a + bf16(o) Wo): a sum of C + 1 terms, then BF16 rounding."""
    vox, H, net, g, flat = _make(N, L, chs)
    H.nn_forward(_t(flat))
    W = {k: onn.bf16(v) for k, v in net.unflatten(flat).items()}
    for l in range(L):
        C = chs[l]
        heads = C // oatt.HEAD_DIM
        order = H.nn_serialization(l + 1).cpu().numpy()
        a = _np(H.nn_activation(l + 1, 1))
        q, k, v = (_ser_to_node(_np(H.nn_activation(l + 1, w)), order) for w in (7, 8, 9))
        o32 = _ser_to_node(_np(H.nn_activation(l + 1, 10)), order)
        s = _np(H.nn_activation(l + 1, 6))
        for name, x, wn in (("q", q, "Wq"), ("k", k, "Wk"), ("v", v, "Wv")):
            ref = a @ W[f"{wn}{l}"]
            S = np.abs(a) @ np.abs(W[f"{wn}{l}"])
            err = np.abs(x - ref)
            bound = _bf16_bound(ref, S, C)
            print(f"[att] level {l + 1} {name}: max err / bound {(err / bound).max():.3f}", flush=True)
            assert np.all(err <= bound), (l, name)
        Wl = oatt.window_size(l)
        th = g.theta(l, heads)
        o_ref, cache = oatt.attention(q, k, v, g.order[l], Wl, th)
        # the score-error scale per query and head: max_j sum_d |q~_d k~_d| / sqrt 8
        qt, kt = np.abs(cache["qt"]), np.abs(cache["kt"])
        bound = np.zeros_like(o_ref)
        for w0 in range(0, q.shape[0], Wl):
            ids = g.order[l][w0:w0 + Wl]
            for hh in range(heads):
                sl = slice(8 * hh, 8 * hh + 8)
                smax = (qt[ids, sl] @ kt[ids, sl].T).max(axis=1) / np.sqrt(8)
                vmax = np.abs(v[ids, sl]).max()
                bound[ids, sl] = (2 * 64 * U32 * smax[:, None] + (len(ids) + 16) * U32) * vmax + 1e-30
        err = np.abs(o32 - o_ref)
        print(f"[att] level {l + 1} o ({q.shape[0]} tokens, window {Wl}): max err {err.max():.2e}, "
              f"max err / bound {(err / bound).max():.3f}", flush=True)
        assert np.all(err <= bound), l
        o16 = onn.bf16(o32)
        ref = a + o16 @ W[f"Wo{l}"]
        S = np.abs(a) + np.abs(o16) @ np.abs(W[f"Wo{l}"])
        err = np.abs(s - ref)
        bound = _bf16_bound(ref, S, C + 1)
        print(f"[att] level {l + 1} s: max err / bound {(err / bound).max():.3f}, "
              f"off the exact rounding {(s != onn.bf16(ref)).mean():.1e}", flush=True)
        assert np.all(err <= bound), l
    H.close()


def _gpu_cache(H, net, g, flat):
    """The oracle's forward cache rebuilt from the GPU's stored activations."""
    L = H.nn_levels
    W = {k: onn.bf16(v) for k, v in net.unflatten(flat).items()}
    act = lambda l, w: _np(H.nn_activation(l + 1, w))  # noqa: E731
    cache = {"W": W, "h": [act(l, 0) for l in range(L)], "a": [act(l, 1) for l in range(L)],
             "s": [act(l, 6) for l in range(L)],
             "t": [act(l, 2) for l in range(L - 1)] + [None],
             "z1": [act(l, 4) for l in range(L - 1)], "z2": [act(l, 5) for l in range(L - 1)]}
    cache["d"] = [act(l, 3) for l in range(L - 1)] + [cache["s"][L - 1]]
    if not H.nn_attention:
        return cache
    att = []
    for l in range(L):
        order = H.nn_serialization(l + 1).cpu().numpy()
        q, k, v = (_ser_to_node(act(l, w), order) for w in (7, 8, 9))
        o = onn.bf16(_ser_to_node(act(l, 10), order))
        th = g.theta(l, net.C[l] // oatt.HEAD_DIM)
        _, ac = oatt.attention(q, k, v, g.order[l], g.window[l], th)
        att.append(dict(q=q, k=k, v=v, o=o, theta=th, cache=ac))
    cache["att"] = att
    return cache


@pytest.mark.parametrize("N,L,chs", [(16, 3, [16, 32, 64]), (32, 4, [16, 32, 64, 64])])
def test_backward_element_wise_on_gpu_activations(N, L, chs):
    """Every parameter gradient (the attention projections included) against the oracle's
    backward run on the GPU's stored activations, each entry within 1e-3 of its tensor's
    largest entry (the bound of the convolutional network's test: chains of FP32 sums,
    here with the softmax backward's sums over the window added)."""
    vox, H, net, g, flat = _make(N, L, chs)
    outs = H.nn_forward(_t(flat))
    cache = _gpu_cache(H, net, g, flat)
    rng = np.random.default_rng(19)
    gouts = [rng.standard_normal((o.shape[0], 18)) for o in outs]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    H.close()
    gref = onn.backward(net, g, cache, gouts)
    Gg, Gr = net.unflatten(_np(grad)), net.unflatten(gref)
    total = np.abs(gref).max()
    worst = {}
    for name, _ in net.shapes():
        err = np.abs(Gg[name] - Gr[name]).max()
        if name.startswith("b3_"):
            assert err <= 1e-3 * total, name
            continue
        worst[name] = err / np.abs(Gr[name]).max()
    print(f"[att] grads {chs}: " + " ".join(f"{k}:{v:.1e}" for k, v in worst.items()), flush=True)
    for l in range(L):
        for p in ("Wq", "Wk", "Wv", "Wo"):
            assert np.abs(Gr[f"{p}{l}"]).max() > 0, (p, l)  # the block is exercised
    bad = {k: v for k, v in worst.items() if v > 1e-3}
    assert not bad, bad


def test_network_matches_oracle_sign_definite():
    """The whole network with attention blocks, GPU against the oracle's own forward and
    backward, in the positive regime of the convolutional network's tests (weights small
    against the biases, so every activation stays positive and the leaky-ReLU pattern is
    fixed on both sides); the same tolerances as there."""
    from test_gpu_nn import BWD_TOL, FWD_TOL
    chs = [16, 32, 64]
    vox, H, net, g, flat = _make(16, 3, chs, sign=1)
    outs = H.nn_forward(_t(flat))
    ref, cache = onn.forward(net, flat, g)
    rng = np.random.default_rng(9)
    gouts = [onn.center(rng.standard_normal(r.shape)) for r in ref]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    s_gpu = [_np(H.nn_activation(l + 1, 6)) for l in range(3)]
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    H.close()
    gref = onn.backward(net, g, cache, gouts)
    for l in range(3):
        assert np.all(cache["s"][l] > 0), l
        e = np.linalg.norm(s_gpu[l] - cache["s"][l]) / np.linalg.norm(cache["s"][l])
        print(f"[att] s{l}: rel err {e:.1e}", flush=True)
        assert e <= FWD_TOL, l
    W = cache["W"]
    unc = [g.N * (cache["z2"][l] @ W[f"W3_{l}"] + W[f"b3_{l}"]) for l in range(len(ref))]
    ferr = [np.linalg.norm(_np(o).reshape(r.shape) - r) / np.linalg.norm(u) for o, r, u in zip(outs, ref, unc)]
    print(f"[att] outputs {['%.1e' % e for e in ferr]}", flush=True)
    assert max(ferr) <= FWD_TOL
    P, Gg = net.unflatten(gref), net.unflatten(_np(grad))
    total = np.linalg.norm(gref)
    head_bias = {f"b{k}_{l}" for k in (1, 2, 3) for l in range(2)}
    berr = {}
    for name, shape in net.shapes():
        if name in head_bias:
            assert np.linalg.norm(Gg[name]) <= 1e-4 * total + 2 * np.linalg.norm(P[name]), name
            continue
        floor = 1e-3 * total * np.sqrt(np.prod(shape) / gref.size)
        berr[name] = np.linalg.norm(Gg[name] - P[name]) / max(np.linalg.norm(P[name]), floor)
    print("[att] grads " + " ".join(f"{k}:{v:.1e}" for k, v in berr.items()), flush=True)
    bad = {k: v for k, v in berr.items() if v > BWD_TOL}
    assert not bad, bad


def test_attention_deterministic():
    """Outputs and gradients with attention blocks are identical bit for bit over repeated
    runs (each thread sums its own outputs in a fixed order; no float atomics)."""
    vox = gyroid_sheet(32, 3, 0.3)
    H = _gmt().Hierarchy(vox, 4)
    H.nn_setup([16, 32, 64, 64], attention=True)
    net = onn.UNet([16, 32, 64, 64], 32, 18, attention=True)
    flat = _t(net.init(2))
    runs = []
    for _ in range(2):
        outs = H.nn_forward(flat)
        rng = np.random.default_rng(1)
        gouts = [_t(rng.standard_normal(tuple(o.shape))) for o in outs]
        grad = torch.zeros_like(flat)
        H.nn_backward(gouts, grad)
        runs.append(([o.clone() for o in outs], grad.clone()))
    (o1, g1), (o2, g2) = runs
    for a, b in zip(o1, o2):
        assert torch.equal(a, b)
    assert torch.equal(g1, g2)
    assert float(g1.abs().sum()) > 0
    H.close()


def test_attention_timing_keeps_the_outputs():
    """gmt_nn_time_attention relaunches a level's attention kernel on the stored q, k, v: it
    reports a positive duration and leaves the stored attention output bit for bit as it was."""
    vox, H, net, g, flat = _make(16, 3, [16, 32, 64])
    H.nn_forward(_t(flat))
    before = [H.nn_activation(l + 1, 10).clone() for l in range(3)]
    for l in range(3):
        assert H.nn_time_attention(l + 1, 3) > 0
    for l in range(3):
        assert torch.equal(H.nn_activation(l + 1, 10), before[l])
    H.nn_setup([16, 32, 64])
    with pytest.raises(_gmt().GmtError):
        H.nn_time_attention(1, 3)
    H.close()


@pytest.mark.parametrize("attention", [False, True])
def test_thermal_network_on_gpu_activations(attention):
    """The network of the thermal problem (3 outputs per node: the 3 load cases x 1 DOF),
    with and without attention blocks: the predictions against the oracle's head on the GPU's
    own last hidden layer (FP32 sum of H + 1 terms scaled by N, then centred), and every
    parameter gradient against the oracle's backward on the GPU's activations (each entry
    within 1e-3 of its tensor's largest entry, as for the elastic network)."""
    chs = [16, 32, 64]
    vox = gyroid_sheet(16, 7, 0.4)
    H = _gmt().Hierarchy(vox, 3, "thermal")
    H.nn_setup(chs, attention=attention)
    net = onn.UNet(chs, 32, 3, attention=attention)
    g = onn.Graph(ohier.build(vox, 3))
    assert H.n_params == net.n_params()
    flat = net.init(11) + 0.02 * np.random.default_rng(12).standard_normal(net.n_params())
    outs = H.nn_forward(_t(flat))
    cache = _gpu_cache(H, net, g, flat)
    W = cache["W"]
    for l, o in enumerate(outs):
        z2 = cache["z2"][l]
        raw = g.N * (z2 @ W[f"W3_{l}"] + W[f"b3_{l}"])
        ref = onn.center(raw)
        S3 = g.N * (np.abs(z2) @ np.abs(W[f"W3_{l}"]) + np.abs(W[f"b3_{l}"]))
        delta = (32 + 3) * U32 * S3
        bound = 2 * delta.max(axis=0, keepdims=True) + delta + 2 * U32 * np.abs(ref)
        err = np.abs(_np(o).reshape(ref.shape) - ref)
        print(f"[thermal att={attention}] out{l}: max err / bound {(err / bound).max():.3f}", flush=True)
        assert np.all(err <= bound), l
    rng = np.random.default_rng(23)
    gouts = [rng.standard_normal((o.shape[0], 3)) for o in outs]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    H.close()
    gref = onn.backward(net, g, cache, gouts)
    Gg, Gr = net.unflatten(_np(grad)), net.unflatten(gref)
    total = np.abs(gref).max()
    worst = {}
    for name, _ in net.shapes():
        err = np.abs(Gg[name] - Gr[name]).max()
        if name.startswith("b3_"):
            assert err <= 1e-3 * total, name
            continue
        worst[name] = err / np.abs(Gr[name]).max()
    print(f"[thermal att={attention}] grads: " + " ".join(f"{k}:{v:.1e}" for k, v in worst.items()), flush=True)
    bad = {k: v for k, v in worst.items() if v > 1e-3}
    assert not bad, bad
