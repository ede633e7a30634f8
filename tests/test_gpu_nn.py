"""GPU parity of the learned initializer (BF16 network, V-cycle loss and its adjoint) against the oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gmt_inputs import gyroid_sheet, random_vectors  # noqa: E402
from oracle import hierarchy as ohier  # noqa: E402
from oracle import nn as onn  # noqa: E402
from oracle import solve as osolve  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"
CH = [16, 32, 64]


def _gmt():
    from paper_2604_26518_amd import binding
    return binding


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# Rounding every activation to BF16 makes the network's outputs depend on the exact
# FP32 summation order: a sum that lands next to a BF16 rounding boundary rounds the
# other way, the changed value moves the sums downstream, and with 27 * C inputs per
# output such one-ulp changes spread through the whole network.  Where activations
# change sign the leaky-ReLU derivative jumps by 10x, so element-wise gradient
# comparisons with the FP64-summed oracle carry a spread of several percent for
# generic weights (the oracle itself moves that much under 6e-8 relative noise added
# before each rounding).  The sharp tests therefore use sign-definite regimes
# (all pre-activations > 0, or all < 0) where the derivative pattern is fixed: there the
# oracle's own spread under that noise is <= 3e-5 on outputs and <= 7.4e-4 on
# gradients (16^3 gyroid, channels up to 64), and the bounds below sit above it.
FWD_TOL = 5e-4
BWD_TOL = 5e-3
CONFIGS = [[16, 16, 16], [32, 32, 32], [16, 32, 64], [32, 64, 64]]


def regime_params(net, seed, sign, wscale=0.12, bias=1.2):
    """Weights small against the biases so every pre-activation has the sign `sign`."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, sh in net.shapes():
        if name.startswith("b"):
            p[name] = sign * bias + 0.1 * rng.standard_normal(sh)
        elif name == "E":
            p[name] = sign * rng.uniform(0.5, 1.5, sh)
        else:
            fan = sh[0] * sh[1] if len(sh) == 3 else sh[0]
            p[name] = rng.uniform(-1, 1, sh) * np.sqrt(3.0 / fan) * wscale
    return net.flatten(p)


def _make(CHs, L, sign=0):
    vox = gyroid_sheet(16, 7, 0.4)
    H = _gmt().Hierarchy(vox, L)
    H.nn_setup(CHs)
    lv = ohier.build(vox, L)
    net = onn.UNet(CHs, 32, 18)
    g = onn.Graph(lv)
    assert H.n_params == net.n_params()
    if sign:
        flat = regime_params(net, 5, sign)
    else:
        flat = net.init(3)
        flat += 0.02 * np.random.default_rng(4).standard_normal(flat.size)  # nonzero biases
    print(f"[nn] channels={CHs} sign={sign} n_params={net.n_params()} n_n={[x.n_n for x in lv]}", flush=True)
    return vox, H, net, g, flat


def _activation_order(L):
    order = []
    for l in range(L):
        order += [("h", 0, l), ("a", 1, l)]
    for l in range(L - 2, -1, -1):
        order += [("t", 2, l), ("d", 3, l)]
    for l in range(L - 1):
        order += [("z1", 4, l), ("z2", 5, l)]
    return order


def _fwd_bwd(H, net, g, flat):
    outs = H.nn_forward(_t(flat))
    ref, cache = onn.forward(net, flat, g)
    rng = np.random.default_rng(9)
    # mean-free output gradients: the centring of the predictions is then the identity on
    # them, and no gradient is a difference of large nearly equal terms
    gouts = [onn.center(rng.standard_normal(r.shape)) for r in ref]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    acts = {(k, l): _np(H.nn_activation(l + 1, w)) for k, w, l in _activation_order(H.L)}
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    gref = onn.backward(net, g, cache, gouts)
    return outs, ref, cache, acts, _np(grad), gref


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("chs", CONFIGS)
def test_sign_definite_forward_backward(chs, sign):
    vox, H, net, g, flat = _make(chs, 3, sign)
    outs, ref, cache, acts, gg, gref = _fwd_bwd(H, net, g, flat)
    H.close()
    # the regime holds in the oracle: every stored activation has the intended sign
    for (k, l), _ in acts.items():
        assert np.all(sign * cache[k][l] > 0), (k, l)
    aerr = {f"{k}{l}": _rel(a, cache[k][l]) for (k, l), a in acts.items()}
    # a centred prediction is a small difference of nearly equal values in these regimes:
    # its error is measured against the size of the head output before centring
    W = cache["W"]
    unc = [g.N * (cache["z2"][l] @ W[f"W3_{l}"] + W[f"b3_{l}"]) for l in range(len(ref))]
    ferr = [np.linalg.norm(_np(o).reshape(r.shape) - r) / np.linalg.norm(u) for o, r, u in zip(outs, ref, unc)]
    P, Gg = net.unflatten(gref), net.unflatten(gg)
    # Centring the predictions makes some gradients vanish in exact arithmetic (in a
    # linear regime a bias only shifts a prediction by a constant); those are compared
    # on the scale of the whole gradient instead of their own (zero) norm.
    # In these linear regimes the head biases only shift a prediction by a constant, which
    # the centring removes: their exact gradient is zero and the GPU's is FP32 rounding of a
    # sum that cancels, checked against the scale of the whole gradient.  In the negative
    # regime the head activations round to one BF16 value at every node, the predictions are
    # identically zero and the head weights' gradients vanish as well.
    total = np.linalg.norm(gref)
    head_bias = {f"b{k}_{l}" for k in (1, 2, 3) for l in range(H.L - 1)}
    head_w = {f"W{k}_{l}" for k in (1, 2, 3) for l in range(H.L - 1)}
    berr = {}
    for name, shape in net.shapes():
        if sign < 0 and (name in head_w or name.startswith("b")):
            # negative regime: the predictions are identically zero, and the head and bias
            # gradients are sums that cancel to FP32 rounding; this regime checks the
            # 0.1-slope branch of the encoder / decoder weight gradients only
            continue
        if name in head_bias:
            assert np.linalg.norm(Gg[name]) <= 1e-4 * total + 2 * np.linalg.norm(P[name]), name
            continue
        floor = 1e-3 * total * np.sqrt(np.prod(shape) / gref.size)
        berr[name] = np.linalg.norm(Gg[name] - P[name]) / max(np.linalg.norm(P[name]), floor)
    print(f"[nn] {chs} sign {sign}: activations " + " ".join(f"{k}:{v:.1e}" for k, v in aerr.items()), flush=True)
    print(f"[nn]   outputs {['%.1e' % e for e in ferr]} grads " + " ".join(f"{k}:{v:.1e}" for k, v in berr.items()),
          flush=True)
    assert max(aerr.values()) <= FWD_TOL, aerr
    assert max(ferr) <= FWD_TOL, ferr
    bad = {k: v for k, v in berr.items() if v > BWD_TOL}
    assert not bad, bad


def test_generic_weights_within_rounding_spread():
    """Generic weights (sign changes): the GPU stays within the oracle's own rounding spread."""
    vox, H, net, g, flat = _make(CH, 3)
    outs, ref, cache, acts, gg, gref = _fwd_bwd(H, net, g, flat)
    H.close()
    rng = np.random.default_rng(9)
    gouts = [onn.center(rng.standard_normal(r.shape)) for r in ref]
    spread_f, spread_g = 0.0, 0.0
    for trial in range(2):
        nrng = np.random.default_rng(100 + trial)
        base = onn.bf16
        try:
            onn.bf16 = lambda x: base(np.asarray(x, dtype=np.float64) * (1 + 6e-8 * nrng.standard_normal(np.shape(x))))
            r2, c2 = onn.forward(net, flat, g)
            g2 = onn.backward(net, g, c2, gouts)
        finally:
            onn.bf16 = base
        spread_f = max(spread_f, max(_rel(a, b) for a, b in zip(r2, ref)))
        spread_g = max(spread_g, _rel(g2, gref))
    ferr = max(_rel(_np(o).reshape(r.shape), r) for o, r in zip(outs, ref))
    gerr = _rel(gg, gref)
    print(f"[nn] generic: outputs {ferr:.2e} (oracle spread {spread_f:.2e}), grads {gerr:.2e} "
          f"(oracle spread {spread_g:.2e})", flush=True)
    assert ferr <= 3 * spread_f + 1e-4
    assert gerr <= 3 * spread_g + 1e-3


@pytest.fixture(scope="module")
def setup():
    return _make(CH, 3, 1)


def test_backward_accumulates(setup):
    vox, H, net, g, flat = setup
    outs = H.nn_forward(_t(flat))
    gouts = [torch.ones_like(o) for o in outs]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward(gouts, grad)
    once = grad.clone()
    H.nn_backward(gouts, grad)
    assert torch.allclose(grad, 2 * once, rtol=1e-5, atol=1e-6)


def test_forward_and_gradients_deterministic():
    """Outputs and every gradient (weights, biases, embedding: fixed-order partial sums,
    no float atomics) are identical bit for bit over repeated runs on the same cell."""
    vox = gyroid_sheet(32, 3, 0.3)
    H = _gmt().Hierarchy(vox, 4)
    H.nn_setup([16, 32, 64, 64])
    from paper_2604_26518_amd.learned import init_params
    flat = init_params(H.n_params, 4, seed=2) + 0.01
    rng = np.random.default_rng(1)
    runs = []
    for _ in range(2):
        outs = H.nn_forward(flat)
        gouts = [_t(rng.standard_normal(tuple(o.shape))) for o in outs]
        rng = np.random.default_rng(1)
        grad = torch.zeros_like(flat)
        H.nn_backward(gouts, grad)
        runs.append(([o.clone() for o in outs], grad.clone()))
    (o1, g1), (o2, g2) = runs
    for a, b in zip(o1, o2):
        assert torch.equal(a, b)
    assert torch.equal(g1, g2)
    assert float(g1.abs().sum()) > 0
    H.close()


def test_vcycle_loss_matches_oracle_and_gradient(setup):
    vox, H, net, g, flat = setup
    P = osolve.Problem(vox, H.L)
    lam = [H.level_info(l)["lambda_max"] for l in range(1, H.L + 1)]
    lo = [x / 30 for x in lam]
    hi = [1.1 * x for x in lam]
    sm = {"kind": "chebyshev", "lo": lo, "hi": hi}
    n1, n2 = P.levels[0].n_n, P.levels[1].n_n
    uh = random_vectors(n1, 18, 11).reshape(n1, 6, 3) * 0.3
    eh = random_vectors(n2, 18, 12).reshape(n2, 6, 3) * 0.05
    lamg = 1e-6
    loss, rn, rel, u1, grads = H.vcycle_loss([_t(uh), _t(eh)], lam=lamg, want_u1=True, lo=lo, hi=hi)
    lref, u1ref = onn.physics_loss(P, uh, [None, eh, None], sm, 2, 2, lamg)
    assert abs(loss - lref) <= 1e-4 * max(1.0, abs(lref))
    assert _rel(_np(u1), u1ref) <= 1e-4
    # directional derivatives against central differences of the FP64 oracle loss
    rng = np.random.default_rng(13)
    for which in (0, 1):
        shape = (n1, 6, 3) if which == 0 else (n2, 6, 3)
        dvec = rng.standard_normal(shape)
        eps = 1e-4 * np.abs(uh if which == 0 else eh).max()

        def L_at(s):
            a = uh + s * dvec if which == 0 else uh
            b = eh + s * dvec if which == 1 else eh
            return onn.physics_loss(P, a, [None, b, None], sm, 2, 2, lamg)[0]

        fd = (L_at(eps) - L_at(-eps)) / (2 * eps)
        an = float((_np(grads[which]) * dvec).sum())
        assert abs(an - fd) <= 2e-3 * abs(fd) + 1e-9, (which, an, fd)


def test_supervised_loss_and_gradient(setup):
    """gmt_nn_supervised_loss against its definition in FP64: the target centred per column,
    loss = alpha |p - t_c|^2 / |t_c|^2, and the gradient added to what the buffer held."""
    vox, H, net, g, flat = setup
    p = H.nn_forward(_t(flat))[0]
    n = H.n_n(1)
    rng = np.random.default_rng(5)
    t = _t(rng.standard_normal(tuple(p.shape)) + 3.0)
    grad = torch.full_like(p, 0.5)
    alpha = 0.7
    loss = H.nn_supervised_loss(p, t, alpha, grad=grad)
    P, T = _np(p).reshape(n, -1), _np(t).reshape(n, -1)
    Tc = T - T.mean(axis=0)
    ref = alpha * ((P - Tc) ** 2).sum() / (Tc ** 2).sum()
    gref = 0.5 + 2 * alpha * (P - Tc) / (Tc ** 2).sum()
    assert abs(loss - ref) <= 1e-12 * ref
    assert np.abs(_np(grad).reshape(n, -1) - gref).max() <= 2.0 ** -22 * np.abs(gref).max()
    assert H.nn_supervised_loss(p, t, alpha) == loss  # without a gradient buffer
    with pytest.raises(_gmt().GmtError):  # a target that is constant per column centres to zero
        H.nn_supervised_loss(p, torch.ones_like(p), alpha)


def test_adamw_step():
    B = _gmt()
    rng = np.random.default_rng(0)
    n = 1000
    p0, g, m0, v0 = (rng.standard_normal(n) for _ in range(4))
    v0 = np.abs(v0)
    p, gt, m, v = (_t(x) for x in (p0, g, m0, v0))
    lr, b1, b2, eps, wd, step, gs = 1e-3, 0.9, 0.999, 1e-8, 1e-2, 7, 0.5
    B.adamw(p, gt, m, v, lr, step, b1, b2, eps, wd, gs)
    gg = g * gs
    mr = b1 * m0 + (1 - b1) * gg
    vr = b2 * v0 + (1 - b2) * gg * gg
    pr = p0 * (1 - lr * wd) - lr * (mr / (1 - b1 ** step)) / (np.sqrt(vr / (1 - b2 ** step)) + eps)
    assert np.abs(_np(p) - pr).max() <= 1e-5 * np.abs(pr).max()
    assert np.abs(_np(m) - mr).max() <= 1e-6 and np.abs(_np(v) - vr).max() <= 1e-6


# ---------------------------------------------------------------------------- layer-local parity
# Every stored BF16 activation is checked element by element against the oracle's
# layer applied to the GPU's own (BF16, hence exact) layer inputs, so no rounding
# decision upstream can make the two sides diverge.  Bound per element, from the
# arithmetic: the GPU sums n FP32 terms (plus bias / skip adds and the slope
# multiply), so its pre-activation is within delta = (n + 3) 2^-24 S of the exact
# one, S the sum of the terms' magnitudes; the leaky ReLU is 1-Lipschitz; BF16
# round-to-nearest-even moves a value by at most 2^-8 of itself.  Hence
# |gpu - act(x)| <= 2^-8 (|act(x)| + delta) + delta.
U32 = 2.0 ** -24


def _act_bound(x, S, nterms):
    delta = (nterms + 3) * U32 * S
    return 2.0 ** -8 * (np.abs(onn.act(x)) + delta) + delta


def _check_layer(name, gpu, x, S, nterms):
    ref = onn.act(x)
    err = np.abs(gpu - ref)
    bound = _act_bound(x, S, nterms)
    worst = float((err / np.maximum(bound, 1e-300)).max())
    frac = float((gpu != onn.bf16(ref)).mean())
    print(f"[layer] {name}: max err / bound {worst:.3f}, elements off the exact rounding {frac:.1e}", flush=True)
    assert np.all(err <= bound), name


@pytest.mark.parametrize("chs", [[16, 32, 64], [32, 64, 64]])
def test_every_layer_element_wise(chs):
    vox, H, net, g, flat = _make(chs, 3)
    H.nn_forward(_t(flat))
    L = H.L
    W = {k: onn.bf16(v) for k, v in net.unflatten(flat).items()}
    A = {(k, l): _np(H.nn_activation(l + 1, w)) for k, w, l in _activation_order(L)}
    absW = {k: np.abs(v) for k, v in W.items()}
    # embedding: a table lookup, bit-exact
    assert np.array_equal(A[("h", 0)], onn.bf16(W["E"][g.occ8]))
    C = net.C
    for l in range(L):
        h = A[("h", l)]
        x = onn._conv(h, g.conv[l], W[f"We{l}"]) + W[f"be{l}"]
        S = onn._conv(np.abs(h), g.conv[l], absW[f"We{l}"]) + absW[f"be{l}"]
        _check_layer(f"a{l}", A[("a", l)], x, S, 27 * C[l])
        if l + 1 < L:
            a = A[("a", l)]
            x = onn._conv(a, g.pool[l], W[f"Wp{l}"]) + W[f"bp{l}"]
            S = onn._conv(np.abs(a), g.pool[l], absW[f"Wp{l}"]) + absW[f"bp{l}"]
            _check_layer(f"h{l + 1}", A[("h", l + 1)], x, S, 27 * C[l])
    for l in range(L - 2, -1, -1):
        dn = A[("a", L - 1)] if l + 1 == L - 1 else A[("d", l + 1)]
        n_l = g.levels[l].n_n
        up = onn._conv_T(dn, g.pool[l], np.transpose(W[f"Wu{l}"], (0, 2, 1)), n_l)
        Su = onn._conv_T(np.abs(dn), g.pool[l], np.transpose(absW[f"Wu{l}"], (0, 2, 1)), n_l)
        a = A[("a", l)]
        _check_layer(f"t{l}", A[("t", l)], up + W[f"bu{l}"] + a, Su + absW[f"bu{l}"] + np.abs(a), 27 * C[l + 1])
        t = A[("t", l)]
        x = onn._conv(t, g.conv[l], W[f"Wd{l}"]) + W[f"bd{l}"]
        S = onn._conv(np.abs(t), g.conv[l], absW[f"Wd{l}"]) + absW[f"bd{l}"]
        _check_layer(f"d{l}", A[("d", l)], x, S, 27 * C[l])
        d = A[("d", l)]
        _check_layer(f"z1_{l}", A[("z1", l)], d @ W[f"W1_{l}"] + W[f"b1_{l}"],
                     np.abs(d) @ absW[f"W1_{l}"] + absW[f"b1_{l}"], C[l])
        z1 = A[("z1", l)]
        _check_layer(f"z2_{l}", A[("z2", l)], z1 @ W[f"W2_{l}"] + W[f"b2_{l}"],
                     np.abs(z1) @ absW[f"W2_{l}"] + absW[f"b2_{l}"], net.H)
    # predictions: FP32 head sums scaled by N, centred with FP64 column means
    outs = H.nn_forward(_t(flat))
    for l in range(L - 1):
        z2 = A[("z2", l)]
        raw = g.N * (z2 @ W[f"W3_{l}"] + W[f"b3_{l}"])
        S3 = g.N * (np.abs(z2) @ absW[f"W3_{l}"] + absW[f"b3_{l}"])
        ref = onn.center(raw)
        delta = (net.H + 3) * U32 * S3
        bound = 2 * delta.max(axis=0, keepdims=True) + delta + 2 * U32 * np.abs(ref)
        err = np.abs(_np(outs[l]).reshape(ref.shape) - ref)
        print(f"[layer] out{l}: max err / bound {(err / bound).max():.3f}", flush=True)
        assert np.all(err <= bound), l
    H.close()


@pytest.mark.parametrize("chs", [[16, 32, 64], [32, 64, 64]])
def test_backward_element_wise_on_gpu_activations(chs):
    """Gradients against the oracle's backward run on the GPU's own stored activations (so the
    leaky-ReLU derivative pattern is the same on both sides), element by element: every entry
    of a parameter tensor within 1e-3 of that tensor's largest entry.  The GPU gradient is a
    chain of FP32 sums (per layer up to 27 x 64 terms in the data gradients and a few thousand
    node products in the weight gradients, over up to ten layers), each adding relative
    rounding of about sqrt(terms) 2^-24 = 3e-6 of its partial sums; the bound leaves more than
    ten times that over the whole chain.  Tensors whose exact gradient vanishes (the head's last
    biases, which the centring removes) are held to 1e-3 of the whole gradient's largest entry.
    (A bound from the magnitudes of all products is valid but vacuous here: through ten layers
    of 27 x C terms the magnitudes exceed the cancelling sums by 1e4 to 1e7.)"""
    vox, H, net, g, flat = _make(chs, 3)
    outs = H.nn_forward(_t(flat))
    L = H.L
    W = {k: onn.bf16(v) for k, v in net.unflatten(flat).items()}
    A = {(k, l): _np(H.nn_activation(l + 1, w)) for k, w, l in _activation_order(L)}
    cache = {"W": W,
             "h": [A[("h", l)] for l in range(L)], "a": [A[("a", l)] for l in range(L)],
             "t": [A[("t", l)] for l in range(L - 1)] + [None],
             "d": [A[("d", l)] for l in range(L - 1)] + [A[("a", L - 1)]],
             "z1": [A[("z1", l)] for l in range(L - 1)], "z2": [A[("z2", l)] for l in range(L - 1)]}
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
    print(f"[grad] {chs}: " + " ".join(f"{k}:{v:.1e}" for k, v in worst.items()), flush=True)
    bad = {k: v for k, v in worst.items() if v > 1e-3}
    assert not bad, bad


def test_norm2_and_ema():
    B = _gmt()
    rng = np.random.default_rng(2)
    for n in (1, 255, 256 * 256 + 17, 3_000_001):
        x = rng.standard_normal(n).astype(np.float32)
        ref = float((x.astype(np.float64) ** 2).sum())
        got = B.norm2(_t(x))
        assert abs(got - ref) <= 1e-12 * ref, (n, got, ref)
    assert B.norm2(_t(np.zeros(1000, dtype=np.float32))) == 0.0
    n = 100_003
    e0 = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    e = _t(e0)
    for decay in (0.999, 0.5, 0.0):
        ref = np.float32(decay) * _np(e).astype(np.float32) + (np.float32(1) - np.float32(decay)) * x
        B.ema(e, _t(x), decay)
        assert np.abs(_np(e) - ref).max() <= 2 * 2.0 ** -24 * np.abs(ref).max()
    assert np.abs(_np(e) - x).max() == 0.0  # decay 0 copies x
