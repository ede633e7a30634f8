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


# FP32 vs FP64 accumulation changes a BF16-rounded activation only where a sum lands within
# ~1e-7 relative of a rounding boundary; emulating FP32 sums in the oracle moves outputs and
# gradients by < 1e-6 relative at this size.  The bounds leave room for a few such flips.
FWD_TOL = 1e-3
BWD_TOL = 2e-3


def _make(CHs, L):
    vox = gyroid_sheet(16, 7, 0.4)
    H = _gmt().Hierarchy(vox, L)
    H.nn_setup(CHs)
    lv = ohier.build(vox, L)
    net = onn.UNet(CHs, 32, 18)
    g = onn.Graph(lv)
    assert H.n_params == net.n_params()
    flat = net.init(3)
    flat += 0.02 * np.random.default_rng(4).standard_normal(flat.size)  # nonzero biases
    print(f"[nn] channels={CHs} n_params={net.n_params()} n_n={[x.n_n for x in lv]}", flush=True)
    return vox, H, net, g, flat


@pytest.fixture(scope="module")
def setup():
    return _make(CH, 3)


@pytest.mark.parametrize("chs", [[16, 16, 16], [32, 32, 32], [16, 32, 64], [32, 64, 64]])
def test_forward_backward_channel_configs(chs):
    vox, H, net, g, flat = _make(chs, 3)
    outs = H.nn_forward(_t(flat))
    ref, cache = onn.forward(net, flat, g)
    ferr = [_rel(_np(o).reshape(r.shape), r) for o, r in zip(outs, ref)]
    rng = np.random.default_rng(9)
    gouts = [rng.standard_normal(r.shape) for r in ref]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    gref = onn.backward(net, g, cache, gouts)
    P, Gg = net.unflatten(gref), net.unflatten(_np(grad))
    berr = {name: _rel(Gg[name], P[name]) for name, _ in net.shapes()}
    print(f"[nn] {chs} forward errors {['%.2e' % e for e in ferr]}", flush=True)
    print("[nn] " + " ".join(f"{k}:{v:.1e}" for k, v in berr.items()), flush=True)
    H.close()
    assert max(ferr) <= FWD_TOL, ferr
    bad = {k: v for k, v in berr.items() if v > BWD_TOL}
    assert not bad, bad


def test_forward_matches_bf16_reference(setup):
    vox, H, net, g, flat = setup
    outs = H.nn_forward(_t(flat))
    ref, _ = onn.forward(net, flat, g)
    for l, (o, r) in enumerate(zip(outs, ref)):
        err = _rel(_np(o).reshape(r.shape), r)
        assert err <= FWD_TOL, (l, err)


def test_backward_matches_reference(setup):
    vox, H, net, g, flat = setup
    outs = H.nn_forward(_t(flat))
    ref, cache = onn.forward(net, flat, g)
    rng = np.random.default_rng(9)
    gouts = [rng.standard_normal(r.shape) for r in ref]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward([_t(x.reshape(o.shape)) for x, o in zip(gouts, outs)], grad)
    gref = onn.backward(net, g, cache, gouts)
    gg = _np(grad)
    P = net.unflatten(gref)
    Gg = net.unflatten(gg)
    errs = {name: _rel(Gg[name], P[name]) for name, _ in net.shapes()}
    print("[nn] " + " ".join(f"{k}:{v:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if v > BWD_TOL}
    assert not bad, bad
    assert _rel(gg, gref) <= BWD_TOL


def test_backward_accumulates(setup):
    vox, H, net, g, flat = setup
    outs = H.nn_forward(_t(flat))
    gouts = [torch.ones_like(o) for o in outs]
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    H.nn_backward(gouts, grad)
    once = grad.clone()
    H.nn_backward(gouts, grad)
    assert torch.allclose(grad, 2 * once, rtol=1e-5, atol=1e-6)


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
