"""GPU: the learned path end to end (network -> one Alg. 2 V-cycle -> FP64 check ->
warm-started GMG-PCG fallback), checked against the oracle, and what the trained
network gains over the method without it.

* Fallback parity (Sec. 4.5 followed by the plain solver): from the network's
  guess, from a zero guess, from a NaN guess and from a guess far worse than
  zero, gmt_solve must reach relative residual 1e-5 as the oracle evaluates it
  in FP64, with C_H within 1e-4 of the oracle's solve to 1e-11 -- elastic and
  thermal, 32^3 and 16^3 cells.
* Gain: on fixed held-out 128^3 cells, one V-cycle from the trained network's
  predictions leaves a smaller residual than one V-cycle from zero.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gmt_inputs import gyroid_sheet, spinodal, truss, workload_cell  # noqa: E402
from oracle import solve as osolve  # noqa: E402

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2604_26518_amd", "weights", "unet128_elastic.npz")

CASES = {
    "gyroid32": (lambda: gyroid_sheet(32, 3, 0.3), 4, "elastic"),
    "truss16": (lambda: truss(16, 5, 0.35), 3, "elastic"),
    "spinodal32_th": (lambda: spinodal(32, 7, 0.4), 4, "thermal"),
}


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", params=sorted(CASES))
def cell(request):
    from paper_2604_26518_amd import binding, learned
    make, L, phys = CASES[request.param]
    vox = make()
    print(f"[learned {request.param}] N={vox.shape[0]} L={L} {phys}", flush=True)
    P = osolve.Problem(vox, L, phys)
    u_ref, _ = osolve.pcg(P, tol=1e-11)
    CH_ref = osolve.homogenize(P, u_ref)
    H = binding.Hierarchy(vox, L, phys)
    H.nn_setup(learned.channels_for(L))
    params = learned.init_params(H.n_params, L, phys, seed=1)
    yield request.param, P, CH_ref, H, params
    H.close()


def _check(P, CH_ref, H, u, info):
    un = _np(u)
    res = float(np.max(osolve.relative_residual(P, un)))
    CH = H.homogenize(u)
    cerr = float(np.linalg.norm(CH - CH_ref) / np.linalg.norm(CH_ref))
    assert info["converged"], info
    assert res <= 1e-5, res
    assert cerr <= 1e-4, cerr
    assert np.abs(un[0]).max() == 0.0  # gauge node pinned in the returned solution
    return res, cerr


def test_learned_solve_matches_oracle(cell):
    from paper_2604_26518_amd import learned
    name, P, CH_ref, H, params = cell
    for inject in (True, False):
        u, info = learned.learned_solve(H, params, tol=1e-5, inject=inject)
        res, cerr = _check(P, CH_ref, H, u, info)
        print(f"[learned {name}] inject={inject}: after V-cycle {info['rel_after_vcycle']:.2e}, "
              f"its {info['iterations']}, residual {res:.1e}, dC_H {cerr:.1e}", flush=True)


@pytest.mark.parametrize("guess", ["zero", "nan", "inf", "huge", "random"])
def test_fallback_from_any_guess(cell, guess):
    name, P, CH_ref, H, params = cell
    f = H.load_vector()
    n = H.n_n(1)
    g = torch.Generator(device="cpu").manual_seed(3)
    u0 = {
        "zero": lambda: torch.zeros(n, H.c, H.d, dtype=torch.float64),
        "nan": lambda: torch.full((n, H.c, H.d), float("nan"), dtype=torch.float64),
        "inf": lambda: torch.randn(n, H.c, H.d, generator=g, dtype=torch.float64).index_fill_(
            0, torch.tensor([n // 2]), float("inf")),
        "huge": lambda: 1e6 * torch.randn(n, H.c, H.d, generator=g, dtype=torch.float64),
        "random": lambda: 0.05 * torch.randn(n, H.c, H.d, generator=g, dtype=torch.float64),
    }[guess]().to("cuda")
    for precision in ("f32", "f64"):
        u, rep = H.solve(f, u=u0.clone(), tol=1e-5, precision=precision, max_iter=3000)
        res, cerr = _check(P, CH_ref, H, u, rep)
        init = max(rep["rel_res_init"])
        print(f"[fallback {name}] {guess} {precision}: initial {init:.2e}, its {rep['iterations']}, "
              f"residual {res:.1e}, dC_H {cerr:.1e}", flush=True)
        if guess in ("nan", "inf"):
            assert not np.isfinite(init)
        if guess == "huge":
            assert init > 1.0


def test_network_beats_zero_init_on_held_out_cells():
    """What the trained network gains: one V-cycle from its predictions against one from zero
    on held-out 128^3 cells (seeds outside the training range), median over the cells."""
    from paper_2604_26518_amd import binding, learned
    params, info = learned.load_weights(WEIGHTS)
    L = info["levels"]
    ratios = []
    for seed in range(900100, 900108):
        fam, vf, vox = workload_cell(128, seed)
        H = binding.Hierarchy(vox, L, "elastic")
        H.nn_setup(info["channels"])
        f64 = H.load_vector()
        f32 = f64.to(torch.float32)
        rel = lambda u: float(np.max(H.relative_residual(f64, u.to(torch.float64))))  # noqa: E731
        u0 = torch.zeros_like(f32)
        H.vcycle(f32, u0)
        preds = H.nn_forward(params)
        u1 = preds[0].clone()
        H.vcycle(f32, u1, e_init=[None] + list(preds[1:]) + [None])
        r0, r1 = rel(u0), rel(u1)
        ratios.append(r1 / r0)
        print(f"[gain] seed {seed} {fam} VF {vf:.2f}: zero init {r0:.3f}, network {r1:.3f}", flush=True)
        H.close()
    med = float(np.median(ratios))
    print(f"[gain] median ratio network / zero init after one V-cycle: {med:.3f}", flush=True)
    assert med <= 0.85


def test_512_network_beats_zero_init_on_a_held_out_cell():
    """The 512^3 network (fine-tuned at 512^3 from the 128^3 one, on the 6 finest of 8 levels)
    against a zero start on a held-out 512^3 workload cell: one V-cycle each."""
    from paper_2604_26518_amd import binding, learned
    params, info = learned.load_weights(os.path.join(ROOT, "paper_2604_26518_amd", "weights", "unet512_elastic.npz"))
    assert info["N"] == 512
    seed = info["held_out_seed0"]
    fam, vf, vox = workload_cell(512, seed)
    print(f"[gain512] seed {seed} {fam} VF {vf:.2f}: cell generated", flush=True)
    H = binding.Hierarchy(vox, binding.default_levels(512), "elastic")
    H.nn_setup(info["channels"])
    f64 = H.load_vector()
    f32 = f64.to(torch.float32)
    rel = lambda u: float(np.max(H.relative_residual(f64, u.to(torch.float64))))  # noqa: E731
    u0 = torch.zeros_like(f32)
    H.vcycle(f32, u0)
    r0 = rel(u0)
    del u0
    preds = H.nn_forward(params)
    u1 = preds[0].clone()
    H.vcycle(f32, u1, e_init=learned.injection(H, preds))
    r1 = rel(u1)
    H.close()
    print(f"[gain512] zero init {r0:.3f}, network {r1:.3f}, ratio {r1 / r0:.3f}", flush=True)
    assert r1 <= 0.85 * r0
