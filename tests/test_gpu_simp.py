"""GPU parity of SIMP inverse homogenization (App. F.3) against the oracle: the density
hierarchy's operators (K.u on every level, Galerkin matrices, diagonal, load), the
solve and C_H, the analytic sensitivities, the objective gradient, the filter and
the OC step -- all through the C ABI."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gmt_inputs import gyroid_sheet, random_vectors  # noqa: E402
from oracle import simp as osimp  # noqa: E402
from oracle import solve as osolve  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gmt():
    from paper_2604_26518_amd import binding
    return binding


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _density(N, seed, prune_some=False):
    """A smooth-ish random density in [0.05, 1] (plus a pruned near-void region when asked)."""
    rng = np.random.default_rng(seed)
    base = gyroid_sheet(N, seed, 0.5).astype(np.float64)
    rho = np.clip(0.3 + 0.6 * base + 0.1 * rng.standard_normal((N, N, N)), 0.05, 1.0)
    if prune_some:
        rho[: N // 4, : N // 4, : N // 4] = 1e-7  # below the pruning threshold
    return rho


CASES = {
    "rho16": dict(N=16, L=3, physics="elastic", prune=0.0, seed=1),
    "rho16_pruned": dict(N=16, L=3, physics="elastic", prune=1e-5, seed=2),
    "rho16_thermal": dict(N=16, L=3, physics="thermal", prune=0.0, seed=3),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    c = CASES[request.param]
    rho = _density(c["N"], c["seed"], prune_some=c["prune"] > 0)
    P = osimp.DensityProblem(rho, c["L"], p=3.0, rho_min=1e-3, prune=c["prune"], physics=c["physics"])
    H = _gmt().Hierarchy(None, c["L"], c["physics"], density=rho, p=3.0, rho_min=1e-3, prune=c["prune"])
    print(f"[simp] {request.param}: n_e={P.levels[0].n_e} n_n={P.levels[0].n_n}", flush=True)
    yield request.param, rho, P, H
    H.close()


def test_maps_and_load(pair):
    name, rho, P, H = pair
    for l in range(P.L):
        m = H.export_maps(l + 1)
        assert np.array_equal(_np(m["elem_lin"]).astype(np.int64), P.levels[l].elem_lin)
        assert np.array_equal(_np(m["node_lin"]).astype(np.int64), P.levels[l].node_lin)
    f = _np(H.load_vector())
    assert np.abs(f - P.f).max() <= 1e-13 * np.abs(P.f).max()


def test_operator_every_level(pair):
    name, rho, P, H = pair
    for l in range(P.L):
        n = P.levels[l].n_n
        u = random_vectors(n, P.c * P.d, 10 + l).reshape(n, P.c, P.d)
        ref = P.Kmul(l, u)
        for dt, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
            got = _np(H.apply_K(_t(u, dt), level=l + 1))
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"[simp] {name} level {l + 1} {dt}: {err:.2e}", flush=True)
            assert err <= tol, (l, dt, err)
        D = _np(H.export_diagonal(l + 1))
        assert np.abs(D - P.D[l]).max() <= 1e-13 * np.abs(P.D[l]).max()
        if l >= 1:
            K = _np(H.export_element_matrices(l + 1))
            assert np.abs(K - P.mats[l]).max() <= 1e-13 * np.abs(P.mats[l]).max()


def test_solve_and_homogenize(pair):
    name, rho, P, H = pair
    u_ref, _ = osolve.pcg(P, tol=1e-11)
    C_ref = osimp.homogenize(P, u_ref)
    f = H.load_vector()
    u, rep = H.solve(f, tol=1e-9, precision="f64", max_iter=2000)
    C = H.homogenize(u)
    err = np.linalg.norm(C - C_ref) / np.linalg.norm(C_ref)
    res = float(np.max(osolve.relative_residual(P, _np(u))))
    print(f"[simp] {name}: FP64 its {rep['iterations']} residual {res:.1e} dC_H {err:.1e}", flush=True)
    assert res <= 1e-9 and err <= 1e-8
    u32, rep32 = H.solve(f, tol=1e-5, precision="f32", max_iter=2000)
    res32 = float(np.max(osolve.relative_residual(P, _np(u32))))
    err32 = np.linalg.norm(H.homogenize(u32) - C_ref) / np.linalg.norm(C_ref)
    print(f"[simp] {name}: mixed its {rep32['iterations']} residual {res32:.1e} dC_H {err32:.1e}", flush=True)
    assert res32 <= 1e-5 and err32 <= 1e-4


def test_sensitivities(pair):
    name, rho, P, H = pair
    u_ref, _ = osolve.pcg(P, tol=1e-11)
    # the same u on both sides: sensitivities are a pure function of (rho, u)
    dC_ref = osimp.sensitivities(P, u_ref)
    G = np.random.default_rng(4).standard_normal((P.c, P.c))
    dJ, dC = H.simp_sensitivity(_t(u_ref), G=G, want_dC=True)
    dC = _np(dC)
    scale = np.abs(dC_ref).max()
    assert np.abs(dC - dC_ref).max() <= 1e-12 * scale
    dJ_ref = np.einsum("eij,ij->e", dC_ref, G)
    assert np.abs(_np(dJ) - dJ_ref).max() <= 1e-12 * np.abs(dJ_ref).max()
    off = np.ones(P.N ** 3, bool)
    off[P.levels[0].elem_lin] = False
    assert (dC[off] == 0).all()


@pytest.mark.parametrize("kind", ["young", "shear", "bulk"])
def test_objective(kind):
    B = _gmt()
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 6))
    C = A @ A.T + 6 * np.eye(6)
    J, G = B.simp_objective(C, kind)
    Jr, Gr = osimp.objective(C, kind)
    assert abs(J - Jr) <= 1e-13 * abs(Jr)
    assert np.abs(G - Gr).max() <= 1e-13 * np.abs(Gr).max()


@pytest.mark.parametrize("N,rmin", [(16, 1.5), (12, 2.6), (9, 3.2)])
def test_filter(N, rmin):
    B = _gmt()
    rng = np.random.default_rng(N)
    rho = rng.uniform(0.0005, 1.0, (N, N, N))
    dc = -rng.uniform(0.0, 1.0, (N, N, N))
    out = _np(B.simp_filter(_t(rho.ravel()), _t(dc.ravel()), rmin)).reshape(N, N, N)
    ref = osimp.filter_sensitivity(rho, dc, rmin)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


def test_oc_step():
    B = _gmt()
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.05, 0.95, 20 ** 3)
    dc = -rng.uniform(0.001, 1.0, rho.size)
    # mean 0.5 -> 0.42: reachable within the move limit 0.15
    new, lam = B.simp_oc(_t(rho), _t(dc), 0.42, move=0.15, eta=0.5, rho_lo=1e-3)
    ref, lam_ref = osimp.oc_update(rho, dc, 0.42, move=0.15, eta=0.5, rho_lo=1e-3)
    new = _np(new)
    assert abs(ref.mean() - 0.42) < 1e-8
    assert abs(new.mean() - 0.42) < 1e-8
    assert abs(lam - lam_ref) <= 1e-8 * lam_ref
    assert np.abs(new - ref).max() <= 1e-7
    assert (np.abs(new - rho) <= 0.15 + 1e-14).all()


def test_density_rejections():
    B = _gmt()
    rho = np.full((8, 8, 8), 0.5)
    with pytest.raises(B.GmtError):
        B.Hierarchy(None, 1, density=rho)  # a density hierarchy needs 2 levels
    with pytest.raises(B.GmtError):
        B.Hierarchy(None, 2, density=rho, p=0.5)
    H = B.Hierarchy(None, 2, density=rho)
    with pytest.raises(B.GmtError):
        H.nn_setup([16, 32])  # the network takes binary occupancy
    with pytest.raises(B.GmtError):
        H.export_element_matrices(1)
    H.close()
    Hb = B.Hierarchy(gyroid_sheet(8, 1, 0.4), 2)
    with pytest.raises(B.GmtError) as ei:
        Hb.simp_sensitivity(torch.zeros(Hb.n_n(1), 6, 3, dtype=torch.float64, device=DEV), G=np.eye(6))
    assert ei.value.status == B.GMT_E_STATE
    Hb.close()
