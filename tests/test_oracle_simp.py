"""Pins of the SIMP oracle (App. F.3): closed forms (uniform solid, two-density
laminates by Backus averaging), scaling of a binary cell, finite differences of C_H
for the analytic sensitivities and of J for the objective gradient, a brute-force
loop for the filter, and the constraint / move limits of the OC step."""

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet
from oracle import fem, simp
from oracle import solve as osolve


def _solve(P):
    return osolve.pcg(P, tol=1e-12)[0]


def test_uniform_density_is_scaled_solid():
    rho = np.full((8, 8, 8), 0.7)
    P = simp.DensityProblem(rho, 2, p=3.0, rho_min=1e-3)
    u = _solve(P)
    s = 1e-3 + 0.7 ** 3
    assert np.abs(u).max() < 1e-10
    C0 = fem.isotropic_C(1.0, 0.3)
    assert np.allclose(simp.homogenize(P, u), s * C0, rtol=0, atol=1e-12)


def test_binary_field_scales_the_binary_problem():
    vox = gyroid_sheet(8, 3, 0.4)
    rho = np.where(vox > 0, 1.0, 1e-9)
    P = simp.DensityProblem(rho, 2, p=3.0, rho_min=0.02, prune=1e-6)
    Q = osolve.Problem(vox, 2)
    u, ub = _solve(P), _solve(Q)
    # every active element has s = rho_min + 1: the same u, C_H scaled
    assert np.abs(osolve.gauge_shift(P, u) - osolve.gauge_shift(Q, ub)).max() < 1e-9
    assert np.allclose(simp.homogenize(P, u), 1.02 * osolve.homogenize(Q, ub), rtol=0, atol=1e-10)


def _backus(E, nu, frac):
    """Effective 6x6 (Voigt order 11,22,33,23,13,12) of isotropic layers normal to z."""
    E = np.asarray(E, float)
    frac = np.asarray(frac, float)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    M = lam + 2 * G
    avg = lambda x: float((frac * x).sum())  # noqa: E731
    C = np.zeros((6, 6))
    C33 = 1.0 / avg(1 / M)
    C13 = avg(lam / M) * C33
    C[2, 2] = C33
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[0, 0] = C[1, 1] = avg(M - lam ** 2 / M) + avg(lam / M) ** 2 * C33
    C[0, 1] = C[1, 0] = avg(lam - lam ** 2 / M) + avg(lam / M) ** 2 * C33
    C[3, 3] = C[4, 4] = 1.0 / avg(1 / G)
    C[5, 5] = avg(G)
    return C


@pytest.mark.parametrize("rho2", [0.3, 0.8])
def test_two_density_laminate_matches_backus(rho2):
    N = 8
    rho = np.ones((N, N, N))
    rho[5:, :, :] = rho2  # slabs normal to z (array index 0 is z)
    p, rmin = 3.0, 1e-3
    P = simp.DensityProblem(rho, 2, p=p, rho_min=rmin)
    u = _solve(P)
    s = np.array([rmin + 1.0, rmin + rho2 ** p])
    C = _backus(s, 0.3, [5 / 8, 3 / 8])
    assert np.allclose(simp.homogenize(P, u), C, rtol=0, atol=1e-9)


def test_sensitivities_match_finite_differences():
    rng = np.random.default_rng(0)
    N = 6
    rho = rng.uniform(0.2, 1.0, (N, N, N))
    P = simp.DensityProblem(rho, 2, p=3.0, rho_min=1e-3)
    u = osolve.direct_solve(P)
    dC = simp.sensitivities(P, u)
    h = 1e-6
    for e in (0, 17, 131, N ** 3 - 1):
        r1, r2 = rho.copy(), rho.copy()
        r1.ravel()[e] += h
        r2.ravel()[e] -= h
        Ps, Pm = simp.DensityProblem(r1, 2, p=3.0, rho_min=1e-3), simp.DensityProblem(r2, 2, p=3.0, rho_min=1e-3)
        fd = (simp.homogenize(Ps, osolve.direct_solve(Ps)) - simp.homogenize(Pm, osolve.direct_solve(Pm))) / (2 * h)
        assert np.abs(fd - dC[e]).max() <= 1e-6 * np.abs(dC[e]).max() + 1e-12, e


@pytest.mark.parametrize("kind", simp.OBJECTIVES)
def test_objective_gradient_finite_differences(kind):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((6, 6))
    C = A @ A.T + 6 * np.eye(6)
    J, G = simp.objective(C, kind)
    h = 1e-6
    for i, j in ((0, 0), (1, 2), (3, 3), (5, 0), (2, 4)):
        Cp, Cm = C.copy(), C.copy()
        Cp[i, j] += h
        Cm[i, j] -= h
        fd = (simp.objective(Cp, kind)[0] - simp.objective(Cm, kind)[0]) / (2 * h)
        assert abs(fd - G[i, j]) <= 1e-7, (kind, i, j)
    S = np.linalg.inv(C)
    want = {"young": np.trace(S[:3, :3]) / 3, "shear": np.trace(S[3:, 3:]) / 3, "bulk": S[:3, :3].sum()}[kind]
    assert abs(J - want) < 1e-14


def test_filter_brute_force_and_constant_fields():
    rng = np.random.default_rng(2)
    N, rmin = 6, 1.8
    rho = rng.uniform(0.05, 1.0, (N, N, N))
    dc = -rng.uniform(0.0, 1.0, (N, N, N))
    out = simp.filter_sensitivity(rho, dc, rmin)
    # brute force over all element pairs with periodic distances
    idx = np.array(np.unravel_index(np.arange(N ** 3), (N, N, N))).T
    for e in (0, 7, 100, N ** 3 - 1):
        dd = np.abs(idx - idx[e])
        dd = np.minimum(dd, N - dd)
        H = np.maximum(0.0, rmin - np.sqrt((dd ** 2).sum(axis=1)))
        want = (H * rho.ravel() * dc.ravel()).sum() / (max(1e-3, rho.ravel()[e]) * H.sum())
        assert abs(out.ravel()[e] - want) < 1e-13
    ones = np.ones((N, N, N))
    assert np.allclose(simp.filter_sensitivity(ones, 3.0 * ones, rmin), 3.0)


def test_oc_update_meets_volume_and_move_limits():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.1, 0.9, (8, 8, 8))
    dc = -rng.uniform(0.01, 1.0, rho.shape)
    new, lam = simp.oc_update(rho, dc, volfrac=0.4, move=0.1, rho_lo=1e-3)
    assert abs(new.mean() - 0.4) < 1e-6
    assert (np.abs(new - rho) <= 0.1 + 1e-15).all()
    assert new.min() >= 1e-3 and new.max() <= 1.0
    # larger (more negative) sensitivities never get smaller densities than smaller ones
    # from the same starting density
    flat = np.full(64, 0.5)
    d = -np.linspace(0.1, 1.0, 64)
    out, _ = simp.oc_update(flat, d, volfrac=0.5, move=0.3)
    assert (np.diff(out) >= -1e-15).all()
