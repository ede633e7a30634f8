"""Pins of the oracle's smoothers, V-cycle (Alg. 1 / Alg. 2) and reference solve."""

import numpy as np
import pytest
import scipy.linalg as sla

from gmt_inputs import gyroid_sheet, random_vectors
from oracle import operators as ops
from oracle import solve as S


def _rand_vox(N, seed, p=0.45):
    rng = np.random.default_rng(seed)
    return (rng.random((N, N, N)) < p).astype(np.uint8)


@pytest.fixture(scope="module")
def prob8():
    return S.Problem(gyroid_sheet(8, 4, 0.45), 3)


def test_jacobi_is_error_polynomial(prob8):
    P = prob8
    n = P.levels[0].n_n
    u0 = random_vectors(n, 18, 5).reshape(n, 6, 3)
    K = P.K[0].toarray()
    Dinv = 1.0 / P.D[0].ravel()
    f = np.zeros_like(u0)
    out = S.jacobi(P, 0, u0, f, 3, 0.6)
    M = np.eye(K.shape[0]) - 0.6 * Dinv[:, None] * K
    ref = ops.from_dofs(np.linalg.matrix_power(M, 3) @ ops.to_dofs(u0), 3)
    assert np.abs(out - ref).max() < 1e-12


@pytest.mark.parametrize("nu", [1, 2, 3, 4])
def test_chebyshev_polynomial_on_eigenvectors(prob8, nu):
    # error of an eigenvector v (D^-1 K v = lam v) is scaled by T_nu((theta-lam)/delta)/T_nu(theta/delta)
    P = prob8
    K = P.K[0].toarray()
    D = P.D[0].ravel()
    lam, V = sla.eigh(K, np.diag(D))
    lo, hi = 0.2 * lam[-1], 1.05 * lam[-1]
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    T = np.polynomial.chebyshev.Chebyshev.basis(nu)
    for j in [len(lam) // 3, len(lam) // 2, len(lam) - 1, 5]:
        v = V[:, j]
        u0 = np.zeros((P.levels[0].n_n, 6, 3))
        u0[:, 2, :] = v.reshape(-1, 3)
        out = S.chebyshev(P, 0, u0, np.zeros_like(u0), nu, lo, hi)
        scale = T((theta - lam[j]) / delta) / T(theta / delta)
        assert np.abs(out[:, 2, :].ravel() - scale * v).max() < 1e-10 * max(1.0, np.abs(v).max())
        assert np.abs(out[:, [0, 1, 3, 4, 5], :]).max() == 0.0


def test_vcycle_two_level_nu0_is_coarse_grid_correction():
    P = S.Problem(_rand_vox(8, 21), 2)
    n = P.levels[0].n_n
    u = random_vectors(n, 18, 1).reshape(n, 6, 3)
    f = P.f
    sm = {"kind": "jacobi", "omega": [0.5, 0.5]}
    out = S.vcycle(P, f, u, sm, nu1=0, nu2=0)
    # dense: u + P Kc_pinned^{-1} Z P^T (f - K u)
    K = P.K[0].toarray()
    Pm = P.P[0].toarray()
    Kc = Pm.T @ K @ Pm
    pin = np.arange(3)
    Kc[pin, :] = 0
    Kc[:, pin] = 0
    Kc[pin, pin] = 1.0
    r = Pm.T @ (ops.to_dofs(f) - K @ ops.to_dofs(u))
    r[pin] = 0.0
    ref = ops.to_dofs(u) + Pm @ np.linalg.solve(Kc, r)
    assert np.abs(ops.to_dofs(out) - ref).max() < 1e-11 * np.abs(ref).max()


def test_vcycle_dense_three_level_with_injection():
    """Alg. 2 composed from dense global matrices (P^T K P) vs the oracle's V-cycle."""
    P = S.Problem(_rand_vox(8, 22), 3)
    L = 3
    lam = [P.lambda_max(l) for l in range(L)]
    sm = {"kind": "jacobi", "omega": [1.0 / x for x in lam]}
    n = [lv.n_n for lv in P.levels]
    u0 = random_vectors(n[0], 18, 2).reshape(n[0], 6, 3)
    e_init = [None] + [random_vectors(n[l], 18, 10 + l).reshape(n[l], 6, 3) for l in range(1, L)]
    out = S.vcycle(P, P.f, u0, sm, nu1=2, nu2=1, e_init=e_init)

    Kd = [P.K[0].toarray()]
    Pd = [P.P[l].toarray() for l in range(L - 1)]
    for l in range(L - 1):
        Kd.append(Pd[l].T @ Kd[l] @ Pd[l])
    Dinv = [1.0 / np.diag(k) for k in Kd]

    def jac(l, u, f, nu):
        for _ in range(nu):
            u = u + sm["omega"][l] * Dinv[l][:, None] * (f - Kd[l] @ u)
        return u

    f = [ops.to_dofs(P.f)] + [None] * (L - 1)
    u = [ops.to_dofs(u0)] + [None] * (L - 1)
    for l in range(L - 1):
        u[l] = jac(l, u[l], f[l], 2)
        f[l + 1] = Pd[l].T @ (f[l] - Kd[l] @ u[l])
        u[l + 1] = ops.to_dofs(e_init[l + 1])
    Kc = Kd[-1].copy()
    Kc[:3, :] = 0
    Kc[:, :3] = 0
    Kc[np.arange(3), np.arange(3)] = 1.0
    fc = f[-1].copy()
    fc[:3] = 0
    u[-1] = np.linalg.solve(Kc, fc)
    for l in range(L - 2, -1, -1):
        u[l] = jac(l, u[l] + Pd[l] @ u[l + 1], f[l], 1)
    assert np.abs(ops.to_dofs(out) - u[0]).max() < 1e-10 * np.abs(u[0]).max()


@pytest.mark.parametrize("physics", ["elastic", "thermal"])
def test_pcg_matches_dense_cholesky(physics):
    P = S.Problem(gyroid_sheet(8, 6, 0.5), 2, physics)
    ud = S.direct_solve(P)
    assert np.max(S.relative_residual(P, ud)) < 1e-12
    for pre in ["vcycle", "jacobi"]:
        u, it = S.pcg(P, tol=1e-12, precond=pre)
        assert np.abs(u - ud).max() <= 1e-9 * np.abs(ud).max()
        assert np.abs(u[0]).max() == 0.0  # gauge node pinned


def test_gauge_shift_is_a_translation():
    P = S.Problem(gyroid_sheet(8, 6, 0.5), 2)
    u, _ = S.pcg(P, tol=1e-12)
    t = u + np.array([0.3, -0.2, 1.1])[None, None, :]
    assert np.abs(S.gauge_shift(P, t) - u).max() < 1e-14
    assert np.abs(S.homogenize(P, t) - S.homogenize(P, u)).max() < 1e-12
