"""Pins of the oracle's effective tensors (App. F.1 / F.2) against closed forms and invariants."""

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet, laminate, schwarz_p_sheet, uniform
from oracle import fem
from oracle import operators as ops
from oracle import solve as S

E, NU = 1.0, 0.3


def _solve(vox, L, physics="elastic", tol=1e-11):
    P = S.Problem(vox, L, physics)
    u, _ = S.pcg(P, tol=tol)
    return P, u, S.homogenize(P, u)


@pytest.mark.parametrize("physics", ["elastic", "thermal"])
def test_uniform_solid_is_C0(physics):
    P = S.Problem(uniform(8), 3, physics)
    assert np.abs(P.f).max() < 1e-14
    CH = S.homogenize(P, np.zeros_like(P.f))
    assert np.abs(CH - fem.base_tensor(physics, E, NU)).max() < 1e-12  # sum of 512 rounded terms


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_elastic_closed_form(axis):
    N, t = 8, 3
    P, u, CH = _solve(laminate(N, t, axis=axis, offset=2), 2)
    vf = t / N
    Q11 = E / (1 - NU ** 2)
    Q12 = NU * E / (1 - NU ** 2)
    G = E / (2 * (1 + NU))
    inplane = [a for a in range(3) if a != axis]  # normal strains in the plane
    shear_in = {frozenset((0, 1)): 5, frozenset((0, 2)): 4, frozenset((1, 2)): 3}[frozenset(inplane)]
    ref = np.zeros((6, 6))
    i, j = inplane
    ref[i, i] = ref[j, j] = vf * Q11
    ref[i, j] = ref[j, i] = vf * Q12
    ref[shear_in, shear_in] = vf * G
    assert np.abs(CH - ref).max() < 1e-9


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_thermal_closed_form(axis):
    N, t = 8, 5
    P, u, KH = _solve(laminate(N, t, axis=axis, offset=1), 2, "thermal")
    ref = np.eye(3) * (t / N)
    ref[axis, axis] = 0.0
    assert np.abs(KH - ref).max() < 1e-9


@pytest.fixture(scope="module")
def gyroid16():
    return _solve(gyroid_sheet(16, 3, 0.3), 3)


def test_energy_form_identity(gyroid16):
    # element sum == (n_e C0 - F^T U - U^T F + U^T K U) / N^3 with assembled f and K
    P, u, CH = gyroid16
    U = ops.to_dofs(u)
    F = ops.to_dofs(P.f)
    KU = P.K[0] @ U
    alt = (P.levels[0].n_e * fem.isotropic_C(E, NU) - F.T @ U - U.T @ F + U.T @ KU) / P.N ** 3
    assert np.abs(alt - CH).max() < 1e-12


def test_symmetric_and_voigt_bound(gyroid16):
    P, u, CH = gyroid16
    assert np.abs(CH - CH.T).max() < 1e-12
    vf = P.levels[0].n_e / P.N ** 3
    assert np.linalg.eigvalsh(vf * fem.isotropic_C(E, NU) - CH).min() > -1e-12
    assert np.linalg.eigvalsh(CH).min() > 0.0


def test_translation_invariance(gyroid16):
    P, u, CH = gyroid16
    vox = gyroid_sheet(16, 3, 0.3)
    _, _, CH2 = _solve(np.roll(vox, shift=(3, -5, 7), axis=(0, 1, 2)), 3)
    assert np.abs(CH2 - CH).max() < 1e-9 * np.abs(CH).max()


def _voigt_perm(p):
    """Voigt index map for the axis permutation new_axis[i] = p[i]."""
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    idx = {frozenset(q) if q[0] != q[1] else (q[0],): k for k, q in enumerate(pairs)}
    out = []
    for a, b in pairs:
        pa, pb = p[a], p[b]
        out.append(idx[frozenset((pa, pb))] if pa != pb else idx[(pa,)])
    return out


def test_permutation_and_reflection_equivariance(gyroid16):
    P, u, CH = gyroid16
    vox = gyroid_sheet(16, 3, 0.3)
    # swap x <-> y (array axes 2 <-> 1): new cell value at (x,y,z) = old at (y,x,z)
    _, _, CHs = _solve(vox.transpose(0, 2, 1).copy(), 3)
    perm = _voigt_perm([1, 0, 2])
    assert np.abs(CHs - CH[np.ix_(perm, perm)]).max() < 1e-9 * np.abs(CH).max()
    # reflection x -> N - x: shears containing x once flip sign
    _, _, CHr = _solve(vox[:, :, ::-1].copy(), 3)
    Q = np.diag([1, 1, 1, 1, -1, -1.0])
    assert np.abs(CHr - Q @ CH @ Q).max() < 1e-9 * np.abs(CH).max()


def test_schwarz_p_cubic_symmetry_and_hs_bound():
    vox = schwarz_p_sheet(16, 0, 0.3, phase=(0.0, 0.0, 0.0), threshold=0.6)
    P, u, CH = _solve(vox, 3)
    s = np.abs(CH).max()
    assert abs(CH[0, 0] - CH[1, 1]) < 1e-9 * s and abs(CH[0, 0] - CH[2, 2]) < 1e-9 * s
    assert abs(CH[0, 1] - CH[0, 2]) < 1e-9 * s and abs(CH[0, 1] - CH[1, 2]) < 1e-9 * s
    assert abs(CH[3, 3] - CH[4, 4]) < 1e-9 * s and abs(CH[3, 3] - CH[5, 5]) < 1e-9 * s
    off = CH.copy()
    off[:3, :3] = 0
    np.fill_diagonal(off, 0)
    assert np.abs(off).max() < 1e-9 * s
    # Hashin-Shtrikman upper bound on the bulk modulus (sanity; FE with void is
    # stiff at coarse N, so allow 5 %)
    vf = vox.mean()
    K0 = E / (3 * (1 - 2 * NU))
    G0 = E / (2 * (1 + NU))
    K_hs = 4 * G0 * K0 * vf / (3 * K0 * (1 - vf) + 4 * G0)
    assert (CH[0, 0] + 2 * CH[0, 1]) / 3 <= 1.05 * K_hs


def test_thermal_bound_and_symmetry():
    vox = gyroid_sheet(16, 9, 0.35)
    P, u, KH = _solve(vox, 3, "thermal")
    vf = vox.mean()
    assert np.abs(KH - KH.T).max() < 1e-12
    assert np.linalg.eigvalsh(vf * np.eye(3) - KH).min() > -1e-12
    assert np.trace(KH) / 3 <= 2 * vf / (3 - vf) * 1.05  # HS upper bound (sanity)
