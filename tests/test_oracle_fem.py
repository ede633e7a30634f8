"""Pins of the oracle's element quantities (App. F.1 / F.2) against closed forms."""

import numpy as np
import pytest

from oracle import fem


def test_isotropic_constants():
    # E=1, nu=0.3: lambda+2G = 1.346154, lambda = 0.576923, G = 0.384615
    C = fem.isotropic_C(1.0, 0.3)
    assert C[0, 0] == pytest.approx(0.7 / (1.3 * 0.4), rel=1e-15)
    assert C[0, 1] == pytest.approx(0.3 / (1.3 * 0.4), rel=1e-15)
    assert C[3, 3] == pytest.approx(1.0 / 2.6, rel=1e-15)
    assert C[0, 3] == 0.0 and C[3, 4] == 0.0


@pytest.mark.parametrize("E,nu", [(1.0, 0.3), (2.5, 0.1), (0.7, 0.45)])
def test_Ke_two_constructions_agree(E, nu):
    K1 = fem.Ke_elastic(E, nu)
    K2 = fem.Ke_elastic_tensor(E, nu)
    assert np.abs(K1 - K2).max() <= 1e-14 * np.abs(K1).max()


def test_Ke_symmetric_psd_rank18():
    K = fem.Ke_elastic(1.0, 0.3)
    assert np.abs(K - K.T).max() < 1e-15
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-13
    assert int(np.sum(w > 1e-10)) == 18  # six rigid modes in the null space


def test_Ke_annihilates_rigid_modes():
    K = fem.Ke_elastic(1.0, 0.3)
    X = fem.CORNERS.astype(float) + np.array([0.3, -1.7, 2.2])  # arbitrary origin
    modes = []
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1.0
        modes.append(t.ravel())
    for axis in np.eye(3):
        modes.append(np.cross(axis[None, :], X).ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-14


def test_affine_energy_is_C0():
    # X0^T K_e X0 = int eps_bar^T C0 eps_bar over the unit voxel = C0 exactly
    for E, nu in [(1.0, 0.3), (3.0, 0.2)]:
        K = fem.Ke_elastic(E, nu)
        X = fem.X0_elastic()
        assert np.abs(X.T @ K @ X - fem.isotropic_C(E, nu)).max() < 1e-14


def test_X0_carries_unit_strains():
    # B X0 = I_6 at any point of the voxel
    X = fem.X0_elastic()
    for xi in ([0.1, 0.7, 0.4], [0.5, 0.5, 0.5], [0.9, 0.0, 1.0]):
        assert np.abs(fem.strain_B(np.array(xi)) @ X - np.eye(6)).max() < 1e-15


def test_thermal_closed_form():
    K = fem.Ke_thermal(1.0)
    ref = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            ndiff = bin(a ^ b).count("1")
            ref[a, b] = {0: 4.0, 1: 0.0, 2: -1.0, 3: -1.0}[ndiff] / 12.0
    assert np.abs(K - ref).max() < 1e-15
    assert np.abs(K.sum(axis=1)).max() < 1e-15
    X = fem.X0_thermal()
    assert np.abs(X.T @ K @ X - np.eye(3)).max() < 1e-15
    assert np.abs(fem.Ke_thermal(2.0) - 2.0 * K).max() < 1e-15
