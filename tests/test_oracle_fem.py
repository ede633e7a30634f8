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


def _corner_map(perm=(0, 1, 2), flip=0):
    """Image of the hex8 corner a + 2b + 4c under the cube symmetry that permutes the axes
    (new axis k takes old axis perm[k]) and then reflects the axes set in the bit mask flip."""
    out = []
    for a in range(8):
        bits = [(a >> k) & 1 for k in range(3)]
        nb = [bits[perm[k]] ^ ((flip >> k) & 1) for k in range(3)]
        out.append(nb[0] + 2 * nb[1] + 4 * nb[2])
    return out


def test_Ke_invariant_under_cube_symmetries():
    """The isotropic voxel element is invariant under the 48 symmetries of the cube: a
    reflection of axis k maps corner a to a ^ 2^k and negates displacement component k, and
    an axis permutation permutes corners and components alike.  So K_e[g(a), g(m)] equals
    K_e[a, m] up to the component map and signs, for every symmetry g (elastic and thermal)."""
    import itertools
    for E, nu in ((1.0, 0.3), (2.5, 0.45)):
        K = fem.Ke_elastic(E, nu).reshape(8, 3, 8, 3)
        for perm in itertools.permutations(range(3)):
            for flip in range(8):
                cm = _corner_map(perm, flip)
                # component k of the image is component perm[k] of the original, with sign
                sign = np.array([-1.0 if (flip >> k) & 1 else 1.0 for k in range(3)])
                P = np.zeros((3, 3))
                for k in range(3):
                    P[k, perm[k]] = sign[k]
                for a in range(8):
                    for m in range(8):
                        img = K[cm[a], :, cm[m], :]
                        assert np.allclose(img, P @ K[a, :, m, :] @ P.T, atol=1e-13 * np.abs(K).max())
    Kt = fem.Ke_thermal(1.0)
    for perm in itertools.permutations(range(3)):
        for flip in range(8):
            cm = _corner_map(perm, flip)
            assert np.allclose(Kt[np.ix_(cm, cm)], Kt, atol=1e-14)


def test_Ke_has_14_symmetry_classes():
    """Consequence used by the GPU operator kernels: after the reflection taking corner a to
    corner 0 (signs (-1)^(a_d + a_d2)), entry (d, d2) of block (a, m) depends only on
    (delta_d, number of other set bits of delta) on the diagonal and on
    (delta_d, delta_d2, delta_third) off it, delta = a xor m: 6 + 8 = 14 values."""
    K = fem.Ke_elastic(1.0, 0.3).reshape(8, 3, 8, 3)
    vals = {}
    for a in range(8):
        for m in range(8):
            dl = a ^ m
            for d in range(3):
                for d2 in range(3):
                    s = (-1) ** (((a >> d) & 1) + ((a >> d2) & 1))
                    if d == d2:
                        key = ("diag", (dl >> d) & 1, bin(dl & ~(1 << d) & 7).count("1"))
                    else:
                        t = 3 - d - d2
                        key = ("off", (dl >> d) & 1, (dl >> d2) & 1, (dl >> t) & 1)
                    vals.setdefault(key, []).append(s * K[a, d, m, d2])
    assert len(vals) == 14
    for key, v in vals.items():
        assert np.ptp(v) <= 1e-13 * np.abs(K).max(), key
