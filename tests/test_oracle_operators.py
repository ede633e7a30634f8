"""Pins of the oracle's operators (Sec. 4.6, Sec. 3.2 Galerkin, App. E.2)."""

import itertools

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet, random_vectors
from oracle import fem, hierarchy, operators as ops
from oracle.solve import Problem


def _rand_vox(N, seed, p=0.35):
    rng = np.random.default_rng(seed)
    return (rng.random((N, N, N)) < p).astype(np.uint8)


def _dense_K_loops(vox, Ke, d):
    """Textbook assembly with explicit loops over voxels and corners."""
    N = vox.shape[0]
    lv = hierarchy.build(vox, 1)[0]
    ids = {p: i for i, p in enumerate(lv.node_lin.tolist())}
    K = np.zeros((lv.n_n * d, lv.n_n * d))
    for z, y, x in itertools.product(range(N), repeat=3):
        if not vox[z, y, x]:
            continue
        g = []
        for c, b, a in itertools.product((0, 1), repeat=3):
            pass
        corners = [((x + a) % N, (y + b) % N, (z + c) % N)
                   for a, b, c in [(k & 1, (k >> 1) & 1, (k >> 2) & 1) for k in range(8)]]
        for i_loc, pi in enumerate(corners):
            for j_loc, pj in enumerate(corners):
                I = ids[pi[0] + N * (pi[1] + N * pi[2])]
                J = ids[pj[0] + N * (pj[1] + N * pj[2])]
                for di in range(d):
                    for dj in range(d):
                        K[I * d + di, J * d + dj] += Ke[i_loc * d + di, j_loc * d + dj]
    return lv, K


@pytest.mark.parametrize("physics", ["elastic", "thermal"])
@pytest.mark.parametrize("N,seed", [(4, 0), (4, 1), (2, 2)])
def test_apply_K_vs_dense_loops(physics, N, seed):
    Ke, X0, d = fem.element(physics)
    vox = _rand_vox(N, seed) if N > 2 else np.ones((2, 2, 2), np.uint8)
    lv, K = _dense_K_loops(vox, Ke, d)
    c = X0.shape[1]
    u = random_vectors(lv.n_n, c * d, seed).reshape(lv.n_n, c, d)
    y = ops.apply_K(lv, Ke, u)
    y_ref = ops.from_dofs(K @ ops.to_dofs(u), d)
    assert np.abs(y - y_ref).max() <= 1e-13 * np.abs(y_ref).max()
    Ks = ops.assemble(lv, Ke, d).toarray()
    assert np.abs(Ks - K).max() < 1e-14
    assert np.abs(K - K.T).max() < 1e-14
    for dd in range(d):  # rigid translation in the null space
        t = np.zeros((lv.n_n, d))
        t[:, dd] = 1.0
        assert np.abs(K @ t.ravel()).max() < 1e-13


@pytest.mark.parametrize("physics", ["elastic", "thermal"])
def test_galerkin_local_equals_global(physics):
    vox = _rand_vox(8, 11, 0.3)
    P = Problem(vox, 3, physics)
    for l in range(2):
        Kg = (P.P[l].T @ P.K[l] @ P.P[l]).toarray()
        Kl = P.K[l + 1].toarray()
        assert np.abs(Kg - Kl).max() <= 1e-14 * np.abs(Kl).max()


def test_galerkin_full_coarse_element_is_scaled_Ke():
    # a coarse element over 8 solid children of the voxel K_e equals 2 * K_e
    # (trilinear fields are reproduced; the hex8 stiffness scales with h)
    Ke = fem.Ke_elastic()
    P = Problem(np.ones((4, 4, 4), np.uint8), 2)
    KE = P.mats[1]
    assert np.abs(KE - 2.0 * Ke[None]).max() < 1e-14


def test_restrict_is_transpose_of_prolong():
    vox = _rand_vox(8, 12, 0.3)
    lv = hierarchy.build(vox, 2)
    f, c = lv[0], lv[1]
    Pd = np.zeros((f.n_n, c.n_n))
    for j in range(c.n_n):
        e = np.zeros((c.n_n, 1, 1))
        e[j] = 1.0
        Pd[:, j] = ops.prolong(f, e)[:, 0, 0]
    r = random_vectors(f.n_n, 1, 3).reshape(f.n_n, 1, 1)
    assert np.abs(ops.restrict(f, r, c.n_n)[:, 0, 0] - Pd.T @ r[:, 0, 0]).max() < 1e-14
    # P reproduces constants
    assert np.abs(Pd.sum(axis=1) - 1.0).max() == 0.0


def test_load_vector_consistent():
    P = Problem(gyroid_sheet(16, 3, 0.3), 2)
    assert np.abs(P.f.sum(axis=0)).max() < 1e-12  # sum f = 0 (translations)
    Pu = Problem(np.ones((8, 8, 8), np.uint8), 2)
    assert np.abs(Pu.f).max() < 1e-14  # uniform solid: interior cancellation


def test_diagonal_matches_assembled():
    P = Problem(_rand_vox(8, 13, 0.4), 3)
    for l in range(3):
        assert np.abs(P.D[l].ravel() - P.K[l].diagonal()).max() < 1e-14
