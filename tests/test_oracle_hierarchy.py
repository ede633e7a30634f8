"""Pins of the oracle's sparse hierarchy (Sec. 4.1, eq. gmgcoarsenode; App. E.1).

Brute force: sets of integer coordinates built with plain Python loops.
"""

import itertools

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet
from oracle import hierarchy


def _rand_vox(N, seed, p=0.3):
    rng = np.random.default_rng(seed)
    return (rng.random((N, N, N)) < p).astype(np.uint8)


def _brute(vox, L):
    N = vox.shape[0]
    levels = []
    elems = {(x, y, z) for z in range(N) for y in range(N) for x in range(N) if vox[z, y, x]}
    n = N
    for l in range(L):
        nodes = set()
        for (x, y, z) in elems:
            for a, b, c in itertools.product((0, 1), repeat=3):
                nodes.add(((x + a) % n, (y + b) % n, (z + c) % n))
        lin = lambda p, n=n: p[0] + n * (p[1] + n * p[2])
        levels.append((n, sorted(lin(e) for e in elems), sorted(lin(p) for p in nodes), elems, nodes))
        if l < L - 1:
            elems = {(x // 2, y // 2, z // 2) for (x, y, z) in elems}
            n //= 2
    return levels


@pytest.mark.parametrize("N,L,seed", [(4, 2, 0), (8, 3, 1), (8, 3, 2), (8, 2, 3)])
def test_sets_and_ids_brute_force(N, L, seed):
    vox = _rand_vox(N, seed)
    lv = hierarchy.build(vox, L)
    bf = _brute(vox, L)
    for l in range(L):
        n, e_lin, n_lin, elems, nodes = bf[l]
        assert lv[l].N == n
        assert lv[l].elem_lin.tolist() == e_lin
        assert lv[l].node_lin.tolist() == n_lin
        ids = {p: i for i, p in enumerate(n_lin)}
        # connectivity: corner a+2b+4c of element e
        for k, el in enumerate(e_lin):
            x, y, z = el % n, (el // n) % n, el // (n * n)
            for a, b, c in itertools.product((0, 1), repeat=3):
                corner = a + 2 * b + 4 * c
                p = ((x + a) % n) + n * (((y + b) % n) + n * ((z + c) % n))
                assert lv[l].elem_nodes[k, corner] == ids[p]


@pytest.mark.parametrize("N,seed", [(4, 5), (8, 6)])
def test_occupancy_brute_force(N, seed):
    vox = _rand_vox(N, seed)
    lv = hierarchy.build(vox, 1)[0]
    for i, p in enumerate(lv.node_lin.tolist()):
        x, y, z = p % N, (p // N) % N, p // (N * N)
        bits = 0
        for a, b, c in itertools.product((0, 1), repeat=3):
            if vox[(z - 1 + c) % N, (y - 1 + b) % N, (x - 1 + a) % N]:
                bits |= 1 << (a + 2 * b + 4 * c)
        assert int(lv.occ8[i]) == bits
        assert bits != 0  # every active node touches an active voxel


@pytest.mark.parametrize("N,L,seed", [(8, 3, 7), (8, 2, 8)])
def test_transfer_brute_force(N, L, seed):
    vox = _rand_vox(N, seed)
    lv = hierarchy.build(vox, L)
    for l in range(L - 1):
        fine, coarse = lv[l], lv[l + 1]
        nf, nc = fine.N, coarse.N
        cid = {p: i for i, p in enumerate(coarse.node_lin.tolist())}
        for i, p in enumerate(fine.node_lin.tolist()):
            xf = (p % nf, (p // nf) % nf, p // (nf * nf))
            for k in range(8):
                o = (k & 1, (k >> 1) & 1, (k >> 2) & 1)
                w = 1.0
                for dd in range(3):
                    w *= 1.0 - abs((xf[dd] % 2) / 2.0 - o[dd])
                if w == 0.0:
                    assert fine.prol_idx[i, k] == -1 and fine.prol_w[i, k] == 0.0
                else:
                    q = [((xf[dd] // 2) + o[dd]) % nc for dd in range(3)]
                    lin = q[0] + nc * (q[1] + nc * q[2])
                    assert lin in cid  # a nonzero-weight corner is always active
                    assert fine.prol_idx[i, k] == cid[lin]
                    assert fine.prol_w[i, k] == w


def test_invariants_gyroid():
    vox = gyroid_sheet(32, 0, 0.3)
    lv = hierarchy.build(vox, 4)
    prev_e = None
    for l, L_ in enumerate(lv):
        # each active node is a corner of >=1 active element
        assert np.array_equal(np.unique(L_.elem_nodes), np.arange(L_.n_n))
        if prev_e is not None:
            assert L_.n_e <= prev_e
        prev_e = L_.n_e
        if L_.prol_w is not None:
            assert np.allclose(L_.prol_w.sum(axis=1), 1.0, rtol=0, atol=0)  # P 1 = 1 exactly
            assert np.all(L_.prol_w[L_.prol_idx < 0] == 0.0)
            assert set(np.unique(L_.prol_w)) <= {0.0, 0.125, 0.25, 0.5, 1.0}


def test_rejects_bad_sizes():
    with pytest.raises(ValueError):
        hierarchy.build(np.ones((6, 6, 6), np.uint8), 3)  # 6 not divisible by 4
    with pytest.raises(ValueError):
        hierarchy.build(np.zeros((4, 4, 4), np.uint8), 2)  # empty
    with pytest.raises(ValueError):
        hierarchy.build(np.ones((4, 4, 4), np.uint8), 3)  # N_L = 1
