"""Sparse active-voxel GMG hierarchy by definition (Sec. 4.1, eq. gmgcoarsenode; App. E.1).

* Level 1 elements are the solid voxels; nodes are the vertex union of the
  active elements (Sec. 4.1.1), each carrying an 8-bit occupancy of the eight
  voxels around it.
* A coarse voxel is active iff any of its 2x2x2 children is active; coarse
  nodes are again the vertex union (eq. gmgcoarsenode).
* Transfer stencil (App. E.1): fine node x_f has parent cell x_c = floor(x_f/2),
  corners (x_c + o_k) mod N_c and weights prod_d (1 - |xi_d - o_k,d|) with
  xi = (x_f mod 2)/2.  Corners with zero weight are stored as id -1, weight 0.

Everything is computed with numpy on dense grids; ids are ranks among the
sorted linear indices ``x + N*(y + N*z)``.  Parity: pinned by the brute-force
set construction in ``tests/test_oracle_hierarchy.py``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fem import CORNERS


@dataclass
class Level:
    N: int
    elem_active: np.ndarray  # bool [N,N,N] indexed [z,y,x]
    elem_lin: np.ndarray  # int64 sorted active element linear indices
    node_lin: np.ndarray  # int64 sorted active node linear indices
    node_id: np.ndarray  # int64 [N,N,N] -> id or -1
    elem_nodes: np.ndarray  # int64 [n_e, 8]
    occ8: np.ndarray  # uint8 [n_n], occupancy of the 8 voxels around a node
    prol_idx: np.ndarray = field(default=None)  # int64 [n_n, 8] into next level
    prol_w: np.ndarray = field(default=None)  # float64 [n_n, 8]

    @property
    def n_e(self):
        return int(self.elem_lin.size)

    @property
    def n_n(self):
        return int(self.node_lin.size)


def _coords(lin, N):
    lin = np.asarray(lin, dtype=np.int64)
    return lin % N, (lin // N) % N, lin // (N * N)


def _lin(x, y, z, N):
    return (x % N) + N * ((y % N) + N * (z % N))


def make_level(elem_active: np.ndarray) -> Level:
    N = elem_active.shape[0]
    elem_lin = np.flatnonzero(elem_active.ravel()).astype(np.int64)
    # a node is active iff one of the 8 elements it is a corner of is active:
    # element (x-a, y-b, z-c) for corner (a,b,c)
    node_active = np.zeros_like(elem_active, dtype=bool)
    for a, b, c in CORNERS:
        node_active |= np.roll(elem_active, shift=(c, b, a), axis=(0, 1, 2))
    node_lin = np.flatnonzero(node_active.ravel()).astype(np.int64)
    node_id = np.full(N ** 3, -1, dtype=np.int64)
    node_id[node_lin] = np.arange(node_lin.size)
    node_id = node_id.reshape(N, N, N)
    ex, ey, ez = _coords(elem_lin, N)
    elem_nodes = np.stack(
        [node_id[(ez + c) % N, (ey + b) % N, (ex + a) % N] for a, b, c in CORNERS], axis=1
    )
    nx, ny, nz = _coords(node_lin, N)
    occ8 = np.zeros(node_lin.size, dtype=np.uint8)
    for k, (a, b, c) in enumerate(CORNERS):
        bit = elem_active[(nz - 1 + c) % N, (ny - 1 + b) % N, (nx - 1 + a) % N]
        occ8 |= (bit.astype(np.uint8) << k)
    return Level(N, elem_active.astype(bool), elem_lin, node_lin, node_id, elem_nodes, occ8)


def coarsen(elem_active: np.ndarray) -> np.ndarray:
    """Coarse voxel (I,J,K) active iff any child (2I+a, 2J+b, 2K+c) is active."""
    N = elem_active.shape[0]
    assert N % 2 == 0
    v = elem_active.reshape(N // 2, 2, N // 2, 2, N // 2, 2)
    return v.any(axis=(1, 3, 5))


def transfer(fine: Level, coarse: Level):
    """Stencil tuple (I, W) of App. E.2 for every active fine node."""
    Nc = coarse.N
    x, y, z = _coords(fine.node_lin, fine.N)
    xc, yc, zc = x // 2, y // 2, z // 2
    xi = np.stack([(x % 2) / 2.0, (y % 2) / 2.0, (z % 2) / 2.0], axis=1)
    idx = np.full((fine.n_n, 8), -1, dtype=np.int64)
    w = np.zeros((fine.n_n, 8))
    for k, o in enumerate(CORNERS):
        wk = np.prod(1.0 - np.abs(xi - o[None, :]), axis=1)
        cid = coarse.node_id[(zc + o[2]) % Nc, (yc + o[1]) % Nc, (xc + o[0]) % Nc]
        nz = wk != 0.0
        idx[nz, k] = cid[nz]
        w[nz, k] = wk[nz]
    return idx, w


def build(voxels: np.ndarray, levels: int):
    """List of ``levels`` Level objects; level l (0-based here) has N / 2^l voxels per axis."""
    N = voxels.shape[0]
    if voxels.shape != (N, N, N):
        raise ValueError("voxels must be N^3")
    if levels < 1 or N % (2 ** (levels - 1)) != 0 or N // 2 ** (levels - 1) < 2:
        raise ValueError("N must be divisible by 2^(L-1) with N_L >= 2")
    act = voxels.astype(bool)
    if not act.any():
        raise ValueError("empty active set")
    out = [make_level(act)]
    for _ in range(levels - 1):
        act = coarsen(act)
        out.append(make_level(act))
    for l in range(levels - 1):
        out[l].prol_idx, out[l].prol_w = transfer(out[l], out[l + 1])
    return out


def node_components(elem_active: np.ndarray) -> int:
    """Number of node-connected components of the active elements (periodic).

    Two active elements are connected when they share at least one node, i.e.
    when their voxel coordinates differ by at most one (mod N) along every
    axis.  Every such component can translate freely, so the periodic
    stiffness matrix has (components x d) rigid translations in its null space
    (one pinned node fixes only one of them).  Graph search by scipy's
    connected_components over that adjacency.
    """
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    act = np.asarray(elem_active, dtype=bool)
    lin = np.flatnonzero(act.ravel())
    if lin.size == 0:
        return 0
    flat = np.full(act.size, -1, dtype=np.int64)
    flat[lin] = np.arange(lin.size)
    eid = flat.reshape(act.shape)
    rows, cols = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = np.roll(eid, shift=(-dz, -dy, -dx), axis=(0, 1, 2))  # nb[z,y,x] = eid[z+dz, y+dy, x+dx]
                m = (eid >= 0) & (nb >= 0)
                rows.append(eid[m])
                cols.append(nb[m])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(lin.size, lin.size))
    return int(connected_components(A, directed=False)[0])


def pinned_node(level: Level) -> int:
    """Gauge node: the lowest-id active node (id 0)."""
    return 0
