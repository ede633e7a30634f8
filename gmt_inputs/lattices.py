"""Seeded periodic lattice families for the homogenization workloads.

Families (all periodic on the N^3 cell, voxel centres at ``(i + 1/2) / N``):

* TPMS sheets ``|F(x)| < t``: gyroid, Schwarz-P and diamond, with a per-seed
  phase shift ``phi ~ U[0, 2 pi)^3``; ``t`` is chosen so that exactly
  ``k = round(VF * N^3)`` voxels are solid before cleanup (ties broken by the
  linear index).
* periodic truss: 8..27 seeded nodes joined by struts to their periodic
  nearest neighbours until the strut graph winds around the cell in x, y and
  z; one common strut radius, set by the volume-fraction quantile of the
  distance field.
* spinodal: white noise filtered by a Gaussian shell ``|k| = k0``
  (``k0 ~ U[6, 10]``, width 1) and thresholded at the volume-fraction quantile.
* laminates and the uniform solid, used by closed-form checks.

Every generated lattice is reduced to its largest periodic face-connected
component (``cleanup_largest_component``) so the solid is one rigid body whose
only zero-energy modes are translations.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

FAMILIES = ("gyroid", "schwarz_p", "diamond", "truss", "spinodal")

_AXES = (2, 1, 0)  # array axis holding x, y, z


def _centres(N: int, phase=(0.0, 0.0, 0.0)):
    t = 2.0 * np.pi * (np.arange(N, dtype=np.float64) + 0.5) / N
    z = t[:, None, None] + phase[2]
    y = t[None, :, None] + phase[1]
    x = t[None, None, :] + phase[0]
    return x, y, z


def _smallest_k(score: np.ndarray, k: int) -> np.ndarray:
    """Mark the k voxels with the smallest score (stable: ties by linear index)."""
    flat = score.ravel()
    order = np.argsort(flat, kind="stable")
    out = np.zeros(flat.size, dtype=np.uint8)
    out[order[:k]] = 1
    return out.reshape(score.shape)


def _sheet(field: np.ndarray, vf: float, threshold=None) -> np.ndarray:
    if threshold is not None:
        return (np.abs(field) < threshold).astype(np.uint8)
    k = int(round(vf * field.size))
    return _smallest_k(np.abs(field), k)


def _phase(seed: int):
    rng = np.random.default_rng(seed)
    return tuple(rng.uniform(0.0, 2.0 * np.pi, size=3))


def gyroid_sheet(N: int, seed: int, vf: float, phase=None, clean: bool = True, threshold=None):
    ph = _phase(seed) if phase is None else phase
    x, y, z = _centres(N, ph)
    f = np.sin(x) * np.cos(y) + np.sin(y) * np.cos(z) + np.sin(z) * np.cos(x)
    v = _sheet(f, vf, threshold)
    return cleanup_largest_component(v) if clean else v


def schwarz_p_sheet(N: int, seed: int, vf: float, phase=None, clean: bool = True, threshold=None):
    ph = _phase(seed) if phase is None else phase
    x, y, z = _centres(N, ph)
    f = np.cos(x) + np.cos(y) + np.cos(z)
    v = _sheet(f, vf, threshold)
    return cleanup_largest_component(v) if clean else v


def diamond_sheet(N: int, seed: int, vf: float, phase=None, clean: bool = True, threshold=None):
    ph = _phase(seed) if phase is None else phase
    x, y, z = _centres(N, ph)
    sx, sy, sz = np.sin(x), np.sin(y), np.sin(z)
    cx, cy, cz = np.cos(x), np.cos(y), np.cos(z)
    f = sx * sy * sz + sx * cy * cz + cx * sy * cz + cx * cy * sz
    v = _sheet(f, vf, threshold)
    return cleanup_largest_component(v) if clean else v


def spinodal(N: int, seed: int, vf: float, k0=None, clean: bool = True, max_tries: int = 20):
    """Thresholded Gaussian random field with a spectral shell at |k| = k0."""
    for attempt in range(max_tries):
        rng = np.random.default_rng([seed, attempt])
        kk = rng.uniform(6.0, 10.0) if k0 is None else float(k0)
        noise = rng.standard_normal((N, N, N))
        f = np.fft.fftfreq(N) * N
        kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
        kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
        filt = np.exp(-0.5 * (kmag - kk) ** 2)
        phi = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
        k = int(round(vf * N ** 3))
        v = _smallest_k(-phi, k)
        if not clean:
            return v
        c = cleanup_largest_component(v)
        if abs(c.mean() - vf) <= 0.02 and winding_rank(c) == 3:
            return c
    raise RuntimeError(f"spinodal: no percolating cell for seed {seed}, vf {vf}")


def _segment_distance(P, A, B):
    """Distance from points P (..., 3) to segment A-B (unwrapped coordinates)."""
    d = B - A
    L2 = float(d @ d)
    t = np.clip(((P - A) @ d) / L2, 0.0, 1.0) if L2 > 0 else np.zeros(P.shape[:-1])
    Q = A + t[..., None] * d
    return np.sqrt(((P - Q) ** 2).sum(-1))


def truss(N: int, seed: int, vf: float, clean: bool = True, max_tries: int = 20):
    """Periodic strut lattice; strut radius from the VF quantile of the distance field."""
    for attempt in range(max_tries):
        rng = np.random.default_rng([seed, attempt])
        nn = int(rng.integers(8, 28))
        pts = rng.uniform(0.0, N, size=(nn, 3))
        # periodic minimum-image differences
        diff = pts[None, :, :] - pts[:, None, :]
        diff -= N * np.round(diff / N)
        dist = np.sqrt((diff ** 2).sum(-1))
        np.fill_diagonal(dist, np.inf)
        order = np.argsort(dist, axis=1)
        rcap = N / 4.0
        v = None
        for kn in range(3, min(nn, 9)):
            edges = set()
            for a in range(nn):
                for b in order[a, :kn]:
                    edges.add((min(a, int(b)), max(a, int(b))))
            D = np.full((N, N, N), np.inf)
            for a, b in sorted(edges):
                A = pts[a]
                B = pts[a] + diff[a, b]
                lo = np.floor(np.minimum(A, B) - rcap).astype(int)
                hi = np.ceil(np.maximum(A, B) + rcap).astype(int)
                hi = np.minimum(hi, lo + N - 1)
                gx = np.arange(lo[0], hi[0] + 1)
                gy = np.arange(lo[1], hi[1] + 1)
                gz = np.arange(lo[2], hi[2] + 1)
                Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
                P = np.stack([X + 0.5, Y + 0.5, Z + 0.5], axis=-1)
                d = _segment_distance(P, A, B)
                iz, iy, ix = np.ix_(gz % N, gy % N, gx % N)
                D[iz, iy, ix] = np.minimum(D[iz, iy, ix], d)
            k = int(round(vf * N ** 3))
            if not np.isfinite(np.sort(D.ravel())[k - 1]):
                continue
            cand = _smallest_k(D, k)
            if winding_rank(cand) == 3:
                v = cand
                break
        if v is None:
            continue
        if not clean:
            return v
        c = cleanup_largest_component(v)
        if abs(c.mean() - vf) <= 0.02 and winding_rank(c) == 3:
            return c
    raise RuntimeError(f"truss: no percolating cell for seed {seed}, vf {vf}")


def laminate(N: int, thickness: int, axis: int = 2, offset: int = 0) -> np.ndarray:
    """Solid slabs normal to ``axis`` (0=x, 1=y, 2=z): layers offset..offset+thickness-1."""
    v = np.zeros((N, N, N), dtype=np.uint8)
    idx = [(offset + i) % N for i in range(thickness)]
    sl = [slice(None)] * 3
    sl[_AXES[axis]] = idx
    v[tuple(sl)] = 1
    return v


def uniform(N: int) -> np.ndarray:
    return np.ones((N, N, N), dtype=np.uint8)


# ---------------------------------------------------------------- components


def _face_edges(lab: np.ndarray):
    """Label pairs joined across the periodic faces, with the unit shift."""
    out = []
    for ax_xyz in range(3):
        ax = _AXES[ax_xyz]
        a = np.take(lab, -1, axis=ax).ravel()
        b = np.take(lab, 0, axis=ax).ravel()
        m = (a > 0) & (b > 0)
        if m.any():
            pairs = np.unique(np.stack([a[m], b[m]], axis=1), axis=0)
            s = np.zeros(3, dtype=np.int64)
            s[ax_xyz] = 1
            for p, q in pairs:
                out.append((int(p), int(q), s))
    return out


def periodic_components(solid: np.ndarray):
    """Periodic face-connected components.

    Returns ``(labels, sizes, windings)`` where ``labels`` is the non-periodic
    label array remapped to periodic component ids 1..C, ``sizes[c-1]`` the
    voxel count and ``windings[c-1]`` the rank of the lattice of closed-loop
    translations of component c (3 = winds around the cell in three
    independent directions).
    """
    lab, n = ndimage.label(solid.astype(bool))
    if n == 0:
        return lab, np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    adj = [[] for _ in range(n + 1)]
    for a, b, s in _face_edges(lab):
        adj[a].append((b, s))
        adj[b].append((a, -s))
    comp = np.zeros(n + 1, dtype=np.int64)
    off = np.zeros((n + 1, 3), dtype=np.int64)
    windings = []
    ncomp = 0
    for root in range(1, n + 1):
        if comp[root]:
            continue
        ncomp += 1
        comp[root] = ncomp
        stack = [root]
        wv = []
        while stack:
            a = stack.pop()
            for b, s in adj[a]:
                if not comp[b]:
                    comp[b] = ncomp
                    off[b] = off[a] + s
                    stack.append(b)
                else:
                    w = off[a] + s - off[b]
                    if w.any():
                        wv.append(w)
        windings.append(int(np.linalg.matrix_rank(np.array(wv))) if wv else 0)
    plab = comp[lab]
    plab[lab == 0] = 0
    sizes = np.bincount(plab.ravel(), minlength=ncomp + 1)[1:]
    return plab, sizes, np.array(windings, dtype=np.int64)


def cleanup_largest_component(solid: np.ndarray) -> np.ndarray:
    plab, sizes, _ = periodic_components(solid)
    if sizes.size == 0:
        return solid.astype(np.uint8)
    keep = int(np.argmax(sizes)) + 1  # argmax: first (lowest label) on ties
    return (plab == keep).astype(np.uint8)


def winding_rank(solid: np.ndarray) -> int:
    """Winding rank of the largest periodic component (3 = percolates in 3D)."""
    plab, sizes, wind = periodic_components(solid)
    if sizes.size == 0:
        return 0
    return int(wind[int(np.argmax(sizes))])


# ------------------------------------------------------------------- batches


def cell(family: str, N: int, seed: int, vf: float) -> np.ndarray:
    fn = {
        "gyroid": gyroid_sheet,
        "schwarz_p": schwarz_p_sheet,
        "diamond": diamond_sheet,
        "truss": truss,
        "spinodal": spinodal,
    }[family]
    return fn(N, seed, vf)


def workload_cell(N: int, seed: int):
    """Mixed-family cell of the batched workloads: family = seed mod 5, VF ~ U(0.15, 0.5).

    A draw that cannot be made at the sampled VF (a thin spinodal that does not
    percolate after cleanup) is repeated at VF + 0.05; the returned VF is the one used.
    """
    rng = np.random.default_rng([seed, 7])
    vf = float(rng.uniform(0.15, 0.5))
    fam = FAMILIES[seed % 5]
    while True:
        try:
            return fam, vf, cell(fam, N, seed, vf)
        except RuntimeError:
            if vf >= 0.5:
                raise
            vf = min(0.5, vf + 0.05)


def random_vectors(n: int, q: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded standard-normal ``[n][q]`` array (test inputs for operator parity)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, q)).astype(dtype)
