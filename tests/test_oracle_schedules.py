"""Pins of the oracle's 8-colour Gauss-Seidel / SOR smoother, the W- and F-cycle
schedules, the node-connected component count and the physics loss.

Each reference here is built from dense matrices by a different route than the
oracle's matrix-free code: the Gauss-Seidel sweep as the SOR splitting
omega (D + omega L)^-1 and as a node-by-node loop, the W- and F-cycles as the
V-cycle with its coarse solve replaced by two iterations of the coarse cycle
(closed forms of iterating a linear method twice), the component count by a
breadth-first search over Python sets, and the loss by a dense V-cycle.
"""

import itertools
from collections import deque

import numpy as np
import pytest

from gmt_inputs import gyroid_sheet, random_vectors
from oracle import hierarchy as H
from oracle import nn as onn
from oracle import operators as ops
from oracle import solve as S


def _rand_vox(N, seed, p=0.45):
    rng = np.random.default_rng(seed)
    return (rng.random((N, N, N)) < p).astype(np.uint8)


@pytest.fixture(scope="module")
def prob8():
    return S.Problem(gyroid_sheet(8, 4, 0.45), 3)


def _node_colour_dofs(level, d):
    N = level.N
    lin = level.node_lin
    x, y, z = lin % N, (lin // N) % N, lin // (N * N)
    return np.repeat((x % 2) + 2 * (y % 2) + 4 * (z % 2), d)


def test_colour_classes_are_uncoupled(prob8):
    # no nonzero of K (any level) joins two different nodes of one colour
    for l in range(prob8.L - 1):
        lv = prob8.levels[l]
        K = prob8.K[l].tocoo()
        col = _node_colour_dofs(lv, prob8.d)
        ni, nj = K.row // prob8.d, K.col // prob8.d
        same = (col[K.row] == col[K.col]) & (ni != nj) & (np.abs(K.data) > 0)
        assert not same.any()
        # and every node has a colour in 0..7, all eight classes used at level 1
        c = S.colours(lv)
        assert c.min() >= 0 and c.max() <= 7
    assert len(np.unique(S.colours(prob8.levels[0]))) == 8


@pytest.mark.parametrize("omega", [1.0, 0.8, 1.2])
@pytest.mark.parametrize("reverse", [False, True])
def test_gauss_seidel_is_sor_splitting(prob8, omega, reverse):
    """One sweep = u + omega (D + omega L)^-1 (f - K u), L the couplings to earlier colours."""
    P = prob8
    for l in (0, 1):
        n = P.levels[l].n_n
        u0 = random_vectors(n, 18, 7 + l).reshape(n, 6, 3)
        f = random_vectors(n, 18, 17 + l).reshape(n, 6, 3)
        K = P.K[l].toarray()
        col = _node_colour_dofs(P.levels[l], 3)
        before = (col[None, :] > col[:, None]) if reverse else (col[None, :] < col[:, None])
        Lm = np.where(before, K, 0.0)
        Dm = np.diag(np.diag(K))
        U = ops.to_dofs(u0)
        for _ in range(2):
            U = U + omega * np.linalg.solve(Dm + omega * Lm, ops.to_dofs(f) - K @ U)
        out = S.gauss_seidel(P, l, u0, f, 2, omega, reverse=reverse)
        assert np.abs(ops.to_dofs(out) - U).max() <= 1e-11 * np.abs(U).max()


def test_gauss_seidel_node_by_node_loop():
    """Brute force: nodes updated one at a time, colour by colour, ascending id."""
    P = S.Problem(_rand_vox(4, 3, 0.6), 2)
    n = P.levels[0].n_n
    K = P.K[0].toarray()
    Dg = np.diag(K)
    u0 = random_vectors(n, 18, 3).reshape(n, 6, 3)
    f = random_vectors(n, 18, 4).reshape(n, 6, 3)
    U = ops.to_dofs(u0).copy()
    F = ops.to_dofs(f)
    col = S.colours(P.levels[0])
    for c in range(8):
        for i in np.flatnonzero(col == c):
            dofs = slice(3 * i, 3 * i + 3)
            r = F[dofs] - K[dofs] @ U
            U[dofs] = U[dofs] + 0.9 * r / Dg[dofs][:, None]
    out = S.gauss_seidel(P, 0, u0, f, 1, 0.9)
    assert np.abs(ops.to_dofs(out) - U).max() <= 1e-12 * np.abs(U).max()


def test_gauss_seidel_vcycle_is_symmetric(prob8):
    """Forward pre- and backward post-smoothing: <V x, y> = <x, V y> on consistent loads."""
    P = prob8
    n = P.levels[0].n_n
    sm = S.default_smoother(P, "gs")
    rng = np.random.default_rng(0)
    for _ in range(3):
        xv = rng.standard_normal((n, 6, 3))
        yv = rng.standard_normal((n, 6, 3))
        xv -= xv.mean(0, keepdims=True)
        yv -= yv.mean(0, keepdims=True)
        xv[0] = 0.0
        yv[0] = 0.0
        Vx = S.vcycle(P, xv, np.zeros_like(xv), sm, 2, 2)
        Vy = S.vcycle(P, yv, np.zeros_like(yv), sm, 2, 2)
        a, b = (Vx * yv).sum(), (xv * Vy).sum()
        assert abs(a - b) <= 1e-10 * max(abs(a), abs(b))
    # a forward post-smoother breaks the symmetry (the check above can fail)
    bad = dict(sm)

    def fwd_only(prob, l, u, f, nu, sm_, post=False):
        return S.gauss_seidel(prob, l, u, f, nu, sm_["omega"][l], reverse=False)

    orig = S.smooth
    try:
        S.smooth = fwd_only
        Vx = S.vcycle(P, xv, np.zeros_like(xv), bad, 2, 2)
        Vy = S.vcycle(P, yv, np.zeros_like(yv), bad, 2, 2)
    finally:
        S.smooth = orig
    a, b = (Vx * yv).sum(), (xv * Vy).sum()
    assert abs(a - b) > 1e-6 * max(abs(a), abs(b))


def test_gauss_seidel_pcg_converges():
    P = S.Problem(gyroid_sheet(8, 6, 0.5), 3)
    ud = S.direct_solve(P)
    u, it = S.pcg(P, tol=1e-12, sm=S.default_smoother(P, "gs"))
    assert np.abs(u - ud).max() <= 1e-9 * np.abs(ud).max()


# ---------------------------------------------------------------- W- and F-cycles, dense

class Dense:
    """Dense matrices of a hierarchy and the linear maps of its cycles (zero start)."""

    def __init__(self, P, sm, nu1=2, nu2=2):
        self.P, self.sm, self.nu1, self.nu2 = P, sm, nu1, nu2
        L = P.L
        self.K = [P.K[0].toarray()]
        self.Pm = [P.P[l].toarray() for l in range(L - 1)]
        for l in range(L - 1):
            self.K.append(self.Pm[l].T @ self.K[l] @ self.Pm[l])
        self.Dinv = [1.0 / np.diag(k) for k in self.K]
        Kc = self.K[-1].copy()
        d = P.d
        Kc[:d, :] = 0
        Kc[:, :d] = 0
        Kc[np.arange(d), np.arange(d)] = 1.0
        self.Kc = Kc

    def smooth(self, l, u, f, nu):
        w = self.sm["omega"][l]
        for _ in range(nu):
            u = u + w * self.Dinv[l][:, None] * (f - self.K[l] @ u)
        return u

    def coarsest(self, g):
        g = g.copy()
        g[:self.P.d] = 0.0
        return np.linalg.solve(self.Kc, g)

    def two_grid(self, l, g, e0, Bc):
        """pre-smooth from e0, coarse correction with the approximate inverse Bc, post-smooth"""
        e = self.smooth(l, e0, g, self.nu1)
        e = e + self.Pm[l] @ Bc(self.Pm[l].T @ (g - self.K[l] @ e))
        return self.smooth(l, e, g, self.nu2)

    def approx(self, l, kind):
        """g -> correction on level l by the named schedule from zero"""
        if l == self.P.L - 1:
            return self.coarsest
        if kind == "V":
            return lambda g: self.two_grid(l, g, np.zeros_like(g), self.approx(l + 1, "V"))
        if kind == "W":
            inner = self.approx(l + 1, "W")
            M = lambda g: self.two_grid(l, g, np.zeros_like(g), inner)  # noqa: E731
            if l + 1 == self.P.L - 1:
                # two iterations of the cycle: e1 = M g, e2 = e1 + M (g - K e1) = (2M - M K M) g
                return lambda g: M(g) + M(g - self.K[l] @ M(g))
            return lambda g: M(g) + M(g - self.K[l] @ M(g))
        # F: an F-visit then a V-visit of the coarse problem:
        # e1 = MF g, e2 = e1 + MV (g - K e1)
        MF = lambda g: self.two_grid(l, g, np.zeros_like(g), self.approx(l + 1, "F"))  # noqa: E731
        MV = lambda g: self.two_grid(l, g, np.zeros_like(g), self.approx(l + 1, "V"))  # noqa: E731
        return lambda g: MF(g) + MV(g - self.K[l] @ MF(g))


def _coarse_map(Dn, l, kind):
    """The approximate inverse the schedule applies to the level-(l+1) problem."""
    if l + 1 == Dn.P.L - 1:
        return Dn.coarsest
    if kind == "V":
        return Dn.approx(l + 1, "V")
    if kind == "W":
        M = Dn.approx(l + 1, "V") if l + 2 == Dn.P.L - 1 else None
        if M is None:
            inner = _coarse_map(Dn, l + 1, "W")
            M = lambda g: Dn.two_grid(l + 1, g, np.zeros_like(g), inner)  # noqa: E731
        return lambda g: M(g) + M(g - Dn.K[l + 1] @ M(g))
    MF = lambda g: Dn.two_grid(l + 1, g, np.zeros_like(g), _coarse_map(Dn, l + 1, "F"))  # noqa: E731
    MV = Dn.approx(l + 1, "V")
    return lambda g: MF(g) + MV(g - Dn.K[l + 1] @ MF(g))


@pytest.mark.parametrize("L", [3, 4])
@pytest.mark.parametrize("kind", ["W", "F"])
def test_w_and_f_cycles_against_dense_iterated_coarse_solves(kind, L):
    P = S.Problem(_rand_vox(16, 31, 0.5) if L == 4 else _rand_vox(8, 30, 0.5), L)
    lam = [P.lambda_max(l) for l in range(L)]
    sm = {"kind": "jacobi", "omega": [1.0 / x for x in lam]}
    n = P.levels[0].n_n
    u0 = random_vectors(n, 18, 2).reshape(n, 6, 3)
    out = S.cycle(P, P.f, u0, sm, nu1=2, nu2=1, kind=kind)
    Dn = Dense(P, sm, 2, 1)
    F = ops.to_dofs(P.f)
    ref = Dn.two_grid(0, F, ops.to_dofs(u0), _coarse_map(Dn, 0, kind))
    assert np.abs(ops.to_dofs(out) - ref).max() <= 1e-10 * np.abs(ref).max()
    # and the schedules really differ from the V-cycle on these hierarchies
    v = S.cycle(P, P.f, u0, sm, nu1=2, nu2=1, kind="V")
    assert np.abs(v - out).max() > 1e-6 * np.abs(v).max()


def test_v_schedule_is_the_vcycle(prob8):
    P = prob8
    sm = S.default_smoother(P, "chebyshev")
    n = [lv.n_n for lv in P.levels]
    u0 = random_vectors(n[0], 18, 2).reshape(n[0], 6, 3)
    e = [None, random_vectors(n[1], 18, 3).reshape(n[1], 6, 3), None]
    a = S.cycle(P, P.f, u0, sm, 2, 2, e_init=e, kind="V")
    b = S.vcycle(P, P.f, u0, sm, 2, 2, e_init=e)
    assert np.abs(a - b).max() == 0.0


def test_w_cycle_injection_starts_the_coarse_iterations():
    """Stage-wise injection at 3 levels: e2 = e_hat + (2M - M K M)(g - K e_hat)."""
    P = S.Problem(_rand_vox(8, 33, 0.5), 3)
    lam = [P.lambda_max(l) for l in range(3)]
    sm = {"kind": "jacobi", "omega": [1.0 / x for x in lam]}
    n = [lv.n_n for lv in P.levels]
    u0 = random_vectors(n[0], 18, 5).reshape(n[0], 6, 3)
    eh = random_vectors(n[1], 18, 6).reshape(n[1], 6, 3)
    out = S.cycle(P, P.f, u0, sm, 2, 2, e_init=[None, eh, None], kind="W")
    Dn = Dense(P, sm, 2, 2)
    M = Dn.approx(1, "V")
    E = ops.to_dofs(eh)

    def Bc(g):
        e1 = E + M(g - Dn.K[1] @ E)
        return e1 + M(g - Dn.K[1] @ e1)

    ref = Dn.two_grid(0, ops.to_dofs(P.f), ops.to_dofs(u0), Bc)
    assert np.abs(ops.to_dofs(out) - ref).max() <= 1e-10 * np.abs(ref).max()


def test_w_cycle_is_symmetric():
    P = S.Problem(gyroid_sheet(16, 3, 0.45), 4)
    sm = S.default_smoother(P, "chebyshev")
    n = P.levels[0].n_n
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((n, 6, 3)), rng.standard_normal((n, 6, 3))
    for v in (x, y):
        v -= v.mean(0, keepdims=True)
        v[0] = 0.0
    Wx = S.cycle(P, x, np.zeros_like(x), sm, 2, 2, kind="W")
    Wy = S.cycle(P, y, np.zeros_like(y), sm, 2, 2, kind="W")
    a, b = (Wx * y).sum(), (x * Wy).sum()
    assert abs(a - b) <= 1e-10 * max(abs(a), abs(b))


# ---------------------------------------------------------------- node-connected components

def _bfs_components(act):
    N = act.shape[0]
    todo = {(z, y, x) for z, y, x in zip(*np.nonzero(act))}
    count = 0
    while todo:
        count += 1
        q = deque([todo.pop()])
        while q:
            z, y, x = q.popleft()
            for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
                nb = ((z + dz) % N, (y + dy) % N, (x + dx) % N)
                if nb in todo:
                    todo.remove(nb)
                    q.append(nb)
    return count


def test_components_closed_cases():
    a = np.zeros((8, 8, 8), dtype=np.uint8)
    assert H.node_components(a) == 0
    a[1, 1, 1] = 1
    assert H.node_components(a) == 1
    a[4, 4, 4] = 1
    assert H.node_components(a) == 2
    a[2, 2, 2] = 1  # touches (1,1,1) at a corner node only
    assert H.node_components(a) == 2
    a[3, 3, 3] = 1  # corner chain (1,1,1)-(2,2,2)-(3,3,3)-(4,4,4)
    assert H.node_components(a) == 1
    b = np.zeros((8, 8, 8), dtype=np.uint8)
    b[0, 0, 0] = b[7, 7, 7] = 1  # neighbours across the periodic wrap
    assert H.node_components(b) == 1
    b[0, 0, 0] = 0
    b[5, 0, 0] = 1
    assert H.node_components(b) == 2
    # two parallel slabs with a void gap of one voxel: separate; a gap of zero: one
    from gmt_inputs import laminate
    two = laminate(8, 2, axis=2) | np.roll(laminate(8, 2, axis=2), 4, axis=0)
    assert H.node_components(two) == 2
    assert H.node_components(gyroid_sheet(16, 1, 0.3)) == 1


@pytest.mark.parametrize("seed", range(6))
def test_components_brute_force(seed):
    act = _rand_vox(6, 100 + seed, 0.08 + 0.03 * seed)
    assert H.node_components(act) == _bfs_components(act.astype(bool))


# ---------------------------------------------------------------- physics loss, dense

@pytest.mark.parametrize("lam", [0.0, 0.37])
def test_physics_loss_dense(lam):
    """log10(||f - K Vcycle(u_hat, e_hat)||_2 + 1e-12) + lam sum_{m,d} (sum_i u_i)^2, dense."""
    P = S.Problem(_rand_vox(8, 22), 3)
    lamv = [P.lambda_max(l) for l in range(3)]
    sm = {"kind": "jacobi", "omega": [1.0 / x for x in lamv]}
    n = [lv.n_n for lv in P.levels]
    uh = random_vectors(n[0], 18, 40).reshape(n[0], 6, 3) + 0.2  # nonzero mean: penalty active
    eh = random_vectors(n[1], 18, 41).reshape(n[1], 6, 3)
    Lval, u1 = onn.physics_loss(P, uh, [None, eh, None], sm, 2, 2, lam)
    Dn = Dense(P, sm, 2, 2)
    E = ops.to_dofs(eh)
    # level 2 is entered once, from the injected e_hat^2, and solved by its two-grid cycle
    Bc = lambda g: Dn.two_grid(1, g, E, Dn.coarsest)  # noqa: E731
    ref_u = Dn.two_grid(0, ops.to_dofs(P.f), ops.to_dofs(uh), Bc)
    R = ops.to_dofs(P.f) - Dn.K[0] @ ref_u
    sums = ref_u.reshape(n[0], 3, 6).sum(axis=0)  # per DOF component and case
    ref = np.log10(np.sqrt((R ** 2).sum()) + 1e-12) + lam * (sums ** 2).sum()
    assert np.abs(ops.to_dofs(u1) - ref_u).max() <= 1e-10 * np.abs(ref_u).max()
    assert abs(Lval - ref) <= 1e-12 * max(1.0, abs(ref))
