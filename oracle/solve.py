"""Smoothers, V-cycle (Alg. 1 / Alg. 2), PCG reference solve and the metrics (Sec. 5.2).

``Problem`` holds the hierarchy, the element matrices of every level and the
sparse Galerkin operators for one voxel cell.

* ``jacobi`` / ``chebyshev``: the smoothers S(K, u, f) used on every level.
  Weighted Jacobi is the paper's point-Jacobi row (smoother study); Chebyshev
  is the polynomial acceleration of the same D^{-1}K iteration on a given
  interval [lo, hi].
* ``coarse_solve``: exact solve at level L of the pinned coarsest operator
  (the lowest-id node's DOFs replaced by identity rows/columns, zero RHS).
* ``gauss_seidel``: the 8-colour Gauss-Seidel / SOR smoother of Sec. 4.6
  (parallel smoothing): nodes coloured by the parity of their coordinates,
  the colours updated one after the other with u_i += omega D_i^-1 r_i.
* ``vcycle``: Alg. 2 -- Alg. 1 with u^1 <- u_hat^1 and u^{l+1} <- e_hat^{l+1}
  instead of 0 when corrections are given.
* ``cycle``: the same recursion with the W- and F-schedules of the schedule
  study (Sec. 6.3): a coarse level is visited twice (W) or by an F-cycle
  followed by a V-cycle (F) per visit of the level above it.
* ``pcg``: CG on the pinned fine system (gauge: lowest-id node fixed),
  preconditioned by Jacobi or by the V-cycle, stopped on the true residual.
* ``relative_residual``: r_m = ||f_m - K u_m||_2 / ||f_m||_2 per load case.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem, hierarchy, operators as ops


class Problem:
    def __init__(self, voxels, levels: int, physics: str = "elastic",
                 E: float = 1.0, nu: float = 0.3, kappa: float = 1.0):
        self.physics = physics
        self.Ke, self.X0, self.d = fem.element(physics, E, nu, kappa)
        self.c = self.X0.shape[1]
        self.N = voxels.shape[0]
        self.levels = hierarchy.build(voxels, levels)
        self.L = levels
        self.mats = ops.level_matrices(self.levels, self.Ke, self.d)
        self.K = [ops.assemble(lv, m, self.d) for lv, m in zip(self.levels, self.mats)]
        self.P = [ops.prolongation_matrix(self.levels[l], self.levels[l + 1].n_n, self.d)
                  for l in range(levels - 1)]
        self.D = [ops.diagonal(lv, m, self.d) for lv, m in zip(self.levels, self.mats)]
        self.f = ops.load_vector(self.levels[0], self.Ke, self.X0)
        self._coarse = None

    # -- operators on [n, c, d] vectors (sparse products of the assembled K)
    def Kmul(self, l: int, u: np.ndarray) -> np.ndarray:
        return ops.from_dofs(self.K[l] @ ops.to_dofs(u), self.d)

    def lambda_max(self, l: int) -> float:
        """Largest eigenvalue of D^{-1} K on level l (symmetric form D^-1/2 K D^-1/2)."""
        s = 1.0 / np.sqrt(self.D[l].ravel())
        A = self.K[l].multiply(s[:, None]).multiply(s[None, :]).tocsr()
        return float(spla.eigsh(A, k=1, which="LA", return_eigenvectors=False, tol=1e-8)[0])

    def coarse_factor(self):
        if self._coarse is None:
            KL = self.K[-1].toarray()
            d = self.d
            p = hierarchy.pinned_node(self.levels[-1])
            pin = np.arange(p * d, (p + 1) * d)
            KL[pin, :] = 0.0
            KL[:, pin] = 0.0
            KL[pin, pin] = 1.0
            self._coarse = (sla.cho_factor(KL, lower=True), pin)
        return self._coarse


def jacobi(prob: Problem, l: int, u, f, nu: int, omega: float):
    Dinv = 1.0 / prob.D[l][:, None, :]
    for _ in range(nu):
        u = u + omega * Dinv * (f - prob.Kmul(l, u))
    return u


def chebyshev(prob: Problem, l: int, u, f, nu: int, lo: float, hi: float):
    """Degree-nu Chebyshev iteration for D^{-1}K on [lo, hi] (three-term recurrence)."""
    if nu <= 0:
        return u
    Dinv = 1.0 / prob.D[l][:, None, :]
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    dvec = Dinv * (f - prob.Kmul(l, u)) / theta
    u = u + dvec
    for _ in range(nu - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        r = f - prob.Kmul(l, u)
        dvec = rho_new * rho * dvec + (2.0 * rho_new / delta) * Dinv * r
        u = u + dvec
        rho = rho_new
    return u


def colours(level) -> np.ndarray:
    """Colour of every active node: (x mod 2) + 2 (y mod 2) + 4 (z mod 2) (Sec. 4.6).

    Two nodes of one colour differ by an even amount along every axis, so on a
    level with an even number of voxels per axis (periodic wrap included) they
    never share an element: each colour class is free of couplings.
    """
    N = level.N
    lin = level.node_lin
    return (lin % N) % 2 + 2 * (((lin // N) % N) % 2) + 4 * ((lin // (N * N)) % 2)


def gauss_seidel(prob: Problem, l: int, u, f, nu: int, omega: float, reverse: bool = False):
    """nu sweeps of the 8-colour Gauss-Seidel smoother (SOR with weight omega), Sec. 4.6.

    One sweep visits the colours 0..7 (7..0 when ``reverse``); the nodes of a
    colour are updated together, u_i += omega D_i^-1 r_i, from the residual
    r = f - K u of the current iterate (so a colour sees the updates of the
    colours before it).  D is the diagonal of K.  The backward sweep is the
    adjoint of the forward one in the K inner product, so a cycle with forward
    pre- and backward post-smoothing is a symmetric preconditioner.
    """
    col = colours(prob.levels[l])
    Dinv = 1.0 / prob.D[l][:, None, :]
    order = range(7, -1, -1) if reverse else range(8)
    u = np.array(u, dtype=np.float64)
    for _ in range(nu):
        for c in order:
            m = col == c
            if not m.any():
                continue
            r = f - prob.Kmul(l, u)
            u[m] = u[m] + omega * Dinv[m] * r[m]
    return u


def coarse_solve(prob: Problem, f):
    (cf, pin) = prob.coarse_factor()
    F = ops.to_dofs(f).copy()
    F[pin, :] = 0.0
    return ops.from_dofs(sla.cho_solve(cf, F), prob.d)


def smooth(prob, l, u, f, nu, sm, post: bool = False):
    """Pre- (post=False) or post-smoothing on level l; Gauss-Seidel runs its colours
    forward before and backward after the coarse correction."""
    if sm["kind"] == "jacobi":
        return jacobi(prob, l, u, f, nu, sm["omega"][l])
    if sm["kind"] == "gs":
        return gauss_seidel(prob, l, u, f, nu, sm["omega"][l], reverse=post)
    return chebyshev(prob, l, u, f, nu, sm["lo"][l], sm["hi"][l])


def vcycle(prob: Problem, f, u, sm, nu1: int = 2, nu2: int = 2, e_init=None):
    """One V-cycle (Alg. 2; Alg. 1 when ``e_init`` is None and u = 0).

    ``sm``: {"kind": "jacobi", "omega": [per level]} or
            {"kind": "chebyshev", "lo": [...], "hi": [...]}.
    ``e_init``: optional list indexed by level (entries for levels 1..L-1,
    0-based) of injected coarse initial corrections.
    """
    L = prob.L
    fl = [None] * L
    ul = [None] * L
    fl[0], ul[0] = f, u
    for l in range(L - 1):
        ul[l] = smooth(prob, l, ul[l], fl[l], nu1, sm)
        r = fl[l] - prob.Kmul(l, ul[l])
        fl[l + 1] = ops.restrict(prob.levels[l], r, prob.levels[l + 1].n_n)
        if e_init is not None and e_init[l + 1] is not None:
            ul[l + 1] = np.array(e_init[l + 1], dtype=np.float64)
        else:
            ul[l + 1] = np.zeros_like(fl[l + 1])
    ul[L - 1] = coarse_solve(prob, fl[L - 1])
    for l in range(L - 2, -1, -1):
        ul[l] = ul[l] + ops.prolong(prob.levels[l], ul[l + 1])
        ul[l] = smooth(prob, l, ul[l], fl[l], nu2, sm, post=True)
    return ul[0]


def cycle(prob: Problem, f, u, sm, nu1: int = 2, nu2: int = 2, e_init=None, kind: str = "V"):
    """One multigrid cycle with the V-, W- or F-schedule (Sec. 6.3 schedule study).

    Visiting level l: pre-smooth, restrict the residual, approximately solve the
    coarse correction problem on level l+1 starting from zero, prolong and add,
    post-smooth.  The coarse problem is treated by one visit (V), two visits in
    a row (W), or an F-visit followed by a V-visit (F); the coarsest level is
    solved exactly (so a repeated visit there is skipped: it changes nothing).
    Injection (Alg. 2 with several stages): e_hat^{l+1} replaces the zero start
    of level l+1 at its first entry in the cycle only; later entries start
    from zero and repeated visits continue from the current iterate.
    """
    if kind not in ("V", "W", "F"):
        raise ValueError("kind must be V, W or F")
    L = prob.L
    entered = [False] * L

    def visit(l, fl, ul, how):
        if l == L - 1:
            return coarse_solve(prob, fl)
        ul = smooth(prob, l, ul, fl, nu1, sm)
        r = fl - prob.Kmul(l, ul)
        fc = ops.restrict(prob.levels[l], r, prob.levels[l + 1].n_n)
        if e_init is not None and e_init[l + 1] is not None and not entered[l + 1] and l + 1 < L - 1:
            uc = np.array(e_init[l + 1], dtype=np.float64)
        else:
            uc = np.zeros_like(fc)
        entered[l + 1] = True
        if how == "V":
            uc = visit(l + 1, fc, uc, "V")
        elif how == "W":
            uc = visit(l + 1, fc, uc, "W")
            if l + 1 < L - 1:
                uc = visit(l + 1, fc, uc, "W")
        else:
            uc = visit(l + 1, fc, uc, "F")
            if l + 1 < L - 1:
                uc = visit(l + 1, fc, uc, "V")
        ul = ul + ops.prolong(prob.levels[l], uc)
        return smooth(prob, l, ul, fl, nu2, sm, post=True)

    return visit(0, f, np.array(u, dtype=np.float64), kind)


def default_smoother(prob: Problem, kind: str = "chebyshev", lo_frac: float = 1.0 / 30.0,
                     hi_frac: float = 1.1, omega: float = 1.0):
    if kind == "gs":
        return {"kind": "gs", "omega": [omega] * prob.L}
    lam = [prob.lambda_max(l) for l in range(prob.L)]
    if kind == "jacobi":
        return {"kind": "jacobi", "omega": [4.0 / (3.0 * x) for x in lam]}
    return {"kind": "chebyshev", "lo": [lo_frac * x for x in lam], "hi": [hi_frac * x for x in lam]}


NULL_LOAD = 1e-12


def relative_residual(prob: Problem, u) -> np.ndarray:
    """||f_m - K u_m|| / ||f_m|| per case (Sec. 5.2), unpinned K and full f.

    A case whose load vanishes by symmetry (||f_m|| at most 1e-12 of the
    largest case, e.g. in-plane modes of a laminate) is normalised by the
    largest case's ||f|| instead, so rounding noise in a zero load is not
    reported as divergence.
    """
    r = prob.f - prob.Kmul(0, u)
    num = np.sqrt((r ** 2).sum(axis=(0, 2)))
    den = np.sqrt((prob.f ** 2).sum(axis=(0, 2)))
    return num / np.where(den <= NULL_LOAD * den.max(), den.max(), den)


def zero_load(prob: Problem) -> bool:
    """Every case's load is rounding noise (uniform solid): max ||f_m|| <= 1e-12 ||f_e||_F sqrt(n_e)."""
    fmax = np.sqrt((prob.f ** 2).sum(axis=(0, 2))).max()
    fe = prob.Ke @ prob.X0
    return fmax <= 1e-12 * np.linalg.norm(fe) * np.sqrt(prob.levels[0].n_e)


def pcg(prob: Problem, tol: float = 1e-11, maxit: int = 20000, precond: str = "vcycle",
        sm=None, nu: int = 2, kind: str = "V"):
    """Zero-initial-guess PCG on the pinned fine system, all load cases at once.

    Pinned system: rows/columns of the gauge node's DOFs replaced by identity,
    RHS zeroed there.  ``kind`` selects the cycle of the preconditioner (V or
    W: both symmetric).  Stops when every case's true relative residual
    ||f - K u|| / ||f|| (unpinned K, full f) is <= tol.  Returns (u, iters).
    """
    d = prob.d
    p = hierarchy.pinned_node(prob.levels[0])
    mask = np.ones((prob.levels[0].n_n, 1, d))
    mask[p] = 0.0
    f = prob.f * mask
    if precond == "vcycle" and sm is None:
        sm = default_smoother(prob)
    Dinv = 1.0 / prob.D[0][:, None, :]

    def A(v):
        return mask * prob.Kmul(0, mask * v) + (1.0 - mask) * v

    def M(r):
        if precond == "jacobi":
            return mask * Dinv * r
        if kind == "V":
            return mask * vcycle(prob, mask * r, np.zeros_like(r), sm, nu, nu)
        return mask * cycle(prob, mask * r, np.zeros_like(r), sm, nu, nu, kind=kind)

    u = np.zeros_like(f)
    if zero_load(prob):
        return u, 0
    r = f.copy()
    z = M(r)
    pvec = z.copy()
    rz = (r * z).sum(axis=(0, 2))
    for it in range(1, maxit + 1):
        q = A(pvec)
        pq = (pvec * q).sum(axis=(0, 2))
        alpha = np.where(pq != 0, rz / np.where(pq != 0, pq, 1.0), 0.0)
        u = u + alpha[None, :, None] * pvec
        r = r - alpha[None, :, None] * q
        if it % 5 == 0 or precond == "vcycle":
            if np.max(relative_residual(prob, u)) <= tol:
                return u, it
        z = M(r)
        rz_new = (r * z).sum(axis=(0, 2))
        beta = np.where(rz != 0, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        pvec = z + beta[None, :, None] * pvec
        rz = rz_new
    raise RuntimeError(f"oracle PCG did not reach {tol} in {maxit} iterations: "
                       f"{relative_residual(prob, u)}")


def direct_solve(prob: Problem):
    """Dense Cholesky of the pinned fine system (small cells only)."""
    d = prob.d
    K = prob.K[0].toarray()
    p = hierarchy.pinned_node(prob.levels[0])
    pin = np.arange(p * d, (p + 1) * d)
    K[pin, :] = 0.0
    K[:, pin] = 0.0
    K[pin, pin] = 1.0
    F = ops.to_dofs(prob.f).copy()
    F[pin, :] = 0.0
    return ops.from_dofs(sla.cho_solve(sla.cho_factor(K, lower=True), F), d)


def gauge_shift(prob: Problem, u):
    """Translate u so that the gauge node's value is zero (same K u, same C_H)."""
    p = hierarchy.pinned_node(prob.levels[0])
    return u - u[p][None, :, :]


def homogenize(prob: Problem, u) -> np.ndarray:
    """C_H (6x6) or kappa_H (3x3) by the element sum of App. F.1 / F.2:

    C_H[i, j] = 1/|Omega| sum_e (X0 - u_e)^(i)T K_e (X0 - u_e)^(j), |Omega| = N^3.
    """
    lv = prob.levels[0]
    W = prob.X0[None, :, :] - ops._gather(u, lv.elem_nodes)  # [n_e, 8d, c]
    CH = np.einsum("eic,ij,ejk->ck", W, prob.Ke, W)
    return CH / float(prob.N ** 3)
