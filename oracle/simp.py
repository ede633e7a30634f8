"""SIMP inverse homogenization (App. F.3), by definition, in FP64.

Test infrastructure: only tests/, the smoke check and the bench's CPU
baseline use this package; the GPU library never does.

* ``DensityProblem``: the periodic cell problem of a density field rho
  (one value per voxel element).  Elements with rho_e > prune are active;
  their tensor is C_e = (rho_min + rho_e^p) C0 (eq. ch), i.e. the element
  matrix s_e K0 with s_e = rho_min + rho_e^p.  The hierarchy, Galerkin
  operators, smoothers and PCG are the ones of ``solve.Problem`` with these
  per-element fine matrices; the load is f = sum_e s_e A_e^T K0 X0.
* ``homogenize``: C_H = 1/|Omega| sum_e s_e d_e^T K0 d_e with d_e = X0 - u_e.
* ``sensitivities``: dC_H[i][j]/d rho_e = p rho_e^{p-1} / |Omega| d_e^(i)T K0 d_e^(j)
  (App. F.3; the u-dependence drops out because u solves the cell problem);
  zero for inactive elements.
* ``objective``: J(C_H) for the three targets of App. F.3 on the compliance
  S = C_H^{-1} (mean of S00, S11, S22; mean of S33, S44, S55; sum of the
  upper-left 3x3 block), and G = dJ/dC_H = -S W S with W = dJ/dS.
* ``filter_sensitivity``: the standard sensitivity filter (the paper names
  it without a formula; reading: the mesh-independence filter
  dc~_e = sum_f H_ef rho_f dc_f / (max(gamma, rho_e) sum_f H_ef) with
  H_ef = max(0, r_min - |x_e - x_f|) over periodic distances, gamma = 1e-3).
* ``oc_update``: Optimality Criteria with move limits (reading: the standard
  heuristic rho_new = clip(rho (-dc / lam)^eta, rho +/- move, [rho_lo, 1])
  with eta = 1/2 and lam by bisection so that mean(rho_new) = v_f).
"""

from __future__ import annotations

import numpy as np

from . import hierarchy, operators as ops
from . import fem
from .solve import Problem


class DensityProblem(Problem):
    def __init__(self, rho, levels: int, p: float = 3.0, rho_min: float = 1e-3, prune: float = 0.0,
                 physics: str = "elastic", E: float = 1.0, nu: float = 0.3, kappa: float = 1.0):
        rho = np.asarray(rho, dtype=np.float64)
        self.rho_field = rho
        self.p, self.rho_min, self.prune = float(p), float(rho_min), float(prune)
        self.physics = physics
        self.Ke, self.X0, self.d = fem.element(physics, E, nu, kappa)
        self.c = self.X0.shape[1]
        self.N = rho.shape[0]
        self.levels = hierarchy.build((rho > prune).astype(np.uint8), levels)
        self.L = levels
        lv = self.levels[0]
        self.rho = rho.ravel()[lv.elem_lin]  # per active element, element order
        self.scale = self.rho_min + self.rho ** self.p
        self.mats = [self.scale[:, None, None] * self.Ke[None, :, :]]
        for l in range(1, levels):
            self.mats.append(ops.coarse_element_matrices(self.levels[l - 1], self.mats[l - 1], self.levels[l],
                                                         self.d))
        self.K = [ops.assemble(lv_, m, self.d) for lv_, m in zip(self.levels, self.mats)]
        self.P = [ops.prolongation_matrix(self.levels[l], self.levels[l + 1].n_n, self.d)
                  for l in range(levels - 1)]
        self.D = [ops.diagonal(lv_, m, self.d) for lv_, m in zip(self.levels, self.mats)]
        self.f = load_vector(lv, self.Ke, self.X0, self.scale)
        self._coarse = None


def load_vector(level, Ke, X0, scale) -> np.ndarray:
    """f = sum_e s_e A_e^T K0 X0."""
    d = Ke.shape[0] // 8
    c = X0.shape[1]
    fe = (Ke @ X0).reshape(8, d, c).transpose(0, 2, 1)  # [8, c, d]
    f = np.zeros((level.n_n, c, d))
    for a in range(8):
        np.add.at(f, level.elem_nodes[:, a], scale[:, None, None] * fe[a][None])
    return f


def element_energies(prob: DensityProblem, u) -> np.ndarray:
    """E_e[i][j] = d_e^(i)T K0 d_e^(j), d_e = X0 - u_e, per active element [n_e, c, c]."""
    W = prob.X0[None, :, :] - ops._gather(u, prob.levels[0].elem_nodes)  # [n_e, 8d, c]
    return np.einsum("eic,ij,ejk->eck", W, prob.Ke, W)


def homogenize(prob: DensityProblem, u) -> np.ndarray:
    """C_H = 1/|Omega| sum_e s_e d_e^T K0 d_e (App. F.1 with C_e = s_e C0)."""
    return np.einsum("e,eck->ck", prob.scale, element_energies(prob, u)) / float(prob.N ** 3)


def sensitivities(prob: DensityProblem, u) -> np.ndarray:
    """dC_H/d rho_e on the dense grid [N^3, c, c] (App. F.3), zero where inactive."""
    Ee = element_energies(prob, u)
    g = prob.p * prob.rho ** (prob.p - 1.0) / float(prob.N ** 3)
    out = np.zeros((prob.N ** 3, prob.c, prob.c))
    out[prob.levels[0].elem_lin] = g[:, None, None] * Ee
    return out


OBJECTIVES = ("young", "shear", "bulk")


def objective(CH, kind: str):
    """J and G = dJ/dC_H for the App. F.3 targets (compliance S = C_H^-1)."""
    S = np.linalg.inv(CH)
    W = np.zeros_like(S)
    if kind == "young":
        W[[0, 1, 2], [0, 1, 2]] = 1.0 / 3.0
    elif kind == "shear":
        W[[3, 4, 5], [3, 4, 5]] = 1.0 / 3.0
    elif kind == "bulk":
        W[:3, :3] = 1.0
    else:
        raise ValueError(kind)
    J = float((W * S).sum())
    G = -S.T @ W @ S.T  # d tr(W^T S) = -tr(W^T S dC S)
    return J, G


def filter_sensitivity(rho, dc, rmin: float, gamma: float = 1e-3) -> np.ndarray:
    """Mesh-independence sensitivity filter with a periodic cone kernel of radius rmin (voxels)."""
    N = rho.shape[0]
    r = int(np.ceil(rmin)) - 1
    num = np.zeros_like(dc)
    den = np.zeros_like(dc)
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                h = rmin - np.sqrt(dx * dx + dy * dy + dz * dz)
                if h <= 0:
                    continue
                sh = (-dz, -dy, -dx)  # value of neighbour (z+dz, y+dy, x+dx) at (z, y, x)
                num += h * np.roll(rho * dc, sh, axis=(0, 1, 2))
                den += h
    del N
    return num / (np.maximum(gamma, rho) * den)


def oc_update(rho, dc, volfrac: float, move: float = 0.2, eta: float = 0.5, rho_lo: float = 1e-3,
              tol: float = 1e-10):
    """Optimality Criteria step with move limits; dc = dJ/drho (<= 0 for a stiffening target).
    Returns (rho_new, lam)."""
    lo, hi = 0.0, 1e9
    B = np.maximum(-dc, 0.0)
    rho_new = rho
    lam = hi
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        cand = rho * (B / lam) ** eta
        rho_new = np.clip(cand, np.maximum(rho_lo, rho - move), np.minimum(1.0, rho + move))
        if rho_new.mean() > volfrac:
            lo = lam
        else:
            hi = lam
        if hi - lo <= tol * max(hi, 1e-30):
            break
    return rho_new, lam
