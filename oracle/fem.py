"""Hex8 voxel element quantities (App. F.1 elasticity, App. F.2 heat conduction).

All functions return float64 numpy arrays for a unit cube voxel ``[0,1]^3``.
The voxel size drops out of the effective tensors (K_e scales with h, the
affine field with h, |Omega| with h^3), so h = 1 throughout.
"""

from __future__ import annotations

import itertools

import numpy as np

CORNERS = np.array([(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)], dtype=np.int64)


def isotropic_C(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic stiffness, Voigt (11,22,33,23,13,12), engineering shear."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    G = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2.0 * G
    C[3, 3] = C[4, 4] = C[5, 5] = G
    return C


def _shape_grad(xi):
    """dN_a/dx_j at a point of the unit cube, shape (8, 3)."""
    g = np.zeros((8, 3))
    for a, (ax, ay, az) in enumerate(CORNERS):
        fx = xi[0] if ax else 1.0 - xi[0]
        fy = xi[1] if ay else 1.0 - xi[1]
        fz = xi[2] if az else 1.0 - xi[2]
        sx, sy, sz = (1.0 if ax else -1.0), (1.0 if ay else -1.0), (1.0 if az else -1.0)
        g[a] = (sx * fy * fz, fx * sy * fz, fx * fy * sz)
    return g


def strain_B(xi) -> np.ndarray:
    """6x24 strain-displacement matrix at xi (DOF 3a+d)."""
    g = _shape_grad(xi)
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = g[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1] = gz  # gamma_23 = du2/dz + du3/dy
        B[3, c + 2] = gy
        B[4, c + 0] = gz  # gamma_13 = du1/dz + du3/dx
        B[4, c + 2] = gx
        B[5, c + 0] = gy  # gamma_12 = du1/dy + du2/dx
        B[5, c + 1] = gx
    return B


def _gauss2():
    p = 0.5 / np.sqrt(3.0)
    pts = (0.5 - p, 0.5 + p)
    return [(np.array(q), 0.125) for q in itertools.product(pts, pts, pts)]


def Ke_elastic(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """K_e = int B^T C0 B over the voxel, 2x2x2 Gauss (exact for trilinear B)."""
    C = isotropic_C(E, nu)
    K = np.zeros((24, 24))
    for xi, w in _gauss2():
        B = strain_B(xi)
        K += w * B.T @ C @ B
    return K


def Ke_elastic_tensor(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """Same K_e built a second, independent way.

    Uses the 4th-order tensor C_ijkl = lam d_ij d_kl + G (d_ik d_jl + d_il d_jk)
    and the exact 1D integrals of products of linear shape functions and their
    derivatives, K[3a+i, 3b+j] = sum_kl C_ikjl int dN_a/dx_k dN_b/dx_l.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    G = E / (2.0 * (1.0 + nu))
    d = np.eye(3)
    Ct = (lam * np.einsum("ij,kl->ijkl", d, d)
          + G * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))

    def mass1(p, q):
        return 1.0 / 3.0 if p == q else 1.0 / 6.0

    def stiff1(p, q):
        return (2 * p - 1) * (2 * q - 1) * 1.0

    def mixed1(p_deriv, q_val):  # int phi'_p phi_q
        return (2 * p_deriv - 1) * 0.5

    def integral(a, b, k, l):
        val = 1.0
        for ax in range(3):
            pa, pb = CORNERS[a][ax], CORNERS[b][ax]
            if ax == k and ax == l:
                val *= stiff1(pa, pb)
            elif ax == k:
                val *= mixed1(pa, pb)
            elif ax == l:
                val *= mixed1(pb, pa)
            else:
                val *= mass1(pa, pb)
        return val

    K = np.zeros((24, 24))
    for a in range(8):
        for b in range(8):
            I = np.array([[integral(a, b, k, l) for l in range(3)] for k in range(3)])
            for i in range(3):
                for j in range(3):
                    K[3 * a + i, 3 * b + j] = np.sum(Ct[i, :, j, :] * I)
    return K


def X0_elastic() -> np.ndarray:
    """24x6 nodal values of the affine fields of the six unit macro-strains.

    This is the paper's x0 = K_e^{-1} f_e read as the affine displacement that
    carries a uniform unit strain (K_e is singular, any rigid offset is
    annihilated by K_e).  Modes (11,22,33,23,13,12) with engineering shear:
    u = (x,0,0), (0,y,0), (0,0,z), (0,z/2,y/2), (z/2,0,x/2), (y/2,x/2,0).
    """
    X = np.zeros((24, 6))
    for a, (x, y, z) in enumerate(CORNERS):
        c = 3 * a
        X[c + 0, 0] = x
        X[c + 1, 1] = y
        X[c + 2, 2] = z
        X[c + 1, 3] = 0.5 * z
        X[c + 2, 3] = 0.5 * y
        X[c + 0, 4] = 0.5 * z
        X[c + 2, 4] = 0.5 * x
        X[c + 0, 5] = 0.5 * y
        X[c + 1, 5] = 0.5 * x
    return X


def Ke_thermal(kappa: float = 1.0) -> np.ndarray:
    """8x8 conductivity matrix kappa * int grad N_a . grad N_b (2x2x2 Gauss)."""
    K = np.zeros((8, 8))
    for xi, w in _gauss2():
        g = _shape_grad(xi)
        K += w * kappa * g @ g.T
    return K


def X0_thermal() -> np.ndarray:
    """8x3 nodal values of T0^(i) = x_i (unit gradient along axis i)."""
    return CORNERS.astype(np.float64).copy()


def element(physics: str, E: float = 1.0, nu: float = 0.3, kappa: float = 1.0):
    """(K_e, X0, d) for 'elastic' (24x24, 24x6, 3) or 'thermal' (8x8, 8x3, 1)."""
    if physics == "elastic":
        return Ke_elastic(E, nu), X0_elastic(), 3
    if physics == "thermal":
        return Ke_thermal(kappa), X0_thermal(), 1
    raise ValueError(physics)


def base_tensor(physics: str, E: float = 1.0, nu: float = 0.3, kappa: float = 1.0):
    """C0 (6x6) or kappa0 * I (3x3)."""
    if physics == "elastic":
        return isotropic_C(E, nu)
    return kappa * np.eye(3)
