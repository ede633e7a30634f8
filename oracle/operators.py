"""Operators on the hierarchy (Sec. 4.6 EBE K.u and Galerkin projection; App. E.2 transfers).

* ``apply_K``: matrix-free element-by-element K u = sum_e A_e^T K_e A_e u
  (Sec. 4.6), for the shared voxel K_e on level 1 and the per-element coarse
  matrices on levels >= 2.
* ``coarse_element_matrices``: local Galerkin K_c = R_loc K_patch P_loc over
  the 2x2x2 child patch of every coarse element (Sec. 4.6), i.e.
  K_E = sum_{active child c} P_c^T K_c P_c with P_c the trilinear map from the
  coarse element's corners to the child's corners.
* ``assemble``: sparse global K from the same element definition (scipy), used
  by the solvers and by the Galerkin check K^{l+1} = P^T K^l P (Sec. 3.2).
* ``prolong`` / ``restrict``: App. E.2 weighted gather and its exact transpose
  (the paper's scatter-add; unscaled R = P^T).

Vectors have shape ``[n_n, c, d]`` (node, load case, DOF).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import CORNERS


def local_prolongation(child) -> np.ndarray:
    """8x8 scalar P_c[m, o]: weight of coarse corner o at corner m of child c."""
    P = np.zeros((8, 8))
    for m, cm in enumerate(CORNERS):
        xi = (np.asarray(child) + cm) / 2.0  # position inside the coarse cell, in {0, .5, 1}
        for o, co in enumerate(CORNERS):
            P[m, o] = np.prod(1.0 - np.abs(xi - co))
    return P


def coarse_element_matrices(fine_level, fine_mats, coarse_level, d: int) -> np.ndarray:
    """Per coarse element K_E = sum_{active children} P_c^T K_child P_c (FP64).

    ``fine_mats`` is either one (8d x 8d) matrix shared by all fine elements or
    an array [n_e_fine, 8d, 8d].
    """
    Nf = fine_level.N
    ne_c = coarse_level.n_e
    ex, ey, ez = (coarse_level.elem_lin % coarse_level.N,
                  (coarse_level.elem_lin // coarse_level.N) % coarse_level.N,
                  coarse_level.elem_lin // (coarse_level.N ** 2))
    fine_eid = np.full(Nf ** 3, -1, dtype=np.int64)
    fine_eid[fine_level.elem_lin] = np.arange(fine_level.n_e)
    fine_eid = fine_eid.reshape(Nf, Nf, Nf)
    shared = np.ndim(fine_mats) == 2
    KE = np.zeros((ne_c, 8 * d, 8 * d))
    I = np.eye(d)
    for c, (a, b, cc) in enumerate(CORNERS):
        Pc = np.kron(local_prolongation((a, b, cc)), I)  # (8d x 8d)
        child = fine_eid[2 * ez + cc, 2 * ey + b, 2 * ex + a]
        on = child >= 0
        if not on.any():
            continue
        Kc = fine_mats if shared else fine_mats[child[on]]
        contrib = Pc.T @ Kc @ Pc if shared else np.einsum("ji,ejk,kl->eil", Pc, Kc, Pc)
        KE[on] += contrib
    return KE


def level_matrices(levels, Ke: np.ndarray, d: int):
    """Element matrices of every level: level 0 the shared K_e, then Galerkin."""
    mats = [Ke]
    for l in range(1, len(levels)):
        mats.append(coarse_element_matrices(levels[l - 1], mats[l - 1], levels[l], d))
    return mats


def _gather(u, elem_nodes):
    """u [n, c, d] -> element vectors [n_e, 8d, c] (DOF 3a+d)."""
    n_e = elem_nodes.shape[0]
    ue = u[elem_nodes]  # [n_e, 8, c, d]
    return ue.transpose(0, 1, 3, 2).reshape(n_e, -1, u.shape[1])


def apply_K(level, mats, u: np.ndarray) -> np.ndarray:
    """y = sum_e A_e^T K_e A_e u, matrix-free (Sec. 4.6)."""
    n, c, d = u.shape
    Ue = _gather(u, level.elem_nodes)
    if np.ndim(mats) == 2:
        Ye = np.einsum("ij,ejc->eic", mats, Ue)
    else:
        Ye = np.einsum("eij,ejc->eic", mats, Ue)
    Ye = Ye.reshape(-1, 8, d, c).transpose(0, 1, 3, 2)  # [n_e, 8, c, d]
    y = np.zeros_like(u)
    np.add.at(y, level.elem_nodes.ravel(), Ye.reshape(-1, c, d))
    return y


def assemble(level, mats, d: int) -> sp.csr_matrix:
    """Sparse global K (DOF index d*i + dof) from the element definition."""
    n_e = level.n_e
    dof = (level.elem_nodes[:, :, None] * d + np.arange(d)[None, None, :]).reshape(n_e, 8 * d)
    rows = np.repeat(dof, 8 * d, axis=1).ravel()
    cols = np.tile(dof, (1, 8 * d)).ravel()
    vals = (np.broadcast_to(mats, (n_e, 8 * d, 8 * d)) if np.ndim(mats) == 2 else mats).reshape(-1)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(level.n_n * d, level.n_n * d))
    return K.tocsr()


def prolongation_matrix(level, n_coarse: int, d: int) -> sp.csr_matrix:
    """Sparse P (fine DOFs x coarse DOFs) from the App. E stencil tuple."""
    nz = level.prol_idx >= 0
    fi = np.nonzero(nz)[0]
    ci = level.prol_idx[nz]
    w = level.prol_w[nz]
    Ps = sp.coo_matrix((w, (fi, ci)), shape=(level.n_n, n_coarse)).tocsr()
    return sp.kron(Ps, sp.identity(d), format="csr")


def prolong(level, uc: np.ndarray) -> np.ndarray:
    """u_f(i) = sum_k W_ik u_c(I_ik)  (App. E.2 weighted gather)."""
    out = np.zeros((level.n_n,) + uc.shape[1:])
    for k in range(8):
        m = level.prol_idx[:, k] >= 0
        out[m] += level.prol_w[m, k][:, None, None] * uc[level.prol_idx[m, k]]
    return out


def restrict(level, rf: np.ndarray, n_coarse: int) -> np.ndarray:
    """r_c(j) = sum_{(i,k): I_ik = j} W_ik r_f(i)  (App. E.2, R = P^T)."""
    out = np.zeros((n_coarse,) + rf.shape[1:])
    for k in range(8):
        m = level.prol_idx[:, k] >= 0
        np.add.at(out, level.prol_idx[m, k], level.prol_w[m, k][:, None, None] * rf[m])
    return out


def diagonal(level, mats, d: int) -> np.ndarray:
    """diag(K) as [n_n, d] (the D of the Jacobi / Chebyshev smoother)."""
    out = np.zeros((level.n_n, d))
    for a in range(8):
        if np.ndim(mats) == 2:
            dg = np.broadcast_to(np.diag(mats)[a * d:(a + 1) * d], (level.n_e, d))
        else:
            dg = np.diagonal(mats, axis1=1, axis2=2)[:, a * d:(a + 1) * d]
        np.add.at(out, level.elem_nodes[:, a], dg)
    return out


def to_dofs(u: np.ndarray) -> np.ndarray:
    """[n, c, d] -> [n*d, c] (DOF-major matrix for sparse products)."""
    n, c, d = u.shape
    return u.transpose(0, 2, 1).reshape(n * d, c)


def from_dofs(U: np.ndarray, d: int) -> np.ndarray:
    nd, c = U.shape
    return U.reshape(nd // d, d, c).transpose(0, 2, 1).copy()


def load_vector(level, Ke: np.ndarray, X0: np.ndarray) -> np.ndarray:
    """f = sum_e A_e^T K_e X0 (App. F.1: f_e = int B^T C0 eps_bar = K_e X0)."""
    d = Ke.shape[0] // 8
    c = X0.shape[1]
    fe = (Ke @ X0).reshape(8, d, c).transpose(0, 2, 1)  # [8, c, d]
    f = np.zeros((level.n_n, c, d))
    for a in range(8):
        np.add.at(f, level.elem_nodes[:, a], np.broadcast_to(fe[a], (level.n_e, c, d)))
    return f


def apply_K_rows(level, mats, u: np.ndarray, rows) -> np.ndarray:
    """Rows ``rows`` of K u only: the element sum of Sec. 4.6 restricted to the
    elements that touch those nodes (for spot checks of very large cells)."""
    rows = np.asarray(rows, dtype=np.int64)
    touch = np.isin(level.elem_nodes, rows)
    elems = np.nonzero(touch.any(axis=1))[0]
    n, c, d = u.shape
    en = level.elem_nodes[elems]
    Ue = u[en].transpose(0, 1, 3, 2).reshape(len(elems), -1, c)
    M = mats if np.ndim(mats) == 2 else mats[elems]
    Ye = (np.einsum("ij,ejc->eic", M, Ue) if np.ndim(M) == 2 else np.einsum("eij,ejc->eic", M, Ue))
    Ye = Ye.reshape(-1, 8, d, c).transpose(0, 1, 3, 2)
    pos = {int(r): k for k, r in enumerate(rows)}
    out = np.zeros((len(rows), c, d))
    for e_loc in range(len(elems)):
        for a in range(8):
            k = pos.get(int(en[e_loc, a]))
            if k is not None:
                out[k] += Ye[e_loc, a]
    return out
