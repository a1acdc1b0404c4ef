"""Finite elements: lumped mass, neo-Hookean tets, cubature (test infrastructure only).

Sec. 3.1: M u'' + f_int(u) = f_ext with M lumped to a diagonal.  The
internal force is f_int = +dE/du (so it appears with a plus sign next to
M u'').  The paper names no material law beyond "nonlinear elastic"; the
compressible neo-Hookean energy is used:
    Psi(F) = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,  J = det F
with first Piola stress P = dPsi/dF = mu (F - F^-T) + lam ln J F^-T and
tangent dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T.
Per tet, F = D_s D_m^-1 with D_s, D_m the edge matrices [x1-x0, x2-x0, x3-x0]
of the deformed and rest shapes; the element force is V_e dPsi/dx and the
element stiffness V_e d2Psi/dx2, obtained here by chaining the 9x9 tangent
with the 9x12 matrix dvec(F)/dx.

Cubature (Sec. 5): the reduced force and stiffness are sums over a subset C
of tets with non-negative weights w_e:
    f_r = sum_e w_e Jt_e^T f_e,   K_r = sum_e w_e Jt_e^T K_e Jt_e
with Jt_e the 12 rows of the stacked Jacobian [U, J] at the tet's vertices.
Full quadrature is C = all tets, w = 1.

Parity: pinned (central differences of energy and force, zero stress at
rest, linear-elastic stiffness at rest, force balance, rotation
invariance).
"""
from __future__ import annotations

import numpy as np


class InvertedElement(RuntimeError):
    pass


def lame(E: float, nu: float):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def edge_matrix(x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """(m, 3, 3) with columns x1 - x0, x2 - x0, x3 - x0."""
    p = x[tets]  # (m, 4, 3)
    return np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)


def rest_shape(X: np.ndarray, tets: np.ndarray):
    Dm = edge_matrix(X, tets)
    Bm = np.linalg.inv(Dm)
    Ve = np.linalg.det(Dm) / 6.0
    return Bm, Ve


def lumped_mass(tets: np.ndarray, Ve: np.ndarray, rho: float, n: int) -> np.ndarray:
    """Per-DOF diagonal: each vertex takes a quarter of each incident tet's mass."""
    mv = np.zeros(n)
    for c in range(4):
        np.add.at(mv, tets[:, c], rho * Ve / 4.0)
    return np.repeat(mv, 3)


def energy_density(F, mu, lam):
    J = np.linalg.det(F)
    lnJ = np.log(J)
    return 0.5 * mu * (np.einsum("...ij,...ij->...", F, F) - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def piola(F, mu, lam):
    J = np.linalg.det(F)
    FinvT = np.swapaxes(np.linalg.inv(F), -1, -2)
    return mu * (F - FinvT) + lam * np.log(J)[..., None, None] * FinvT


def tangent(F, mu, lam):
    """dvec(P)/dvec(F), (..., 9, 9), row-major vec: index 3*i + j for entry (i, j)."""
    J = np.linalg.det(F)
    lnJ = np.log(J)
    A = np.swapaxes(np.linalg.inv(F), -1, -2)  # F^-T
    I3 = np.eye(3)
    # C_ijkl = mu d_ik d_jl + (mu - lam lnJ) A_il A_kj + lam A_ij A_kl
    C = (mu * np.einsum("ik,jl->ijkl", I3, I3)[None]
         + (mu - lam * lnJ)[:, None, None, None, None] * np.einsum("...il,...kj->...ijkl", A, A)
         + lam * np.einsum("...ij,...kl->...ijkl", A, A))
    return C.reshape(F.shape[:-2] + (9, 9))


def dF_dx(Bm: np.ndarray) -> np.ndarray:
    """(m, 9, 12): d vec(F) / d x_e with x_e = (x0, x1, x2, x3), 3 coords each.

    F_ij = sum_k (x_{k+1} - x_0)_i Bm_kj.
    """
    m = Bm.shape[0]
    G = np.zeros((m, 4, 3))
    G[:, 1:, :] = Bm
    G[:, 0, :] = -Bm.sum(axis=1)
    D = np.zeros((m, 3, 3, 4, 3))  # (i, j, a, c)
    for i in range(3):
        D[:, i, :, :, i] = np.swapaxes(G, 1, 2)  # dF_ij/dx_{a,i} = G_aj
    return D.reshape(m, 9, 12)


def element_force_stiffness(X, tets, u, Bm, Ve, mu, lam):
    """Per-tet f_e (m, 12) and K_e (m, 12, 12) at displacement u (N,)."""
    x = X + u.reshape(-1, 3)
    F = edge_matrix(x, tets) @ Bm
    J = np.linalg.det(F)
    if np.any(J <= 0):
        raise InvertedElement(f"{int(np.sum(J <= 0))} tets with det F <= 0")
    P = piola(F, mu, lam).reshape(-1, 9)
    C = tangent(F, mu, lam)
    D = dF_dx(Bm)
    f = Ve[:, None] * np.einsum("mki,mk->mi", D, P)
    K = Ve[:, None, None] * np.einsum("mki,mkl,mlj->mij", D, C, D)
    return f, K


def tet_dofs(tets: np.ndarray) -> np.ndarray:
    """(m, 12) global DOF ids 3 v + c."""
    return (3 * tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)


def cubature_force_stiffness(X, tets, u, Jt, cub_ids, w, Bm, Ve, mu, lam):
    """f_int (N,), f_r (R,), K_r (R, R) summed over the cubature tets."""
    T = tets[cub_ids]
    f, K = element_force_stiffness(X, T, u, Bm[cub_ids], Ve[cub_ids], mu, lam)
    dofs = tet_dofs(T)
    Je = Jt[dofs]  # (c, 12, R)
    f_int = np.zeros(u.size)
    np.add.at(f_int, dofs.ravel(), (w[:, None] * f).ravel())
    fr = np.einsum("e,eir,ei->r", w, Je, f)
    Kr = np.einsum("e,eir,eij,ejs->rs", w, Je, K, Je)
    return f_int, fr, Kr


def total_energy(X, tets, u, Ve, Bm, mu, lam):
    x = X + u.reshape(-1, 3)
    F = edge_matrix(x, tets) @ Bm
    return float(np.sum(Ve * energy_density(F, mu, lam)))
