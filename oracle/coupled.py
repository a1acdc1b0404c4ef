"""Coupled multi-domain reduced simulation in FP64 (test infrastructure only).

Sec. 6.8 combines the reduced model with domain decomposition: the scene is
split into domains (the strings of the puffer ball, the branches of the
cactus), each with its own subspace u_d = U_d p_d + D_d(q_d), and the
domains are joined at their interfaces.  The paper names deformation
substructuring and multi-domain subspace methods for the coupling but gives
no equations for it.  The reading taken here is the multi-domain form in
which neighbouring domains own separate copies of their interface vertices
and the copies are tied by stiff zero-length springs:

    E_tie = kappa / 2 * sum over tied vertex pairs (a in domain d, b in c)
                        |(X_a + u_a) - (X_b + u_b)|^2

The total energy is the sum of the domain energies and E_tie, so the
coupled implicit-Euler step (Sec. 3.2) solves phi(r) = 0 for the stacked
coordinates r = [r_0; r_1; ...], where domain d's block is its own reduced
equation of motion (eq. our_equation_of_motion) with the tie force
f_tie = dE_tie/du_d entering wherever the internal force does, and the
Newton matrix (eq. system_mat) gains the tie stiffness:
    A_dd += dt^2 kappa Jt_d,T^T Jt_d,T,   A_dc = -dt^2 kappa Jt_d,T^T Jt_c,T
over the tied rows T of Jt = [U, J] of each domain.  The coupled system is
assembled whole and solved by dense LU with partial pivoting; Newton starts
from r = rbar in every domain and takes a fixed number of full steps.

Parity: pinned by the full-space reduction (U = identity on the free DOFs
of every domain, no decoder: the textbook implicit-Euler step of the
union mesh with its tie springs), by central differences of the coupled
phi, and by the decoupled limit kappa = 0.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import scipy.linalg

from .newton import Instance, State


class Coupled:
    """Domain 0 and domains 1.. tied to it.

    ties[k] (n_k, 2) int: pairs (vertex of domain k + 1, vertex of domain 0)
    whose copies are joined by a tie spring of stiffness kappa."""

    def __init__(self, core, others: Sequence, ties: Sequence[np.ndarray], kappa: float):
        self.insts: List[Instance] = [Instance(core)] + [Instance(p) for p in others]
        self.ties = [np.asarray(t, np.int64).reshape(-1, 2) for t in ties]
        self.kappa = float(kappa)
        self.R = [x.R for x in self.insts]
        self.off = np.concatenate([[0], np.cumsum(self.R)])
        self.dt = self.insts[0].dt
        assert all(abs(x.dt - self.dt) == 0 for x in self.insts)

    def tie_dofs(self, k: int):
        """DOF pairs (other domain k + 1, domain 0) of the ties of domain k + 1."""
        t = self.ties[k]
        d_o = (3 * t[:, :1] + np.arange(3)[None]).ravel()
        d_c = (3 * t[:, 1:] + np.arange(3)[None]).ravel()
        return d_o, d_c

    def tie_forces(self, us):
        """f_tie = dE_tie/du for every domain (N_d each)."""
        f = [np.zeros(x.N) for x in self.insts]
        X = [np.asarray(x.p.X, np.float64).ravel() for x in self.insts]
        for k in range(len(self.ties)):
            d_o, d_c = self.tie_dofs(k)
            gap = (X[k + 1][d_o] + us[k + 1][d_o]) - (X[0][d_c] + us[0][d_c])
            f[k + 1][d_o] += self.kappa * gap
            f[0][d_c] -= self.kappa * gap
        return f

    def system(self, rs, rbars, rdots, ws):
        """phi and dphi/dr of the stacked coordinates, and per-domain parts."""
        us = [x.displacement(r) for x, r in zip(self.insts, rs)]
        ft = self.tie_forces(us)
        parts = [x.system(r, rb, rd, w, f_extra=f) for x, r, rb, rd, w, f in zip(self.insts, rs, rbars, rdots, ws, ft)]
        n = int(self.off[-1])
        A = np.zeros((n, n))
        phi = np.zeros(n)
        for d, sd in enumerate(parts):
            s = slice(self.off[d], self.off[d + 1])
            A[s, s] = sd["A"]
            phi[s] = sd["phi"]
        c = slice(self.off[0], self.off[1])
        k2 = self.dt ** 2 * self.kappa
        for k in range(len(self.ties)):
            d_o, d_c = self.tie_dofs(k)
            o = slice(self.off[k + 1], self.off[k + 2])
            Jo = parts[k + 1]["Jt"][d_o]
            Jc = parts[0]["Jt"][d_c]
            A[o, o] += k2 * Jo.T @ Jo
            A[c, c] += k2 * Jc.T @ Jc
            A[o, c] -= k2 * Jo.T @ Jc
            A[c, o] -= k2 * Jc.T @ Jo
        return dict(phi=phi, A=A, parts=parts, u=us, f_tie=ft)

    def initial_state(self) -> List[State]:
        return [x.initial_state() for x in self.insts]

    def split(self, v):
        return [v[self.off[d]:self.off[d + 1]] for d in range(len(self.insts))]

    def step(self, sts: List[State], iters: int):
        """One coupled implicit-Euler step; returns the new states and ||phi||
        of the stacked system per iteration."""
        ws = [x.cubature_weights(s.rbar) for x, s in zip(self.insts, sts)]
        rbars = [s.rbar for s in sts]
        rdots = [s.rdot_bar for s in sts]
        r = np.concatenate(rbars)
        norms = []
        for _ in range(iters):
            sysd = self.system(self.split(r), rbars, rdots, ws)
            norms.append(float(np.linalg.norm(sysd["phi"])))
            lu = scipy.linalg.lu_factor(sysd["A"])
            r = r + scipy.linalg.lu_solve(lu, -sysd["phi"])
        rs = self.split(r)
        return [State(rbar=x, rdot_bar=(x - rb) / self.dt) for x, rb in zip(rs, rbars)], norms
