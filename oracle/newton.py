"""Reduced implicit-Euler Newton iteration in FP64 (test infrastructure only).

Sec. 3.6: u = U p + D(q) with U^T D = 0, r = [p; q], Jt = [U, J].  Implicit
Euler (Sec. 3.2) turns the reduced equation of motion into phi(r) = 0,
    phi = Jt^T M Jt (r - rbar - dt rdot_bar) + Jt^T f_fict
          + dt^2 Jt^T (f_int - f_ext),
    f_fict = M [(H . dq) dq],  dq = q - qbar           (eq. fict)
and its Newton matrix (eq. system_mat)
    dphi/dr = Ht^T a + Jt^T M [U, J + dJ] + dt^2 Jt^T K Jt
    a       = M Jt (r - rbar - dt rdot_bar) + f_fict + dt^2 (f_int - f_ext)
    dJ      = (S . dq) . dq + H . (3 dq - dt qdot_bar)  (eq. delta_j)
with Ht^T a = diag(0, a . H).  eq. system_mat prints the f_int - f_ext
contraction with a minus sign; differentiating phi gives a plus sign (the
same sign as the term dt^2 Jt^T K Jt that comes from the same summand), and
that is what is used.  The three Ht^T terms share one contraction with a by
linearity, evaluated by complex-step backpropagation (Sec. 4.4).  Lumped
mass M (Sec. 3.1), cubature for f_int and K (Sec. 5), weights from the
weight net at rbar once per step (Sec. 5.2).  The matrix is not symmetric
(the dJ block), so it is solved by LU with partial pivoting.  Newton starts
each step from r = rbar and takes a fixed number of full steps; after them
rdot = (r - rbar) / dt and rbar = r (Sec. 3.2).

Trimmed formulation (the comparison with latent space dynamics, Sec. 3.3
and Sec. 6): f_fict is dropped from phi, and the Newton matrix is the exact
derivative of that phi, i.e. dJ becomes H . (dq - dt qdot_bar) and a has no
M H(dq, dq) term.

Parity: phi pinned by textbook reductions (full-space implicit Euler when
the basis spans every free DOF; linear reduction for identity activations);
the Newton matrix pinned by central differences of phi and by quadratic
convergence; whole trajectories are parity unpinned beyond these.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import decoder as dec
from . import fd
from . import fem
from .wnet import wnet_weights


@dataclass
class State:
    rbar: np.ndarray
    rdot_bar: np.ndarray


class Instance:
    """Precomputed rest-shape data of one problem (a synth.Problem)."""

    def __init__(self, prob, h_cs: float = dec.H_CS, fd_h: float = None, fd_dtype=np.float64):
        """fd_h: derivatives by recursive central differences of step fd_h
        (oracle/fd.py, evaluated in fd_dtype) instead of complex steps."""
        self.p = prob
        self.h = h_cs
        self.fd_h = fd_h if fd_h is not None else (prob.fd_h if getattr(prob, "fd_h", 0.0) > 0 else None)
        self.fd_dtype = fd_dtype
        self.N = prob.N
        self.n_p = prob.n_p
        self.n_q = prob.n_q if prob.weights else 0
        self.R = self.n_p + self.n_q
        self.Bm, self.Ve = fem.rest_shape(prob.X, prob.tets)
        self.mass = fem.lumped_mass(prob.tets, self.Ve, prob.rho, prob.n)
        self.mu, self.lam = fem.lame(prob.E, prob.nu)
        self.pin_dof = np.repeat(prob.pinned, 3)
        self.f_ext = self.mass * np.tile(prob.gravity, prob.n)
        self.dt = prob.dt

    # -- weights -----------------------------------------------------------
    def cubature_weights(self, rbar):
        p = self.p
        if p.cub_w is not None:
            return np.asarray(p.cub_w, np.float64)
        return wnet_weights(p.wnet_weights, p.wnet_biases, p.wnet_scale, rbar)

    # -- decoder (Sec. 4) --------------------------------------------------
    def decode(self, q, dq, qdot_bar):
        """u_q = D(q), J, dJ, Hdd = H(dq, dq): all after filter and pin mask."""
        p = self.p
        if self.n_q == 0:
            z = np.zeros(self.N)
            return dict(m=z, J=np.zeros((self.N, 0)), dJ=np.zeros((self.N, 0)), Hdd=z.copy())
        if self.fd_h is None:
            rc = dec.right_contractions(p.weights, p.biases, p.act, q, dq, qdot_bar, n_rows=self.N, h=self.h)
        else:
            rc = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qdot_bar, n_rows=self.N, h=self.fd_h,
                                          dtype=self.fd_dtype)
        trimmed = p.formulation == "trimmed"
        dJ = dec.delta_J(rc, self.dt, trimmed)
        f = lambda x: dec.filter_pin(x, p.U, self.pin_dof)
        Hdd = np.zeros(self.N) if trimmed else f(rc["Hdd"])
        return dict(m=f(rc["m"]), J=f(rc["J"]), dJ=f(dJ), Hdd=Hdd)

    def left(self, q, a):
        """(J^T a, a . H) of D = P (I - U U^T) m through complex-step BP."""
        p = self.p
        s = dec.filter_pin_T(a, p.U, self.pin_dof)
        if self.fd_h is not None:
            return fd.left_contraction_fd(p.weights, p.biases, p.act, q, s, h=self.fd_h, dtype=self.fd_dtype)
        return dec.left_contraction(p.weights, p.biases, p.act, q, s, h=self.h)

    # -- one Newton linearisation ------------------------------------------
    def system(self, r, rbar, rdot_bar, w, f_extra=None):
        """phi(r), dphi/dr and intermediates at iterate r of the step from rbar.

        f_extra (N, optional): a further internal force at the DOFs (the
        interface force of a coupled domain, oracle/coupled.py); it enters
        a and phi exactly as f_int does.  Its stiffness is the caller's."""
        n_p, n_q, dt = self.n_p, self.n_q, self.dt
        p_, q = r[:n_p], r[n_p:]
        dq = q - rbar[n_p:]
        qdot_bar = rdot_bar[n_p:]
        d = self.decode(q, dq, qdot_bar)
        U = self.p.U
        u = (U @ p_ if n_p else 0.0) + d["m"]
        Jt = np.concatenate([U, d["J"]], axis=1)
        f_int, fr, Kr = fem.cubature_force_stiffness(
            self.p.X, self.p.tets, u, Jt, self.p.cub_ids, w, self.Bm, self.Ve, self.mu, self.lam)
        M = self.mass
        w_r = r - rbar - dt * rdot_bar
        f_fict = M * d["Hdd"]
        f_all = f_int if f_extra is None else f_int + f_extra
        a = M * (Jt @ w_r) + f_fict + dt * dt * (f_all - self.f_ext)
        phi = Jt.T @ (M * (Jt @ w_r)) + Jt.T @ f_fict + dt * dt * (Jt.T @ (f_all - self.f_ext))
        A = Jt.T @ (M[:, None] * np.concatenate([U, d["J"] + d["dJ"]], axis=1)) + dt * dt * Kr
        if n_q:
            JTa, B = self.left(q, a)
            A[n_p:, n_p:] += B
        else:
            JTa, B = np.zeros(0), np.zeros((0, 0))
        return dict(phi=phi, A=A, u=u, J=d["J"], Jt=Jt, dJ=d["dJ"], Hdd=d["Hdd"], f_int=f_int,
                    fr=fr, Kr=Kr, a=a, B=B, JTa=JTa, w=w)

    # -- time stepping -----------------------------------------------------
    def step(self, st: State, iters: int):
        """One implicit-Euler step; returns the new state and ||phi|| per iteration."""
        w = self.cubature_weights(st.rbar)
        r = st.rbar.copy()
        norms = []
        for _ in range(iters):
            sysd = self.system(r, st.rbar, st.rdot_bar, w)
            norms.append(float(np.linalg.norm(sysd["phi"])))
            lu = scipy.linalg.lu_factor(sysd["A"])
            r = r + scipy.linalg.lu_solve(lu, -sysd["phi"])
        rdot = (r - st.rbar) / self.dt
        return State(rbar=r, rdot_bar=rdot), norms

    def initial_state(self) -> State:
        return State(rbar=np.asarray(self.p.r0, np.float64).copy(),
                     rdot_bar=np.asarray(self.p.rdot0, np.float64).copy())

    def displacement(self, r):
        n_p = self.n_p
        if self.n_q == 0:
            return self.p.U @ r
        q = r[n_p:]
        m = dec.mlp_real(self.p.weights, self.p.biases, self.p.act, q)[: self.N]
        u = dec.filter_pin(m, self.p.U, self.pin_dof)
        return u + (self.p.U @ r[:n_p] if n_p else 0.0)

    def simulate(self, steps: int, iters: int, st: State = None):
        st = st or self.initial_state()
        traj, norms = [st], []
        for _ in range(steps):
            st, nrm = self.step(st, iters)
            traj.append(st)
            norms.append(nrm)
        return traj, norms
