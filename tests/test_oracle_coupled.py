"""Pins of the oracle's coupled multi-domain step (Sec. 6.8 with the tie-spring
reading of the domain coupling; Sec. 3.2, eq. system_mat per domain)."""
import numpy as np
import pytest

from oracle import fem
from oracle.coupled import Coupled
from oracle.newton import Instance
from paper_2102_11026_amd import synth

rng = np.random.default_rng(17)


def full_basis(p, r_scale=0.003, v_scale=0.05):
    """The same domain with U = identity on its free DOFs and no decoder."""
    free = np.flatnonzero(np.repeat(p.pinned, 3) == 0)
    U = np.zeros((p.N, free.size))
    U[free, np.arange(free.size)] = 1.0
    return p.replace(U=U, weights=[], biases=[], r0=rng.normal(size=free.size) * r_scale,
                     rdot0=rng.normal(size=free.size) * v_scale), free


def test_scene_geometry():
    """Tied vertex copies coincide at rest, every tet is positively oriented
    and no core vertex is tied to two rods."""
    s = synth.config_coupled_tiny(2)
    used = set()
    for rod, t in zip(s.rods, s.ties):
        np.testing.assert_array_equal(rod.X[t[:, 0]], s.core.X[t[:, 1]])
        assert not used & set(t[:, 1].tolist())
        used |= set(t[:, 1].tolist())
        assert not s.core.pinned[t[:, 1]].any()
    for p in [s.core] + s.rods:
        e = p.X[p.tets[:, 1:]] - p.X[p.tets[:, :1]]
        assert (np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2])) > 0).all()
    # the frame basis is orthonormal and holds the rod's translations
    U = s.rods[0].U
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    t = np.tile([1.0, 0.0, 0.0], s.rods[0].n)
    np.testing.assert_allclose(U @ (U.T @ t), t, atol=1e-12)


def assemble(p, u, Bm, Ve, mu, lam):
    f, K = fem.element_force_stiffness(p.X, p.tets, u, Bm, Ve, mu, lam)
    dofs = fem.tet_dofs(p.tets)
    fg = np.zeros(p.N)
    Kg = np.zeros((p.N, p.N))
    for e in range(p.tets.shape[0]):
        fg[dofs[e]] += f[e]
        Kg[np.ix_(dofs[e], dofs[e])] += K[e]
    return fg, Kg


def test_full_basis_coupled_step_is_full_space_implicit_euler_of_the_union():
    """Every domain with U = identity on its free DOFs and no decoder: the
    coupled reduced Newton iterates are those of textbook full-space implicit
    Euler on the union mesh, the tied copies joined by springs,
    (M + dt^2 (K + K_tie)) delta = -[M (u - ubar - dt udot) + dt^2 (f + f_tie - f_ext)]."""
    s = synth.config_coupled_tiny(2)
    doms, frees = zip(*[full_basis(p) for p in [s.core] + s.rods])
    kappa = 3.0e4
    c = Coupled(doms[0], doms[1:], s.ties, kappa)
    sts, _ = c.step(c.initial_state(), 3)
    # the union mesh, assembled here from the element routines alone
    offs = np.concatenate([[0], np.cumsum([p.N for p in doms])])
    Ntot = int(offs[-1])
    free = np.concatenate([f + o for f, o in zip(frees, offs[:-1])])
    mass = np.zeros(Ntot)
    fext = np.zeros(Ntot)
    pre = []
    for p, o in zip(doms, offs[:-1]):
        Bm, Ve = fem.rest_shape(p.X, p.tets)
        mu, lam = fem.lame(p.E, p.nu)
        m = fem.lumped_mass(p.tets, Ve, p.rho, p.n)
        mass[o:o + p.N] = m
        fext[o:o + p.N] = m * np.tile(p.gravity, p.n)
        pre.append((Bm, Ve, mu, lam))
    Xall = np.concatenate([p.X.ravel() for p in doms])
    pairs = []
    for k, t in enumerate(s.ties):
        for a, b in t:
            for d in range(3):
                pairs.append((offs[k + 1] + 3 * a + d, offs[0] + 3 * b + d))
    ubar = np.concatenate([p.U @ p.r0 for p in doms])
    udot = np.concatenate([p.U @ p.rdot0 for p in doms])
    dt = doms[0].dt
    u = ubar.copy()
    for _ in range(3):
        f = np.zeros(Ntot)
        K = np.zeros((Ntot, Ntot))
        for p, o, (Bm, Ve, mu, lam) in zip(doms, offs[:-1], pre):
            fd, Kd = assemble(p, u[o:o + p.N], Bm, Ve, mu, lam)
            f[o:o + p.N] += fd
            K[o:o + p.N, o:o + p.N] += Kd
        for ia, ib in pairs:
            g = (Xall[ia] + u[ia]) - (Xall[ib] + u[ib])
            f[ia] += kappa * g
            f[ib] -= kappa * g
            K[ia, ia] += kappa
            K[ib, ib] += kappa
            K[ia, ib] -= kappa
            K[ib, ia] -= kappa
        g = mass * (u - ubar - dt * udot) + dt ** 2 * (f - fext)
        Mat = np.diag(mass) + dt ** 2 * K
        d = np.zeros(Ntot)
        d[free] = np.linalg.solve(Mat[np.ix_(free, free)], -g[free])
        u = u + d
    got = np.concatenate([p.U @ st.rbar for p, st in zip(doms, sts)])
    np.testing.assert_allclose(got, u, rtol=1e-10, atol=1e-13)
    # the ties pull: the coupled step differs from the uncoupled one
    c0 = Coupled(doms[0], doms[1:], s.ties, 0.0)
    sts0, _ = c0.step(c0.initial_state(), 3)
    got0 = np.concatenate([p.U @ st.rbar for p, st in zip(doms, sts0)])
    assert np.abs(got0 - got).max() > 1e-4 * np.abs(got).max()


def test_coupled_newton_matrix_is_the_derivative_of_phi():
    """Stacked coupled phi (nonlinear decoders in every domain) against
    central differences: the tie stiffness blocks, the cross blocks and the
    tie force inside the a . H contraction."""
    s = synth.config_coupled_tiny(2)
    c = Coupled(s.core, s.rods, s.ties, s.kappa)
    sts = c.initial_state()
    rbars = [x.rbar for x in sts]
    rdots = [rng.normal(size=x.rbar.size) * 0.3 for x in sts]
    ws = [x.cubature_weights(b) for x, b in zip(c.insts, rbars)]
    r = np.concatenate(rbars) + rng.normal(size=int(c.off[-1])) * 0.004
    sysd = c.system(c.split(r), rbars, rdots, ws)
    A = sysd["A"]
    eps = 1e-6
    cols = []
    for k in range(r.size):
        e = np.zeros(r.size)
        e[k] = eps
        cols.append((c.system(c.split(r + e), rbars, rdots, ws)["phi"]
                     - c.system(c.split(r - e), rbars, rdots, ws)["phi"]) / (2 * eps))
    fd = np.stack(cols, axis=1)
    np.testing.assert_allclose(A, fd, rtol=1e-6, atol=1e-6 * np.abs(A).max())
    # the cross blocks are there and matter
    cs = slice(c.off[0], c.off[1])
    o1 = slice(c.off[1], c.off[2])
    assert np.abs(A[cs, o1]).max() > 1e-3 * np.abs(A).max()


def test_zero_kappa_is_independent_domains():
    """kappa = 0: each domain steps on its own (from rest: a free rod whose
    random decoder starts it deformed can invert without its tie)."""
    s = synth.config_coupled_tiny(2)
    doms = [p.replace(r0=np.zeros(p.R)) for p in [s.core] + s.rods]
    c = Coupled(doms[0], doms[1:], s.ties, 0.0)
    sts, _ = c.step(c.initial_state(), 3)
    for p, st in zip(doms, sts):
        oi = Instance(p)
        ref, _ = oi.step(oi.initial_state(), 3)
        np.testing.assert_allclose(st.rbar, ref.rbar, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(st.rdot_bar, ref.rdot_bar, rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("kappa", [1.0e4, 1.0e6])
def test_tie_force_is_the_gradient_of_the_tie_energy(kappa):
    s = synth.config_coupled_tiny(1)
    c = Coupled(s.core, s.rods, s.ties, kappa)
    us = [rng.normal(size=x.N) * 0.01 for x in c.insts]
    X = [x.p.X.ravel() for x in c.insts]

    def energy(us):
        e = 0.0
        for k, t in enumerate(c.ties):
            for a, b in t:
                g = (X[k + 1][3 * a:3 * a + 3] + us[k + 1][3 * a:3 * a + 3]) - (X[0][3 * b:3 * b + 3] + us[0][3 * b:3 * b + 3])
                e += 0.5 * kappa * g @ g
        return e

    f = c.tie_forces(us)
    for d in range(2):
        for i in list(c.ties[0][:, 1 - d] * 3) + [0]:
            for h in (1e-6,):
                up = [u.copy() for u in us]
                um = [u.copy() for u in us]
                up[d][i] += h
                um[d][i] -= h
                assert abs((energy(up) - energy(um)) / (2 * h) - f[d][i]) < 1e-6 * max(1.0, abs(f[d][i]))
