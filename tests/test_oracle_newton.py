"""Pins of the oracle's reduced Newton iteration (Sec. 3.2, 3.6; eq. system_mat,
eq. delta_j) against finite differences and textbook reductions."""
import numpy as np
import pytest
import scipy.linalg

from oracle import decoder as dec
from oracle import fem
from oracle.newton import Instance, State
from oracle.wnet import wnet_weights
from paper_2102_11026_amd import synth

rng = np.random.default_rng(5)


def moving_state(inst, scale=0.005):
    R = inst.R
    rbar = inst.p.r0.copy()
    rdot = rng.normal(size=R) * scale * 30
    r = rbar + rng.normal(size=R) * scale
    return r, rbar, rdot


@pytest.mark.parametrize("act,n_p", [("tanh", 0), ("elu", 2), ("sin", 3)])
def test_newton_matrix_is_the_derivative_of_phi(act, n_p):
    """eq. system_mat (with the sign of the f_int - f_ext contraction that
    differentiation gives) against central differences of phi."""
    p = synth.tiny_problem(widths=(2, 6, 6, 36), act=act, n_p=n_p, name=f"fd{act}{n_p}", q_std=0.3, out_scale=0.05)
    inst = Instance(p)
    r, rbar, rdot = moving_state(inst)
    w = np.ones(p.tets.shape[0]) * 1.3
    A = inst.system(r, rbar, rdot, w)["A"]
    eps = 1e-6
    fd = np.stack([(inst.system(r + eps * e, rbar, rdot, w)["phi"] - inst.system(r - eps * e, rbar, rdot, w)["phi"])
                   / (2 * eps) for e in np.eye(inst.R)], axis=1)
    np.testing.assert_allclose(A, fd, rtol=1e-6, atol=1e-6 * np.abs(A).max())
    # the printed minus sign would not match
    sysd = inst.system(r, rbar, rdot, w)
    q = r[n_p:]
    _, Bext = inst.left(q, 2 * inst.dt ** 2 * (sysd["f_int"] - inst.f_ext))
    A_printed = A.copy()
    A_printed[n_p:, n_p:] -= Bext
    assert np.abs(A_printed - fd).max() > 1e3 * np.abs(A - fd).max()


def test_quadratic_convergence():
    """Newton with the exact matrix: ||phi_k+1|| ~ C ||phi_k||^2 near the root
    (192-vertex bar, tanh decoder, second step)."""
    inst = Instance(synth.config_plain_fp64())
    st, _ = inst.step(inst.initial_state(), 3)
    _, norms = inst.step(st, 6)
    norms = np.array(norms)
    k = [i for i in range(1, len(norms)) if norms[i - 1] < 1e-2 * norms[0] and norms[i] > 1e-13 * norms[0]]
    assert len(k) >= 1
    for i in k:
        assert norms[i] < 10 * norms[i - 1] ** 2 / norms[0]
    assert norms[-1] < 1e-12 * norms[0]


def assemble_full(p, u, Bm, Ve, mu, lam):
    f, K = fem.element_force_stiffness(p.X, p.tets, u, Bm, Ve, mu, lam)
    dofs = fem.tet_dofs(p.tets)
    fg = np.zeros(p.N)
    Kg = np.zeros((p.N, p.N))
    for e in range(p.tets.shape[0]):
        fg[dofs[e]] += f[e]
        Kg[np.ix_(dofs[e], dofs[e])] += K[e]
    return fg, Kg


def test_full_basis_reduces_to_full_space_implicit_euler():
    """n_q = 0 and U = identity on the free DOFs: textbook full-space Newton,
    (M + dt^2 K) delta = -[M (u - ubar - dt udot_bar) + dt^2 (f_int - f_ext)]."""
    base = synth.tiny_problem(name="fullspace")
    free = np.flatnonzero(np.repeat(base.pinned, 3) == 0)
    U = np.zeros((base.N, free.size))
    U[free, np.arange(free.size)] = 1.0
    p = base.replace(U=U, weights=[], biases=[], r0=rng.normal(size=free.size) * 0.003,
                     rdot0=rng.normal(size=free.size) * 0.05)
    inst = Instance(p)
    st = inst.initial_state()
    st1, _ = inst.step(st, 3)
    # textbook
    Bm, Ve = fem.rest_shape(p.X, p.tets)
    mu, lam = fem.lame(p.E, p.nu)
    m = fem.lumped_mass(p.tets, Ve, p.rho, p.n)
    fext = m * np.tile(p.gravity, p.n)
    ubar, udot = U @ p.r0, U @ p.rdot0
    u = ubar.copy()
    for _ in range(3):
        f, K = assemble_full(p, u, Bm, Ve, mu, lam)
        g = m * (u - ubar - p.dt * udot) + p.dt ** 2 * (f - fext)
        Mat = np.diag(m) + p.dt ** 2 * K
        d = np.zeros(p.N)
        d[free] = np.linalg.solve(Mat[np.ix_(free, free)], -g[free])
        u = u + d
    np.testing.assert_allclose(U @ st1.rbar, u, rtol=1e-10, atol=1e-14)


def test_identity_activation_is_linear_reduction():
    """eq. linear_reduction with implicit Euler: D linear gives H = 0, J = P W."""
    p = synth.tiny_problem(widths=(3, 5, 5, 36), act="identity", name="linred", q_std=0.2, out_scale=0.05)
    inst = Instance(p)
    Ueff = np.linalg.multi_dot(p.weights[::-1]) * (np.repeat(p.pinned, 3) == 0)[:, None]
    r, rbar, rdot = moving_state(inst)
    w = np.ones(p.tets.shape[0])
    sysd = inst.system(r, rbar, rdot, w)
    Bm, Ve = fem.rest_shape(p.X, p.tets)
    mu, lam = fem.lame(p.E, p.nu)
    m = fem.lumped_mass(p.tets, Ve, p.rho, p.n)
    u = Ueff @ r  # zero biases
    f, K = assemble_full(p, u, Bm, Ve, mu, lam)
    fext = m * np.tile(p.gravity, p.n)
    Mp = Ueff.T @ (m[:, None] * Ueff)
    phi = Mp @ (r - rbar - p.dt * rdot) + p.dt ** 2 * Ueff.T @ (f - fext)
    A = Mp + p.dt ** 2 * Ueff.T @ K @ Ueff
    np.testing.assert_allclose(sysd["phi"], phi, rtol=1e-10, atol=1e-12 * np.abs(phi).max())
    np.testing.assert_allclose(sysd["A"], A, rtol=1e-10, atol=1e-12 * np.abs(A).max())


def test_collective_newton_matches_full_tensor_newton():
    """Tiny nonlinear net [2,4,4,36]: phi and dphi/dr written with the full
    tensors J, H, S (eq. our_equation_of_motion, eq. fict, eq. system_mat,
    eq. delta_j), three Newton iterates compared."""
    p = synth.tiny_problem(widths=(2, 4, 4, 36), act="tanh", name="fulltensor", q_std=0.3, out_scale=0.05)
    inst = Instance(p)
    Bm, Ve = fem.rest_shape(p.X, p.tets)
    mu, lam = fem.lame(p.E, p.nu)
    m = fem.lumped_mass(p.tets, Ve, p.rho, p.n)
    fext = m * np.tile(p.gravity, p.n)
    keep = (np.repeat(p.pinned, 3) == 0).astype(float)
    dt = p.dt
    rbar = p.r0.copy()
    rdot = rng.normal(size=2) * 0.4
    r = rbar.copy()
    r_or = rbar.copy()
    w = np.ones(p.tets.shape[0])
    for _ in range(3):
        Wb = (p.weights, p.biases, p.act)
        u = dec.mlp_real(*Wb, r) * keep
        J = dec.full_jacobian(*Wb, r) * keep[:, None]
        H = dec.full_hessian(*Wb, r) * keep[:, None, None]
        S = dec.full_third(*Wb, r) * keep[:, None, None, None]
        f, K = assemble_full(p, u, Bm, Ve, mu, lam)
        dq = r - rbar
        wr = r - rbar - dt * rdot
        ffict = m * (H @ dq @ dq)
        phi = J.T @ (m * (J @ wr)) + J.T @ ffict + dt ** 2 * J.T @ (f - fext)
        a = m * (J @ wr) + ffict + dt ** 2 * (f - fext)
        dJ = S @ dq @ dq + H @ (3 * dq - dt * rdot)
        A = np.einsum("i,ikl->kl", a, H) + J.T @ (m[:, None] * (J + dJ)) + dt ** 2 * J.T @ K @ J
        r = r - np.linalg.solve(A, phi)
        sysd = inst.system(r_or, rbar, rdot, w)
        r_or = r_or - scipy.linalg.solve(sysd["A"], sysd["phi"])
        np.testing.assert_allclose(r_or, r, rtol=1e-10, atol=1e-13)


def test_wnet_closed_form():
    """Zero weights and biases: every layer outputs ln 2, so w = scale ln 2."""
    Ws = [np.zeros((5, 3)), np.zeros((4, 5)), np.zeros((7, 4))]
    bs = [np.zeros(5), np.zeros(4), np.zeros(7)]
    np.testing.assert_allclose(wnet_weights(Ws, bs, 2.5, rng.normal(size=3)), 2.5 * np.log(2.0), rtol=1e-15)
    # one layer, generic: scale * log(1 + exp(W r + b))
    W, b, r = rng.normal(size=(6, 3)), rng.normal(size=6), rng.normal(size=3)
    np.testing.assert_allclose(wnet_weights([W], [b], 1.7, r), 1.7 * np.log1p(np.exp(W @ r + b)), rtol=1e-14)


def test_wnet_softplus_after_the_hidden_layer():
    """Sec. 5.2 weight net with a softplus after every layer: a zero first
    layer outputs softplus(0) = ln 2 whatever r is, and a second layer of
    weight 1 maps it to softplus(ln 2) = ln(1 + 2) = ln 3.  A net that skipped
    the hidden softplus would give softplus(0) = ln 2 instead."""
    Ws = [np.zeros((1, 4)), np.ones((1, 1))]
    bs = [np.zeros(1), np.zeros(1)]
    for _ in range(3):
        np.testing.assert_allclose(wnet_weights(Ws, bs, 0.8, rng.normal(size=4)), [0.8 * np.log(3.0)], rtol=1e-15)
    # two hidden units, output weights (1, -1) and bias 2: softplus(ln2 - ln2 + 2)
    Ws = [np.zeros((2, 3)), np.array([[1.0, -1.0]])]
    bs = [np.zeros(2), np.array([2.0])]
    np.testing.assert_allclose(wnet_weights(Ws, bs, 1.0, rng.normal(size=3)), [np.log1p(np.exp(2.0))], rtol=1e-15)


# --------------------------------------------------------------------------
# trimmed formulation: the fictitious force dropped (Sec. 3.3, Sec. 6)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("act,n_p", [("tanh", 0), ("sin", 2)])
def test_trimmed_newton_matrix_is_the_derivative_of_trimmed_phi(act, n_p):
    """With f_fict dropped, dJ = H . (dq - dt qdot_bar) and a without M Hdd
    still give the exact Newton matrix of the trimmed phi (central differences)."""
    p = synth.tiny_problem(widths=(2, 6, 6, 36), act=act, n_p=n_p, name=f"tr{act}{n_p}", q_std=0.3, out_scale=0.05)
    inst = Instance(p.replace(formulation="trimmed"))
    r, rbar, rdot = moving_state(inst)
    w = np.ones(p.tets.shape[0]) * 1.3
    A = inst.system(r, rbar, rdot, w)["A"]
    eps = 1e-6
    fd = np.stack([(inst.system(r + eps * e, rbar, rdot, w)["phi"] - inst.system(r - eps * e, rbar, rdot, w)["phi"])
                   / (2 * eps) for e in np.eye(inst.R)], axis=1)
    np.testing.assert_allclose(A, fd, rtol=1e-6, atol=1e-6 * np.abs(A).max())
    # the full-formulation matrix is not the derivative of the trimmed phi
    A_full = Instance(p).system(r, rbar, rdot, w)["A"]
    assert np.abs(A_full - fd).max() > 1e3 * np.abs(A - fd).max()


def test_trimmed_equals_full_for_a_linear_decoder():
    """Identity activations: H = S = 0, so dropping f_fict changes nothing."""
    p = synth.tiny_problem(widths=(2, 6, 6, 36), act="identity", n_p=1, name="trlin", q_std=0.3, out_scale=0.05)
    a, b = Instance(p), Instance(p.replace(formulation="trimmed"))
    r, rbar, rdot = moving_state(a)
    w = np.ones(p.tets.shape[0])
    sa, sb = a.system(r, rbar, rdot, w), b.system(r, rbar, rdot, w)
    np.testing.assert_array_equal(sa["phi"], sb["phi"])
    np.testing.assert_array_equal(sa["A"], sb["A"])


def test_full_minus_trimmed_phi_is_the_fictitious_force():
    """phi_full - phi_trimmed = Jt^T M H(dq, dq), H from the exhaustive
    one-pass-per-pair Hessian (eq. mcfd_hessian), not from the collective seed."""
    p = synth.tiny_problem(widths=(3, 8, 8, 36), act="sin", n_p=2, name="trff", q_std=0.3, out_scale=0.05)
    full, trim = Instance(p), Instance(p.replace(formulation="trimmed"))
    r, rbar, rdot = moving_state(full, scale=0.02)
    w = np.ones(p.tets.shape[0])
    sf, st = full.system(r, rbar, rdot, w), trim.system(r, rbar, rdot, w)
    q, dq = r[p.n_p:], (r - rbar)[p.n_p:]
    H = dec.full_hessian(p.weights, p.biases, p.act, q)[: p.N]
    Hdd = dec.filter_pin(np.einsum("ikl,k,l->i", H, dq, dq), p.U, full.pin_dof)
    Jt = np.concatenate([p.U, sf["J"]], axis=1)
    np.testing.assert_allclose(sf["phi"] - st["phi"], Jt.T @ (full.mass * Hdd), rtol=1e-9,
                               atol=1e-12 * np.abs(sf["phi"]).max())
