"""Pins of the oracle's neural cubature training (Sec. 5): training data,
both losses' gradients, Adam, selection and the alternation's bookkeeping."""
import numpy as np
import pytest

from oracle import cubature_train as ct
from oracle import fem
from oracle.newton import Instance
from paper_2102_11026_amd import synth

rng = np.random.default_rng(5)


@pytest.fixture(scope="module")
def tiny():
    t = synth.config_cubature_tiny()
    inst = Instance(t.prob)
    data = [ct.element_forces(inst, r) for r in t.poses]
    return t, inst, data


def test_element_forces_are_the_energy_gradient_along_the_subspace(tiny):
    """sum_e Jt_e^T f_e = d E(u(r)) / dr (central differences of the neo-Hookean
    energy of the decoded displacement)."""
    t, inst, data = tiny
    p = t.prob
    r = t.poses[3]
    F, f, u = data[3]

    def energy(r):
        u, _ = ct.pose_jacobian(inst, r)
        return fem.total_energy(p.X, p.tets, u, inst.Ve, inst.Bm, inst.mu, inst.lam)

    h = 1e-6
    fd = np.array([(energy(r + h * e) - energy(r - h * e)) / (2 * h) for e in np.eye(r.size)])
    np.testing.assert_allclose(f, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
    np.testing.assert_allclose(F.sum(axis=0), f, rtol=1e-13, atol=1e-13 * np.abs(f).max())
    # and the full-quadrature reduced force of the simulator
    _, Jt = ct.pose_jacobian(inst, r)
    m = p.tets.shape[0]
    _, fr, _ = fem.cubature_force_stiffness(p.X, p.tets, u, Jt, np.arange(m), np.ones(m), inst.Bm, inst.Ve,
                                            inst.mu, inst.lam)
    np.testing.assert_allclose(fr, f, rtol=1e-12, atol=1e-12 * np.abs(f).max())


def wnet_params(t):
    return [W.copy() for W in t.wnet_weights], [b.copy() for b in t.wnet_biases]


def test_loss_W_gradient_against_central_differences(tiny):
    t, inst, data = tiny
    Ws, bs = wnet_params(t)
    for W in Ws:
        W += rng.normal(size=W.shape) * 0.3
    for b in bs:
        b += rng.normal(size=b.shape) * 0.3
    C = [5, 17, 2, 40, 33, 8]
    dw = [(r, F, f) for r, (F, f, _) in zip(t.poses, data)]
    L, gW, gb = ct.loss_W(Ws, bs, t.scale, C, dw)
    assert L > 0
    h = 1e-6
    for arrs, grads in ((Ws, gW), (bs, gb)):
        for l, (A, G) in enumerate(zip(arrs, grads)):
            for idx in [tuple(rng.integers(0, s) for s in A.shape) for _ in range(6)] + [tuple(s - 1 for s in A.shape)]:
                old = A[idx]
                A[idx] = old + h
                lp = ct.loss_W(Ws, bs, t.scale, C, dw)[0]
                A[idx] = old - h
                lm = ct.loss_W(Ws, bs, t.scale, C, dw)[0]
                A[idx] = old
                assert abs((lp - lm) / (2 * h) - G[idx]) < 1e-6 * max(abs(G[idx]), 1e-3 * L), (l, idx)
    # rows of the last layer beyond |C| get no gradient
    assert not gW[-1][len(C):].any() and not gb[-1][len(C):].any()
    assert gW[-1][:len(C)].any()


def test_loss_W_vanishes_at_full_quadrature(tiny):
    """C = every element with weights identically one (a constant last layer:
    zero weights, bias softplus^-1(1 / scale)) reproduces f exactly."""
    t, inst, data = tiny
    m = t.prob.tets.shape[0]
    Ws, bs = wnet_params(t)
    scale = 3.0
    Ws[-1] = np.zeros((m, Ws[-1].shape[1]))
    bs[-1] = np.full(m, np.log(np.expm1(1.0 / scale)))
    w, _ = ct.wnet_forward(Ws, bs, scale, m, t.poses[0])
    np.testing.assert_allclose(w, 1.0, rtol=1e-14)
    dw = [(r, F, f) for r, (F, f, _) in zip(t.poses, data)]
    L, _, _ = ct.loss_W(Ws, bs, scale, list(range(m)), dw)
    assert L < 1e-26


def test_mesh_graph_two_tets():
    """Two tets sharing the face {1, 2, 3}: the face vertices see all five
    vertices (d = 5), the apexes 0 and 4 see four (d = 4) and not each other."""
    tets = np.array([[0, 1, 2, 3], [4, 1, 3, 2]])
    A = ct.mesh_graph(tets, 5)
    d = np.array([4, 5, 5, 5, 4], float)
    for i in range(5):
        for j in range(5):
            want = 0.0 if {i, j} == {0, 4} else 1.0 / np.sqrt(d[i] * d[j])
            assert A[i, j] == pytest.approx(want, rel=1e-15)
    # sqrt(d) is an eigenvector with eigenvalue one
    np.testing.assert_allclose(A @ np.sqrt(d), np.sqrt(d), rtol=1e-15)


def test_selection_net_with_no_input_gives_uniform_scores(tiny):
    """G0 = 0: every vertex feature vanishes, every logit equals
    A2 . sin(a1) + a2, and the scores are e^c / |candidates|."""
    t, inst, data = tiny
    th = ct.s_unpack(t.theta.copy())
    th["G0"] = np.zeros((3, 8))
    th["a1"] = rng.normal(size=8)
    th["a2"] = 0.3
    th["c"] = 1.7
    theta = ct.s_pack(th)
    p = t.prob
    A = ct.mesh_graph(p.tets, p.n)
    cand = np.arange(7, 50)
    z, s, _ = ct.snet_forward(theta, A, p.tets, data[0][2], cand)
    np.testing.assert_allclose(z, th["A2"] @ np.sin(th["a1"]) + 0.3, rtol=1e-14)
    np.testing.assert_allclose(s, np.exp(1.7) / cand.size, rtol=1e-14)


def test_loss_S_gradient_against_central_differences(tiny):
    t, inst, data = tiny
    p = t.prob
    A = ct.mesh_graph(p.tets, p.n)
    # displacements large enough that every sine is in its nonlinear range
    theta = t.theta + rng.normal(size=ct.S_SIZE) * 0.5
    theta[-1] = 0.4
    cand = np.array([e for e in range(p.tets.shape[0]) if e % 7])
    ds = [(u * 40.0, F, f * 0.5) for (F, f, u) in data[:4]]
    L, g = ct.loss_S(theta, A, p.tets, cand, ds)
    assert L > 0
    h = 1e-6
    for k in range(ct.S_SIZE):
        e = np.zeros(ct.S_SIZE)
        e[k] = h
        fd = (ct.loss_S(theta + e, A, p.tets, cand, ds)[0] - ct.loss_S(theta - e, A, p.tets, cand, ds)[0]) / (2 * h)
        # central-difference rounding ~ 1e-16 L / h ~ 1e-10
        assert abs(fd - g[k]) < 1e-6 * abs(g[k]) + 2e-9, (k, fd, g[k])
    assert np.abs(g[:24]).min() > 1e-7          # the first convolution is reached


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2, so p moves by
    -lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-9, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    ad = ct.Adam(lr=1e-3)
    q = p.copy()
    ad.step([q], [g])
    np.testing.assert_allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    # a second step with the same gradient moves by the same amount
    r = q.copy()
    ad.step([r], [g])
    np.testing.assert_allclose(r - q, q - p, rtol=1e-12, atol=1e-20)


def test_select_top_breaks_ties_to_the_lower_id():
    cand = np.array([2, 5, 6, 9, 11])
    s = np.array([0.1, 0.3, 0.3, 0.05, 0.3])
    assert ct.select_top(s, cand, 2) == [5, 6]
    assert ct.select_top(s, cand, 4) == [5, 6, 11, 2]


def test_voronoi_samples_on_a_line():
    """Tets whose centroids lie at x = 0, 1, ..., 9: farthest-point sampling
    from 0 takes 9, then the middle (4, the lower of 4 and 5), then 2 (first
    of the two gaps of width 4: 2 and 6/7)."""
    X = np.zeros((40, 3))
    tets = np.zeros((10, 4), int)
    for e in range(10):
        X[4 * e:4 * e + 4] = [[4.0 * e, 0, 0], [0, 1, 0], [0, 0, 1], [0, -1, -1]]
        tets[e] = np.arange(4 * e, 4 * e + 4)
    assert ct.voronoi_samples(X, tets, 4) == [0, 9, 4, 2]


def test_alternation_bookkeeping_and_descent(tiny):
    t, inst, data = tiny
    m = t.prob.tets.shape[0]
    C0 = ct.voronoi_samples(t.prob.X, t.prob.tets, t.n_c0)
    res = ct.train(inst, t.poses, t.wnet_weights, t.wnet_biases, t.scale, t.theta, C0, t.K, t.alternations,
                   t.epochs, data=data)
    assert len(res.C) == t.c_max == len(set(res.C))
    assert res.C[:t.n_c0] == C0
    assert all(0 <= e < m for e in res.C)
    for k, add in enumerate(res.added):
        cand, mean = res.mean_scores[k]
        assert not set(add) & set(res.C[:t.n_c0 + t.K * k])
        assert add == ct.select_top(mean, cand, t.K)
    # Adam descends on both losses within an alternation
    assert res.loss_w[0][-1] < res.loss_w[0][0]
    assert res.loss_s[0][-1] < res.loss_s[0][0]
    # the inputs were not modified
    assert not np.shares_memory(res.Ws[-1], t.wnet_weights[-1])
    assert (res.Ws[-1] != t.wnet_weights[-1]).any()
