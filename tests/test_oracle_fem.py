"""Pins of the oracle's element, mass and cubature routines (Sec. 3.1, Sec. 5)."""
import numpy as np
import pytest

from oracle import fem
from paper_2102_11026_amd import synth

rng = np.random.default_rng(3)
MU, LAM = fem.lame(1e5, 0.45)


def one_tet(perturb=0.0):
    X = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.1]], float) + rng.normal(size=(4, 3)) * 0.01
    T = np.array([[0, 1, 2, 3]], np.int32)
    Bm, Ve = fem.rest_shape(X, T)
    u = rng.normal(size=12) * perturb
    return X, T, Bm, Ve, u


def test_rest_state_has_no_stress_and_linear_stiffness():
    X, T, Bm, Ve, _ = one_tet()
    u = np.zeros(12)
    f, K = fem.element_force_stiffness(X, T, u, Bm, Ve, MU, LAM)
    assert np.abs(f).max() < 1e-10
    # textbook linear-elastic tet: K = V B^T D B with the Voigt strain operator
    G = np.vstack([-Bm[0].sum(axis=0), Bm[0]])  # (4, 3): gradient of each hat function
    Bv = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = G[a]
        Bv[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz], [gy, gx, 0], [0, gz, gy], [gz, 0, gx]]
    D = np.zeros((6, 6))
    D[:3, :3] = LAM
    D[np.arange(3), np.arange(3)] = LAM + 2 * MU
    D[np.arange(3, 6), np.arange(3, 6)] = MU
    np.testing.assert_allclose(K[0], Ve[0] * Bv.T @ D @ Bv, rtol=1e-10, atol=1e-6)


def test_force_and_stiffness_against_finite_differences():
    X, T, Bm, Ve, u = one_tet(perturb=0.004)
    f, K = fem.element_force_stiffness(X, T, u, Bm, Ve, MU, LAM)
    eps = 1e-7
    E = lambda uu: fem.total_energy(X, T, uu, Ve, Bm, MU, LAM)
    fd_f = np.array([(E(u + eps * e) - E(u - eps * e)) / (2 * eps) for e in np.eye(12)])
    np.testing.assert_allclose(f[0], fd_f, rtol=1e-5, atol=1e-4)
    fd_K = np.stack([(fem.element_force_stiffness(X, T, u + eps * e, Bm, Ve, MU, LAM)[0][0]
                      - fem.element_force_stiffness(X, T, u - eps * e, Bm, Ve, MU, LAM)[0][0]) / (2 * eps)
                     for e in np.eye(12)], axis=1)
    np.testing.assert_allclose(K[0], fd_K, rtol=1e-5, atol=1e-2)
    np.testing.assert_allclose(K[0], K[0].T, rtol=1e-12, atol=1e-8)


def test_force_balance_and_torque_free():
    X, T, Bm, Ve, u = one_tet(perturb=0.01)
    f, _ = fem.element_force_stiffness(X, T, u, Bm, Ve, MU, LAM)
    fv = f[0].reshape(4, 3)
    assert np.abs(fv.sum(axis=0)).max() < 1e-9 * np.abs(fv).max()
    x = X + u.reshape(4, 3)
    assert np.abs(np.cross(x, fv).sum(axis=0)).max() < 1e-9 * np.abs(fv).max()


def test_energy_rotation_invariance():
    F = np.eye(3) + 0.1 * rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Q *= np.sign(np.linalg.det(Q))
    assert fem.energy_density(Q @ F, MU, LAM) == pytest.approx(fem.energy_density(F, MU, LAM), rel=1e-12)
    # P = dPsi/dF by central differences
    P = fem.piola(F[None], MU, LAM)[0]
    eps = 1e-7
    for i in range(3):
        for j in range(3):
            E = np.zeros((3, 3))
            E[i, j] = eps
            d = (fem.energy_density(F + E, MU, LAM) - fem.energy_density(F - E, MU, LAM)) / (2 * eps)
            assert P[i, j] == pytest.approx(d, rel=1e-5, abs=1e-2)


def test_inverted_element_is_reported():
    X, T, Bm, Ve, _ = one_tet()
    u = np.zeros(12)
    u[3] = -0.25  # push vertex 1 through the opposite face
    with pytest.raises(fem.InvertedElement):
        fem.element_force_stiffness(X, T, u, Bm, Ve, MU, LAM)


def test_grid_mesh_volume_and_mass():
    X, T = synth.grid_mesh(3, 4, 5, spacing=0.1)
    Bm, Ve = fem.rest_shape(X, T)
    assert np.all(Ve > 0)
    assert Ve.sum() == pytest.approx(2 * 3 * 4 * 1e-3, rel=1e-12)
    m = fem.lumped_mass(T, Ve, 1000.0, X.shape[0])
    assert m.sum() / 3 == pytest.approx(1000.0 * 0.024, rel=1e-12)
    # conforming: every interior face shared by exactly two tets
    faces = {}
    for t in T:
        for skip in range(4):
            key = tuple(sorted(np.delete(t, skip)))
            faces[key] = faces.get(key, 0) + 1
    counts = np.array(list(faces.values()))
    assert counts.max() == 2
    n_boundary = (counts == 1).sum()
    assert n_boundary == 2 * 2 * (2 * 3 + 2 * 4 + 3 * 4)


def test_full_quadrature_force_is_energy_gradient():
    p = synth.tiny_problem(name="quad")
    Bm, Ve = fem.rest_shape(p.X, p.tets)
    u = rng.normal(size=p.N) * 0.003
    Jt = rng.normal(size=(p.N, 4))
    w = np.ones(p.tets.shape[0])
    ids = np.arange(p.tets.shape[0])
    f_int, fr, Kr = fem.cubature_force_stiffness(p.X, p.tets, u, Jt, ids, w, Bm, Ve, MU, LAM)
    eps = 1e-7
    E = lambda uu: fem.total_energy(p.X, p.tets, uu, Ve, Bm, MU, LAM)
    for i in rng.choice(p.N, 6, replace=False):
        e = np.zeros(p.N)
        e[i] = eps
        assert f_int[i] == pytest.approx((E(u + e) - E(u - e)) / (2 * eps), rel=1e-5, abs=1e-3)
    np.testing.assert_allclose(fr, Jt.T @ f_int, rtol=1e-12)
    # reduced stiffness = d(fr)/dr along u + Jt r (Jt fixed)
    fd = np.stack([(fem.cubature_force_stiffness(p.X, p.tets, u + eps * Jt[:, k], Jt, ids, w, Bm, Ve, MU, LAM)[1]
                    - fem.cubature_force_stiffness(p.X, p.tets, u - eps * Jt[:, k], Jt, ids, w, Bm, Ve, MU, LAM)[1])
                   / (2 * eps) for k in range(4)], axis=1)
    np.testing.assert_allclose(Kr, fd, rtol=1e-5, atol=1e-2)
