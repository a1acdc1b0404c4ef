"""Pins of the oracle's decoder derivatives (Sec. 4.3 right contractions,
Sec. 4.4 left contractions, Sec. 3.5 filter)."""
import numpy as np
import pytest

from oracle import decoder as dec
from paper_2102_11026_amd import synth

rng = np.random.default_rng(11)


def net(widths, scale=1.0, bias=0.3):
    Ws = [rng.normal(size=(widths[l + 1], widths[l])) * scale / np.sqrt(widths[l])
          for l in range(len(widths) - 1)]
    bs = [bias * rng.normal(size=widths[l + 1]) for l in range(len(widths) - 1)]
    return Ws, bs


def test_jacobian_against_central_differences():
    Ws, bs = net([4, 16, 16, 30])
    q = rng.normal(size=4) * 0.5
    for act in ("tanh", "elu", "sin"):
        J = dec.full_jacobian(Ws, bs, act, q)
        eps = 1e-6
        fd = np.stack([(dec.mlp_real(Ws, bs, act, q + eps * e) - dec.mlp_real(Ws, bs, act, q - eps * e)) / (2 * eps)
                       for e in np.eye(4)], axis=1)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-8)


def test_one_layer_tanh_closed_forms():
    """m(q) = W2 tanh(W1 q + b1) + b2: J, H, S and every contraction in closed form."""
    nq, hid, out = 3, 7, 11
    Ws, bs = net([nq, hid, out])
    W1, W2 = Ws
    q, dq, v = rng.normal(size=nq), rng.normal(size=nq) * 0.1, rng.normal(size=nq)
    t = np.tanh(W1 @ q + bs[0])
    t1, t2, t3 = 1 - t ** 2, -2 * t * (1 - t ** 2), -2 * (1 - t ** 2) * (1 - 3 * t ** 2)
    J = W2 @ (t1[:, None] * W1)
    H = np.einsum("oh,h,hk,hl->okl", W2, t2, W1, W1)
    S = np.einsum("oh,h,hk,hl,hm->oklm", W2, t3, W1, W1, W1)
    np.testing.assert_allclose(dec.full_jacobian(Ws, bs, "tanh", q), J, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(dec.full_hessian(Ws, bs, "tanh", q), H, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dec.full_third(Ws, bs, "tanh", q), S, rtol=1e-12, atol=1e-13)
    rc = dec.right_contractions(Ws, bs, "tanh", q, dq, v)
    np.testing.assert_allclose(rc["m"], W2 @ t + bs[1], rtol=1e-14)
    np.testing.assert_allclose(rc["J"], J, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(rc["Hdq"], H @ dq, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rc["Hv"], H @ v, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rc["Sdd"], S @ dq @ dq, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rc["Hdd"], H @ dq @ dq, rtol=1e-12, atol=1e-14)
    s = rng.normal(size=out)
    g, B = dec.left_contraction(Ws, bs, "tanh", q, s)
    np.testing.assert_allclose(g, J.T @ s, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(B, np.einsum("o,okl->kl", s, H), rtol=1e-12, atol=1e-13)


def test_identity_activation_is_linear():
    Ws, bs = net([3, 8, 8, 20])
    q = rng.normal(size=3)
    Wprod = Ws[2] @ Ws[1] @ Ws[0]
    np.testing.assert_allclose(dec.full_jacobian(Ws, bs, "identity", q), Wprod, rtol=1e-13, atol=1e-14)
    assert np.abs(dec.full_hessian(Ws, bs, "identity", q)).max() == 0.0
    assert np.abs(dec.full_third(Ws, bs, "identity", q)).max() == 0.0
    rc = dec.right_contractions(Ws, bs, "identity", q, rng.normal(size=3), rng.normal(size=3))
    for k in ("Hdq", "Sdd", "Hv", "Hdd"):
        assert np.abs(rc[k]).max() == 0.0


@pytest.mark.parametrize("act", ["tanh", "elu", "sin"])
def test_symmetry_of_H_and_S(act):
    Ws, bs = net([3, 10, 10, 10, 12])
    q = rng.normal(size=3) * 0.5
    H = dec.full_hessian(Ws, bs, act, q)
    S = dec.full_third(Ws, bs, act, q)
    np.testing.assert_allclose(H, np.swapaxes(H, 1, 2), rtol=1e-12, atol=1e-14)
    for perm in [(0, 2, 1, 3), (0, 1, 3, 2), (0, 3, 2, 1)]:
        np.testing.assert_allclose(S, np.transpose(S, perm), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("act", ["tanh", "elu", "sin"])
def test_collective_contractions_equal_exhaustive_tensors(act):
    """The n_q collective passes reproduce the full tensors contracted, with
    the second and third units scaled by every element of dq."""
    nq = 4
    Ws, bs = net([nq, 12, 12, 12, 25])
    q = rng.normal(size=nq) * 0.5
    dq, v = rng.normal(size=nq) * 0.2, rng.normal(size=nq)
    H = dec.full_hessian(Ws, bs, act, q)
    S = dec.full_third(Ws, bs, act, q)
    rc = dec.right_contractions(Ws, bs, act, q, dq, v)
    np.testing.assert_allclose(rc["Hdq"], H @ dq, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rc["Hv"], H @ v, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rc["Sdd"], S @ dq @ dq, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rc["Hdd"], H @ dq @ dq, rtol=1e-11, atol=1e-13)
    s = rng.normal(size=25)
    g, B = dec.left_contraction(Ws, bs, act, q, s)
    np.testing.assert_allclose(g, dec.full_jacobian(Ws, bs, act, q).T @ s, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(B, np.einsum("o,okl->kl", s, H), rtol=1e-11, atol=1e-13)
    # delta_J of eq. delta_j from the same tensors
    dt = 1 / 60
    np.testing.assert_allclose(dec.delta_J(rc, dt), S @ dq @ dq + H @ (3 * dq - dt * v), rtol=1e-11, atol=1e-13)


def test_hessian_against_central_differences_of_jacobian():
    Ws, bs = net([3, 9, 9, 14])
    q = rng.normal(size=3) * 0.5
    H = dec.full_hessian(Ws, bs, "elu", q)
    eps = 1e-6
    for k in range(3):
        e = np.eye(3)[k]
        fd = (dec.full_jacobian(Ws, bs, "elu", q + eps * e) - dec.full_jacobian(Ws, bs, "elu", q - eps * e)) / (2 * eps)
        np.testing.assert_allclose(H[:, :, k], fd, rtol=1e-5, atol=1e-8)


def test_filter_makes_decoder_orthogonal_to_U():
    """U^T D = 0 for D = P (I - U U^T) m when U has zero pinned rows (Sec. 3.6)."""
    p = synth.tiny_problem(n_p=3, name="filt")
    pin = np.repeat(p.pinned, 3)
    x = rng.normal(size=(p.N, 4))
    y = dec.filter_pin(x, p.U, pin)
    np.testing.assert_allclose(p.U.T @ y, 0.0, atol=1e-13)
    assert np.all(y[pin == 1] == 0)
    # transpose consistency: <P(I-UU^T)x, a> = <x, (I-UU^T)P a>
    a = rng.normal(size=p.N)
    assert float(y[:, 0] @ a) == pytest.approx(float(x[:, 0] @ dec.filter_pin_T(a, p.U, pin)), rel=1e-12)
