"""Decoder passes in multicomplex arithmetic (test infrastructure only).

The decoder m(q) is the MLP z_0 = q, z_l = sigma(W_l z_{l-1} + b_l) for the
hidden layers and m = W_L z_{L-1} + b_L (Sec. 3.5).  The decoder part of the
autoencoder appends the fixed filtering layer (I - U U^T) of Sec. 3.5; the
Dirichlet mask P of pinned DOFs is applied after it, D(q) = P (I - U U^T) m(q).

Derivatives follow Sec. 4:
  * right contractions (Sec. 4.3): for each latent index j one tricomplex
    forward pass from q + h e_j i1 + h dq i2 + h dq i3 (i1 at element j, i2
    and i3 scaled by every element of dq = q - qbar).  Its components give
        i1 / h           = J e_j
        i1 i2 / h^2      = H(e_j, dq)
        i1 i2 i3 / h^3   = S(e_j, dq, dq)
        i2 i3 / h^2      = H(dq, dq)
    and one bicomplex pass from q + h e_j i1 + h qdot_bar i2 gives
        i1 i2 / h^2      = H(e_j, qdot_bar)
    (eq. mcfd_hessian generalised to directions, Sec. 4.1 / 4.3);
  * left contractions (Sec. 4.4): complex-step backpropagation.  A complex
    forward pass from q + h e_j i, then backpropagation of g = s . m(q) run
    entirely in complex arithmetic; the input adjoint holds Re = m_q^T s and
    Im / h = column j of the Hessian of g, i.e. of s . H.

Layers act on each multicomplex component separately because the weights are
real (the block structure of the Cauchy-Riemann form, Sec. 6.7).

Parity: pinned by central differences, closed-form one-layer tanh
derivatives, identity-activation weight products, symmetry of H and S,
exhaustive full-tensor contractions and the worked example of Fig. bp.
"""
from __future__ import annotations

from typing import List

import numpy as np

from . import multicomplex as mc

H_CS = 1e-20  # complex-step size in FP64: no subtractive cancellation (eq. cfd)


# --------------------------------------------------------------------------
# layers with a complex-capable forward and vector-Jacobian product
# --------------------------------------------------------------------------
class Linear:
    def __init__(self, W: np.ndarray, b: np.ndarray):
        self.W = np.asarray(W, np.float64)
        self.b = np.asarray(b, np.float64)

    def forward(self, x):
        # x: (n_in, cols, 2^n); real weights act on every component
        y = np.einsum("oi,ick->ock", self.W, x)
        y[..., 0] += self.b[:, None]
        return y

    def vjp(self, x, ybar):
        return np.einsum("oi,ock->ick", self.W, ybar)


class Activation:
    def __init__(self, name: str):
        self.name = name
        self.f = mc.act(name)
        self.df = mc.dact(name)

    def forward(self, x):
        return self.f(x)

    def vjp(self, x, ybar):
        return mc.mul(self.df(x), ybar)


class Product:
    """Two inputs (rows 0, 1) -> their product (one row)."""

    def forward(self, x):
        return mc.mul(x[0:1], x[1:2])

    def vjp(self, x, ybar):
        return np.concatenate([mc.mul(ybar, x[1:2]), mc.mul(ybar, x[0:1])], axis=0)


class Square:
    def forward(self, x):
        return mc.mul(x, x)

    def vjp(self, x, ybar):
        return 2.0 * mc.mul(ybar, x)


def mlp_layers(weights: List[np.ndarray], biases: List[np.ndarray], act: str):
    layers = []
    L = len(weights)
    for l in range(L):
        layers.append(Linear(weights[l], biases[l]))
        if l < L - 1:
            layers.append(Activation(act))
    return layers


def forward(layers, x):
    """Run ``x`` through ``layers``; returns the output and the tape of inputs."""
    tape = []
    for layer in layers:
        tape.append(x)
        x = layer.forward(x)
    return x, tape


def backward(layers, tape, ybar):
    """Backpropagate ``ybar`` with every product taken in the multicomplex
    algebra of the forward pass (complex-step BP, Sec. 4.4)."""
    for layer, x in zip(reversed(layers), reversed(tape)):
        ybar = layer.vjp(x, ybar)
    return ybar


# --------------------------------------------------------------------------
# filter and pin mask
# --------------------------------------------------------------------------
def filter_pin(x: np.ndarray, U: np.ndarray, pin_dof: np.ndarray) -> np.ndarray:
    """P (I - U U^T) x applied column-wise to x with N rows (Sec. 3.5)."""
    y = x - U @ (U.T @ x) if U.shape[1] else x.copy()
    keep = (pin_dof == 0).astype(np.float64)
    return y * (keep[:, None] if y.ndim == 2 else keep)


def filter_pin_T(x: np.ndarray, U: np.ndarray, pin_dof: np.ndarray) -> np.ndarray:
    """(P (I - U U^T))^T x = (I - U U^T) P x."""
    keep = (pin_dof == 0).astype(np.float64)
    y = x * keep
    return y - U @ (U.T @ y) if U.shape[1] else y


# --------------------------------------------------------------------------
# collective right contractions (Sec. 4.3)
# --------------------------------------------------------------------------
def right_contractions(weights, biases, act, q, dq, qdot_bar, n_rows=None, h=H_CS):
    """Decoder output m(q) and its contracted derivatives, before the filter.

    Returns a dict of arrays with n_rows rows (default: every output):
      m    (n,)      m(q)
      J    (n, nq)   J e_j
      Hdq  (n, nq)   H(e_j, dq)
      Sdd  (n, nq)   S(e_j, dq, dq)
      Hv   (n, nq)   H(e_j, qdot_bar)
      Hdd  (n,)      H(dq, dq)
    """
    q = np.asarray(q, np.float64)
    nq = q.size
    layers = mlp_layers(weights, biases, act)
    eye = np.eye(nq)
    # tricomplex: components bit0 = i1, bit1 = i2, bit2 = i3
    z = mc.real(np.repeat(q[:, None], nq, axis=1), 3)
    z[..., 1] = h * eye                       # i1 at element j for pass j
    z[..., 2] = h * np.asarray(dq)[:, None]   # i2 along dq
    z[..., 4] = h * np.asarray(dq)[:, None]   # i3 along dq
    y3, _ = forward(layers, z)
    # bicomplex: bit0 = i1 (e_j), bit1 = i2 (qdot_bar)
    z2 = mc.real(np.repeat(q[:, None], nq, axis=1), 2)
    z2[..., 1] = h * eye
    z2[..., 2] = h * np.asarray(qdot_bar)[:, None]
    y2, _ = forward(layers, z2)
    rows = slice(0, n_rows)
    return dict(
        m=y3[rows, 0, 0],
        J=y3[rows, :, 1] / h,
        Hdq=y3[rows, :, 3] / h ** 2,
        Sdd=y3[rows, :, 7] / h ** 3,
        Hdd=y3[rows, 0, 6] / h ** 2,
        Hv=y2[rows, :, 3] / h ** 2,
    )


def delta_J(rc: dict, dt: float, trimmed: bool = False) -> np.ndarray:
    """eq. delta_j: (S . dq) . dq + H . (3 dq - dt qdot_bar), per column j.

    trimmed: the derivative of M J w_r alone, H . (dq - dt qdot_bar), which is
    what remains of the Newton matrix once the fictitious force is dropped
    (its derivative M (S . dq . dq + 2 H . dq) is the rest of eq. delta_j)."""
    if trimmed:
        return rc["Hdq"] - dt * rc["Hv"]
    return rc["Sdd"] + 3.0 * rc["Hdq"] - dt * rc["Hv"]


# --------------------------------------------------------------------------
# left contraction by complex-step backpropagation (Sec. 4.4)
# --------------------------------------------------------------------------
def left_contraction(weights, biases, act, q, s, h=H_CS):
    """For g(q) = s . m(q): returns (grad g = m_q^T s, Hessian of g = s . H).

    One complex forward pass per latent index j (all j as columns of one
    batch, Sec. 4.4), then complex BP seeded with s.
    """
    q = np.asarray(q, np.float64)
    nq = q.size
    layers = mlp_layers(weights, biases, act)
    z = mc.real(np.repeat(q[:, None], nq, axis=1), 1)
    z[..., 1] = h * np.eye(nq)
    y, tape = forward(layers, z)
    s_full = np.zeros(y.shape[0])
    s_full[: s.size] = s
    ybar = mc.real(np.repeat(s_full[:, None], nq, axis=1), 1)
    qbar = backward(layers, tape, ybar)
    grad = qbar[:, 0, 0]
    hess = qbar[:, :, 1] / h  # column j from pass j
    return grad, hess


# --------------------------------------------------------------------------
# exhaustive full tensors (independent brute-force routes for the tests)
# --------------------------------------------------------------------------
def full_jacobian(weights, biases, act, q, h=H_CS):
    q = np.asarray(q, np.float64)
    nq = q.size
    layers = mlp_layers(weights, biases, act)
    z = mc.real(np.repeat(q[:, None], nq, axis=1), 1)
    z[..., 1] = h * np.eye(nq)
    y, _ = forward(layers, z)
    return y[:, :, 1] / h


def full_hessian(weights, biases, act, q, h=H_CS):
    """H[:, k, l] from one bicomplex pass per pair (k, l) (eq. mcfd_hessian)."""
    q = np.asarray(q, np.float64)
    nq = q.size
    layers = mlp_layers(weights, biases, act)
    pairs = [(k, l) for k in range(nq) for l in range(nq)]
    z = mc.real(np.repeat(q[:, None], len(pairs), axis=1), 2)
    for c, (k, l) in enumerate(pairs):
        z[k, c, 1] += h
        z[l, c, 2] += h
    y, _ = forward(layers, z)
    return (y[:, :, 3] / h ** 2).reshape(-1, nq, nq)


def full_third(weights, biases, act, q, h=H_CS):
    """S[:, k, l, m] from one tricomplex pass per triple."""
    q = np.asarray(q, np.float64)
    nq = q.size
    layers = mlp_layers(weights, biases, act)
    trip = [(k, l, m) for k in range(nq) for l in range(nq) for m in range(nq)]
    z = mc.real(np.repeat(q[:, None], len(trip), axis=1), 3)
    for c, (k, l, m) in enumerate(trip):
        z[k, c, 1] += h
        z[l, c, 2] += h
        z[m, c, 4] += h
    y, _ = forward(layers, z)
    return (y[:, :, 7] / h ** 3).reshape(-1, nq, nq, nq)


def mlp_real(weights, biases, act, q):
    """Plain real forward pass m(q)."""
    y, _ = forward(mlp_layers(weights, biases, act), mc.real(np.asarray(q, np.float64)[:, None], 0))
    return y[:, 0, 0]
