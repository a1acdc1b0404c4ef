"""Recursive central finite differences of the decoder (test infrastructure).

The comparison of CSFD with finite differences (Sec. 4.1 and the FD
comparison of Sec. 6): the same contractions as the collective complex-step
passes, obtained by applying the central difference (f(x + h v) -
f(x - h v)) / (2 h) recursively, on plain real forward passes and on real
backpropagation.  With m the raw decoder output and e_j the j-th unit vector,

    J e_j        = [m(q + h e_j) - m(q - h e_j)] / (2h)
    H(e_j, v)    = [m(+e_j +v) - m(-e_j +v) - m(+e_j -v) + m(-e_j -v)] / (4h^2)
    S(e_j,dq,dq) = [g(q + h e_j) - g(q - h e_j)] / (2h),
                   g(x) = [m(x + 2h dq) - 2 m(x) + m(x - 2h dq)] / (4h^2)
    H(dq, dq)    = g(q)
    m_q^T s      = grad (s . m)(q)        (real backpropagation)
    (s . H) e_j  = [grad (s . m)(q + h e_j) - grad (s . m)(q - h e_j)] / (2h)

where (+e_j +v) is short for q + h e_j + h v.  Every evaluation is made in the
given floating-point type (float64 or float32), the perturbed inputs
included, so the subtractive cancellation the paper names is reproduced in
the precision of choice.  Independent of oracle/decoder.py (own forward and
backward passes) and of the HIP path.
"""
from __future__ import annotations

import numpy as np


def _act(name, x):
    if name == "tanh":
        return np.tanh(x)
    if name == "elu":
        return np.where(x > 0, x, np.expm1(np.minimum(x, 0)))
    if name == "sin":
        return np.sin(x)
    if name == "identity":
        return x
    raise ValueError(name)


def _dact(name, x):
    if name == "tanh":
        t = np.tanh(x)
        return 1 - t * t
    if name == "elu":
        return np.where(x > 0, np.ones_like(x), np.exp(np.minimum(x, 0)))
    if name == "sin":
        return np.cos(x)
    if name == "identity":
        return np.ones_like(x)
    raise ValueError(name)


def mlp(weights, biases, act, Q, dtype=np.float64):
    """Outputs m(Q[:, c]) for every column c of Q (n_q x cols), in dtype."""
    z = np.asarray(Q, dtype)
    L = len(weights)
    for l, (W, b) in enumerate(zip(weights, biases)):
        z = np.asarray(W, dtype) @ z + np.asarray(b, dtype)[:, None]
        if l < L - 1:
            z = _act(act, z).astype(dtype)
    return z


def mlp_grad(weights, biases, act, Q, s, dtype=np.float64):
    """grad_q (s . m)(Q[:, c]) for every column c (n_q x cols): real BP."""
    z = np.asarray(Q, dtype)
    pre = []
    L = len(weights)
    for l, (W, b) in enumerate(zip(weights, biases)):
        x = np.asarray(W, dtype) @ z + np.asarray(b, dtype)[:, None]
        if l < L - 1:
            pre.append(x)
            z = _act(act, x).astype(dtype)
    g = np.repeat(np.asarray(s, dtype)[:, None], Q.shape[1], axis=1)
    for l in range(L - 1, -1, -1):
        g = np.asarray(weights[l], dtype).T @ g
        if l > 0:
            g = (_dact(act, pre[l - 1]) * g).astype(dtype)
    return g


def right_contractions_fd(weights, biases, act, q, dq, qdot_bar, n_rows=None, h=1e-3, dtype=np.float64):
    """Same keys as the collective complex-step contractions: m, J (cols j),
    Hdq = H(e_j, dq), Hv = H(e_j, qdot_bar), Sdd = S(e_j, dq, dq), Hdd."""
    q = np.asarray(q, dtype)
    dq = np.asarray(dq, dtype)
    qd = np.asarray(qdot_bar, dtype)
    h = dtype(h)
    nq = q.size
    E = np.eye(nq, dtype=dtype) * h
    cols = [q]
    for j in range(nq):
        cols += [q + E[j], q - E[j]]
    for v in (h * dq, h * qd, 2 * h * dq):
        for j in range(nq):
            cols += [q + E[j] + v, q - E[j] + v, q + E[j] - v, q - E[j] - v]
    cols += [q + 2 * h * dq, q - 2 * h * dq]
    Y = mlp(weights, biases, act, np.stack(cols, axis=1), dtype)
    if n_rows is not None:
        Y = Y[:n_rows]
    m = Y[:, 0]
    pm = lambda j: (Y[:, 1 + 2 * j], Y[:, 2 + 2 * j])
    base = 1 + 2 * nq
    four = lambda blk, j: [Y[:, base + 4 * (blk * nq + j) + k] for k in range(4)]
    J = np.stack([(pm(j)[0] - pm(j)[1]) / (2 * h) for j in range(nq)], axis=1)
    Hdq, Hv, Sdd = [], [], []
    for j in range(nq):
        a, b, c, d = four(0, j)
        Hdq.append((a - b - c + d) / (4 * h * h))
        a, b, c, d = four(1, j)
        Hv.append((a - b - c + d) / (4 * h * h))
        pp, mp, pm_, mm = four(2, j)   # (+e_j +2dq), (-e_j +2dq), (+e_j -2dq), (-e_j -2dq)
        plus, minus = pm(j)
        g_plus = (pp - 2 * plus + pm_) / (4 * h * h)
        g_minus = (mp - 2 * minus + mm) / (4 * h * h)
        Sdd.append((g_plus - g_minus) / (2 * h))
    Hdd = (Y[:, -2] - 2 * m + Y[:, -1]) / (4 * h * h)
    f64 = lambda x: np.asarray(x, np.float64)
    return dict(m=f64(m), J=f64(J), Hdq=f64(np.stack(Hdq, axis=1)), Hv=f64(np.stack(Hv, axis=1)),
                Sdd=f64(np.stack(Sdd, axis=1)), Hdd=f64(Hdd))


def left_contraction_fd(weights, biases, act, q, s, h=1e-3, dtype=np.float64):
    """(m_q^T s, s . H) from real backpropagation at q and q +- h e_j."""
    q = np.asarray(q, dtype)
    h = dtype(h)
    nq = q.size
    E = np.eye(nq, dtype=dtype) * h
    cols = [q] + [q + E[j] for j in range(nq)] + [q - E[j] for j in range(nq)]
    s_full = np.zeros(np.asarray(weights[-1]).shape[0])
    s_full[: np.size(s)] = s  # the seed covers the first N output rows
    G = mlp_grad(weights, biases, act, np.stack(cols, axis=1), s_full, dtype)
    grad = G[:, 0]
    hess = (G[:, 1:1 + nq] - G[:, 1 + nq:]) / (2 * h)
    return np.asarray(grad, np.float64), np.asarray(hess, np.float64)
