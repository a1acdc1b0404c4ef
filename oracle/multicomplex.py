"""Multicomplex numbers C^n in FP64 (test infrastructure only, see package header).

Sec. 4.1 defines C^0 = R and C^n = {z1 + z2 i_n : z1, z2 in C^(n-1)}, with
commuting imaginary units i_k^2 = -1.  An element of C^n is stored as a
numpy array whose LAST axis has 2**n entries; entry c is the coefficient of
the product of the units i_k whose bit (k-1) is set in c.  So the first half
of the last axis is z1 and the second half is z2 in the recursive split on
the highest unit i_n.

Every operation here recurses on that split down to real numpy arithmetic:
  (a + b i_n)(c + d i_n) = (ac - bd) + (ad + bc) i_n
  exp(a + b i_n)  = exp(a) (cos b + i_n sin b)
  sin(a + b i_n)  = sin a cosh b + i_n cos a sinh b
  cos(a + b i_n)  = cos a cosh b - i_n sin a sinh b
  sinh(a + b i_n) = sinh a cos b + i_n cosh a sin b
  cosh(a + b i_n) = cosh a cos b + i_n sinh a sin b
  (a + b i_n)^-1  = (a - b i_n) (a^2 + b^2)^-1
which are the addition theorems of the elementary functions with i_n^2=-1.
The first-order sine printed in Appendix A has its factors swapped; the
textbook form above is used, and the Appendix's second-order sine formulas
are a test pin for this module.  The third order is obtained by the same
recursion rather than by expanding the Appendix's partial listing.

Parity: pinned (Appendix A second-order sine, the Cauchy-Riemann real-matrix
form of Sec. 6.7, algebraic identities, complex-step derivative identities).
"""
from __future__ import annotations

import numpy as np


def order(z: np.ndarray) -> int:
    n = int(round(np.log2(z.shape[-1])))
    assert 2 ** n == z.shape[-1]
    return n


def split(z: np.ndarray):
    h = z.shape[-1] // 2
    return z[..., :h], z[..., h:]


def join(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.concatenate([a, b], axis=-1)


def real(x, n: int) -> np.ndarray:
    """Embed a real array into C^n."""
    x = np.asarray(x, dtype=np.float64)
    z = np.zeros(x.shape + (2 ** n,))
    z[..., 0] = x
    return z


def re(z: np.ndarray) -> np.ndarray:
    """Fully real component."""
    return z[..., 0]


def mul(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    if x.shape[-1] == 1:
        return x * y
    a, b = split(x)
    c, d = split(y)
    return join(mul(a, c) - mul(b, d), mul(a, d) + mul(b, c))


def exp(z):
    if z.shape[-1] == 1:
        return np.exp(z)
    a, b = split(z)
    ea = exp(a)
    return join(mul(ea, cos(b)), mul(ea, sin(b)))


def sin(z):
    if z.shape[-1] == 1:
        return np.sin(z)
    a, b = split(z)
    return join(mul(sin(a), cosh(b)), mul(cos(a), sinh(b)))


def cos(z):
    if z.shape[-1] == 1:
        return np.cos(z)
    a, b = split(z)
    return join(mul(cos(a), cosh(b)), -mul(sin(a), sinh(b)))


def sinh(z):
    if z.shape[-1] == 1:
        return np.sinh(z)
    a, b = split(z)
    return join(mul(sinh(a), cos(b)), mul(cosh(a), sin(b)))


def cosh(z):
    if z.shape[-1] == 1:
        return np.cosh(z)
    a, b = split(z)
    return join(mul(cosh(a), cos(b)), mul(sinh(a), sin(b)))


def inv(z):
    if z.shape[-1] == 1:
        return 1.0 / z
    a, b = split(z)
    d = inv(mul(a, a) + mul(b, b))
    return join(mul(a, d), -mul(b, d))


def tanh(z):
    return mul(sinh(z), inv(cosh(z)))


def elu(z):
    """ELU with alpha = 1, branching on the fully real component."""
    pos = re(z) > 0
    neg = exp(z)
    neg[..., 0] -= 1.0
    return np.where(pos[..., None], z, neg)


def identity(z):
    return z


def one(shape, n: int) -> np.ndarray:
    return real(np.ones(shape), n)


# activation functions and their first derivative, both as maps C^n -> C^n
def act(name: str):
    return {"tanh": tanh, "elu": elu, "sin": sin, "identity": identity}[name]


def dact(name: str):
    """sigma'(z) evaluated in the same algebra as z."""
    if name == "tanh":
        def d(z):
            t = tanh(z)
            o = -mul(t, t)
            o[..., 0] += 1.0
            return o
        return d
    if name == "elu":
        def d(z):
            pos = re(z) > 0
            return np.where(pos[..., None], one(z.shape[:-1], order(z)), exp(z))
        return d
    if name == "sin":
        return cos
    if name == "identity":
        return lambda z: one(z.shape[:-1], order(z))
    raise ValueError(name)


def cr_matrix(z: np.ndarray) -> np.ndarray:
    """Cauchy-Riemann real-matrix form of one multicomplex number (Sec. 6.7):
    z = z0 + z1 i_n  ->  [[CR(z0), -CR(z1)], [CR(z1), CR(z0)]], recursively."""
    if z.shape[-1] == 1:
        return z.reshape(1, 1)
    a, b = split(z)
    A, B = cr_matrix(a), cr_matrix(b)
    return np.block([[A, -B], [B, A]])
