"""Cubature weight prediction at inference (test infrastructure only).

Sec. 5.2: a plain MLP maps the generalized coordinate to non-negative
weights of the cubature tets and is evaluated once per time step.  The
paper's trained net ends in a square; the synthetic stand-in applies a
softplus after every layer (positive and smooth) and multiplies by a fixed
scale, so that at zero pre-activation every weight equals |mesh| / |C|.

Parity: pinned by a closed form (zero weights give the scale times ln 2 at
every layer's output; see the tests).
"""
from __future__ import annotations

import numpy as np


def softplus(x):
    return np.logaddexp(0.0, x)


def wnet_weights(Ws, bs, scale, r):
    z = np.asarray(r, np.float64)
    for W, b in zip(Ws, bs):
        z = softplus(W @ z + b)
    return scale * z
