"""Pins of the recursive central-difference decoder derivatives (oracle/fd.py)
against the complex-step contractions and against what floating point fixes
(the FD comparison of Sec. 6)."""
import numpy as np
import pytest

from oracle import decoder as dec
from oracle import fd
from paper_2102_11026_amd import synth

KEYS = ("J", "Hdq", "Hv", "Sdd", "Hdd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def setup(act="tanh", widths=(3, 16, 24, 48)):
    p = synth.tiny_problem(widths=widths, act=act, name=f"fd{act}", q_std=0.3)
    rng = np.random.default_rng(3)
    nq = p.n_q
    q = p.r0[p.n_p:] + rng.normal(size=nq) * 0.05
    dq, qd = rng.normal(size=nq) * 0.02, rng.normal(size=nq) * 0.5
    s = rng.normal(size=p.N)
    ex = dec.right_contractions(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N)
    _, B = dec.left_contraction(p.weights, p.biases, p.act, q, s)
    return p, q, dq, qd, s, ex, B


@pytest.mark.parametrize("act", ["tanh", "sin"])
def test_fd_converges_to_csfd_at_second_order(act):
    """Central differences are O(h^2): from h = 0.2 to 0.02 every contraction's
    error against the complex-step values drops by about 100 (at 0.01 the
    H(dq, dq) stencil, whose step is 2 h |dq|, already meets rounding)."""
    p, q, dq, qd, s, ex, B = setup(act)
    errs = {}
    for h in (2e-1, 2e-2):
        f = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=h)
        _, Bf = fd.left_contraction_fd(p.weights, p.biases, p.act, q, s, h=h)
        errs[h] = {k: rel(f[k], ex[k]) for k in KEYS} | {"B": rel(Bf, B)}
        assert rel(f["m"], ex["m"]) < 1e-13
    for k in errs[2e-1]:
        ratio = errs[2e-1][k] / errs[2e-2][k]
        assert 70 < ratio < 140, (k, errs[2e-1][k], errs[2e-2][k])


def test_elu_decoder_values_and_jacobian_match_the_independent_passes():
    """ELU (alpha = 1) is C^1 with a jump of its second derivative at 0, so
    stencils that straddle a kink do not converge at second order; the value
    and first-order channel still pin the multicomplex ELU against fd.py's
    plain real passes (np.expm1 on the negative branch): m(q) to rounding and
    the central-difference Jacobian at h = 1e-5 to its truncation error (a
    multicomplex ELU without the "- 1" of its negative branch fails the
    first check)."""
    p, q, dq, qd, s, ex, B = setup("elu")
    f = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=1e-5)
    assert rel(f["m"], ex["m"]) < 1e-13
    assert rel(f["J"], ex["J"]) < 1e-8


def test_fd_of_a_linear_decoder():
    """Identity activations: the first difference is exact and every higher
    one is zero up to the cancellation of a few ulps."""
    p, q, dq, qd, s, ex, B = setup("identity")
    f = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=1e-2)
    assert rel(f["J"], ex["J"]) < 1e-12
    scale = np.abs(f["m"]).max() + np.abs(f["J"]).max()
    for k in ("Hdq", "Hv", "Hdd"):
        assert np.abs(f[k]).max() < 1e-11 * scale / 1e-4
    assert np.abs(f["Sdd"]).max() < 1e-11 * scale / 1e-6


def test_fd_cancellation_profile():
    """The paper finds no step that works.  In FP32, the precision a GPU
    network runs in, the second- and third-order contractions are off by more
    than half at every step it tried (1e-3 ... 1e-9; at the smallest the
    perturbation vanishes in the input's rounding and they come out zero) while
    the first-order one is not; in FP64 the same stencils at h = 1e-3 are still
    accurate to 1e-3."""
    p, q, dq, qd, s, ex, B = setup("tanh")
    for h in (1e-3, 1e-5, 1e-7, 1e-9):
        f32 = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=h, dtype=np.float32)
        assert rel(f32["Sdd"], ex["Sdd"]) > 0.5, h
        assert rel(f32["Hdd"], ex["Hdd"]) > 0.5, h
    f32 = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=1e-3, dtype=np.float32)
    assert rel(f32["J"], ex["J"]) < 1e-3
    f64 = fd.right_contractions_fd(p.weights, p.biases, p.act, q, dq, qd, n_rows=p.N, h=1e-3)
    assert max(rel(f64[k], ex[k]) for k in KEYS) < 1e-3
