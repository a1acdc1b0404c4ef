"""Pins of the oracle's multicomplex algebra (Sec. 4.1, Sec. 6.7, Appendix A)."""
import json
import os

import numpy as np
import pytest

from oracle import multicomplex as mc

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(7)


def rand_mc(n, shape=()):
    return rng.normal(size=shape + (2 ** n,))


def test_appendix_a_second_order_sine():
    """The Appendix's bicomplex sine, term by term, at generic (not small) parts."""
    spec = json.load(open(os.path.join(GOLD, "appendix_a_sin2.json")))
    fns = dict(sin=np.sin, cos=np.cos, sinh=np.sinh, cosh=np.cosh)
    for _ in range(20):
        a, b, c, d = rng.normal(size=4) * 1.5
        got = mc.sin(np.array([a, b, c, d]))  # components 1, i1, i2, i1 i2
        for k, name in enumerate(["a'", "b'", "c'", "d'"]):
            val = 0.0
            for sign, f1, f2, f3, f4 in spec["terms"][name]:
                t = fns[f1](a) * fns[f2](b) * fns[f3](c) * fns[f4](d)
                val += t if sign == "+" else -t
            assert got[k] == pytest.approx(val, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("fname", ["exp", "sin", "cos", "sinh", "cosh", "tanh"])
def test_first_order_matches_library_complex(fname):
    """C^1 is the complex plane: compare with numpy's complex functions."""
    z = rand_mc(1, (50,))
    got = getattr(mc, fname)(z)
    ref = getattr(np, fname)(z[:, 0] + 1j * z[:, 1])
    np.testing.assert_allclose(got[:, 0], ref.real, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(got[:, 1], ref.imag, rtol=1e-13, atol=1e-14)


def test_bicomplex_as_pairs_of_complex():
    """C^2 = {z1 + z2 i2}, z1, z2 complex: product against numpy complex arithmetic."""
    x, y = rand_mc(2, (30,)), rand_mc(2, (30,))
    c = lambda v, lo: v[:, lo] + 1j * v[:, lo + 1]
    a, b, cc, d = c(x, 0), c(x, 2), c(y, 0), c(y, 2)
    got = mc.mul(x, y)
    lo, hi = a * cc - b * d, a * d + b * cc
    np.testing.assert_allclose(got[:, 0] + 1j * got[:, 1], lo, rtol=1e-13)
    np.testing.assert_allclose(got[:, 2] + 1j * got[:, 3], hi, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_cauchy_riemann_form_is_a_homomorphism(n):
    """eq. cr_form: the 2^n x 2^n real matrix of a product is the product of matrices."""
    for _ in range(5):
        x, y = rand_mc(n), rand_mc(n)
        np.testing.assert_allclose(mc.cr_matrix(mc.mul(x, y)), mc.cr_matrix(x) @ mc.cr_matrix(y),
                                   rtol=1e-12, atol=1e-12)
    z = np.array([0.3, -1.2])
    np.testing.assert_array_equal(mc.cr_matrix(z), [[0.3, 1.2], [-1.2, 0.3]])


def test_algebra_laws_c3():
    x, y, z = rand_mc(3, (10,)), rand_mc(3, (10,)), rand_mc(3, (10,))
    np.testing.assert_allclose(mc.mul(x, y), mc.mul(y, x), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(mc.mul(mc.mul(x, y), z), mc.mul(x, mc.mul(y, z)), rtol=1e-12, atol=1e-12)
    # distributivity
    np.testing.assert_allclose(mc.mul(x, y + z), mc.mul(x, y) + mc.mul(x, z), rtol=1e-12, atol=1e-12)


def test_function_identities_c3():
    z = 0.7 * rand_mc(3, (10,))
    one = mc.one((10,), 3)
    s, c = mc.sin(z), mc.cos(z)
    np.testing.assert_allclose(mc.mul(s, s) + mc.mul(c, c), one, atol=1e-12)
    sh, ch = mc.sinh(z), mc.cosh(z)
    np.testing.assert_allclose(mc.mul(ch, ch) - mc.mul(sh, sh), one, atol=1e-12)
    np.testing.assert_allclose(mc.mul(mc.exp(z), mc.exp(-z)), one, atol=1e-12)
    np.testing.assert_allclose(mc.mul(z, mc.inv(z)), one, atol=1e-11)
    np.testing.assert_allclose(mc.mul(mc.tanh(z), ch), sh, atol=1e-12)
    # exp(z) = cosh z + sinh z
    np.testing.assert_allclose(mc.exp(z), ch + sh, atol=1e-12)


def test_unit_squares_to_minus_one():
    for n in (1, 2, 3):
        for k in range(n):
            e = np.zeros(2 ** n)
            e[1 << k] = 1.0
            sq = mc.mul(e, e)
            ref = np.zeros(2 ** n)
            ref[0] = -1.0
            np.testing.assert_array_equal(sq, ref)


def test_elu_closed_form_values():
    """ELU with alpha = 1 (Sec. 3.5 activations): exp(x) - 1 for x <= 0 and x
    for x > 0.  At x = -ln 2 the value is -1/2 and every derivative is
    exp(-ln 2) = 1/2, so along units i1, i2, i3 of step h the tricomplex
    components are -1/2, h/2, h^2/2 and h^3/2; dropping the "- 1" of the
    negative branch, or branching the wrong way, fails this."""
    h = 1e-5
    z = mc.real(-np.log(2.0), 3)
    z[1] = z[2] = z[4] = h          # i1, i2, i3
    y = mc.elu(z)
    assert y[0] == pytest.approx(-0.5, rel=1e-9)
    for comp, k in ((1, 1), (2, 1), (4, 1), (3, 2), (5, 2), (6, 2), (7, 3)):
        assert y[comp] == pytest.approx(0.5 * h ** k, rel=1e-9), comp
    # positive branch: the identity, every unit passes through unchanged
    z = mc.real(0.7, 3)
    z[1:] = rng.normal(size=7)
    np.testing.assert_array_equal(mc.elu(z), z)
    # C^1 at generic parts: exp(a + bi) - 1 in library complex arithmetic
    a, b = -np.abs(rng.normal(size=20)) - 0.1, rng.normal(size=20)
    got = mc.elu(np.stack([a, b], axis=-1))
    ref = np.exp(a + 1j * b) - 1.0
    np.testing.assert_allclose(got[:, 0], ref.real, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got[:, 1], ref.imag, rtol=1e-13, atol=1e-15)
