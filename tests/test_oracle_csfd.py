"""Pins of complex-step differentiation in the oracle (eq. cfd, eq. mcfd_hessian,
Fig. bp of Sec. 4.4)."""
import json
import os

import numpy as np
import pytest

from oracle import decoder as dec
from oracle import multicomplex as mc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f_scalar(z):
    """e^x sin x in any multicomplex order."""
    return mc.mul(mc.exp(z), mc.sin(z))


@pytest.mark.parametrize("h", [1e-10, 1e-20, 1e-30, 1e-100])
def test_first_order_cfd_has_no_cancellation(h):
    x = np.linspace(-2, 2, 9)
    z = mc.real(x, 1)
    z[:, 1] = h
    d = f_scalar(z)[:, 1] / h
    np.testing.assert_allclose(d, np.exp(x) * (np.sin(x) + np.cos(x)), rtol=2e-15, atol=1e-15)


def test_second_order_mcfd_hessian():
    """eq. mcfd_hessian on f(x, y) = sin(x) y^3."""
    h = 1e-20
    x0, y0 = 0.7, -1.3

    def f(x, y):
        return mc.mul(mc.sin(x), mc.mul(y, mc.mul(y, y)))

    def c2(xi1, xi2, yi1, yi2):
        x = mc.real(x0, 2)
        y = mc.real(y0, 2)
        x[1], x[2], y[1], y[2] = xi1, xi2, yi1, yi2
        return f(x, y)[3] / h ** 2

    assert c2(h, h, 0, 0) == pytest.approx(-np.sin(x0) * y0 ** 3, rel=1e-14)
    assert c2(0, 0, h, h) == pytest.approx(6 * np.sin(x0) * y0, rel=1e-14)
    assert c2(h, 0, 0, h) == pytest.approx(3 * np.cos(x0) * y0 ** 2, rel=1e-14)


def test_third_order_derivative_is_step_invariant():
    """i1 i2 i3 / h^3 of sin(x + h i1 + h i2 + h i3) is -cos x for any tiny h."""
    x0 = 0.4
    for h in (1e-10, 1e-20, 1e-40):
        z = mc.real(x0, 3)
        z[1] = z[2] = z[4] = h
        assert mc.sin(z)[7] / h ** 3 == pytest.approx(-np.cos(x0), rel=1e-14)


def test_fig_bp_worked_example():
    """Complex-step BP through z = x y, w = z^2 from x = 2 + h i, y = 3."""
    g = json.load(open(os.path.join(GOLD, "fig_bp_example.json")))
    h = 1e-20
    layers = [dec.Product(), dec.Square()]
    x = mc.real(np.array([[g["x"]], [g["y"]]]), 1)
    x[0, 0, 1] = h
    w, tape = dec.forward(layers, x)
    # dw/dz = 2 z, the printed intermediate
    dwdz = layers[1].vjp(tape[1], mc.real(np.ones((1, 1)), 1))
    assert dwdz[0, 0, 0] == pytest.approx(g["printed"]["dw_dz"]["re"], rel=1e-15)
    assert dwdz[0, 0, 1] / h == pytest.approx(g["printed"]["dw_dz"]["im_over_h"], rel=1e-15)
    xbar = dec.backward(layers, tape, mc.real(np.ones((1, 1)), 1))
    ref = g["completed_by_hand"]
    assert xbar[0, 0, 0] == pytest.approx(ref["xbar"]["re"], rel=1e-15)
    assert xbar[0, 0, 1] / h == pytest.approx(ref["xbar"]["im_over_h"], rel=1e-15)
    assert xbar[1, 0, 0] == pytest.approx(ref["ybar"]["re"], rel=1e-15)
    assert xbar[1, 0, 1] / h == pytest.approx(ref["ybar"]["im_over_h"], rel=1e-15)


def test_nested_central_differences_fail_where_csfd_does_not():
    """Sec. 6.6: recursive central differences for a third derivative are far
    off at every step tried while the complex step is exact to rounding."""
    x0 = 0.4
    exact = -np.cos(x0)
    z = mc.real(x0, 3)
    z[1] = z[2] = z[4] = 1e-20
    assert abs(mc.sin(z)[7] / 1e-60 - exact) < 1e-15
    for h in (1e-3, 1e-5, 1e-7, 1e-9):
        d3 = (np.sin(x0 + 2 * h) - 2 * np.sin(x0 + h) + 2 * np.sin(x0 - h) - np.sin(x0 - 2 * h)) / (2 * h ** 3)
        assert abs(d3 - exact) > 1e-7
