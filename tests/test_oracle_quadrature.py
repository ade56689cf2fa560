"""Pins for the 7-point triangle rule (Radon's degree-5 rule)."""

import math

import numpy as np
import pytest

from oracle import quadrature as quad


def _exact_monomial(a, b):
    # integral of x^a y^b over the unit right triangle (0,0),(1,0),(0,1)
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def _rule(a, b):
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    p = quad.points(tri)
    return 0.5 * np.sum(quad.WEIGHTS * p[:, 0] ** a * p[:, 1] ** b)


@pytest.mark.parametrize("deg", range(6))
def test_exact_to_degree_5(deg):
    for a in range(deg + 1):
        b = deg - a
        assert _rule(a, b) == pytest.approx(_exact_monomial(a, b), rel=1e-14, abs=1e-16)


def test_not_exact_at_degree_6():
    errs = [abs(_rule(a, 6 - a) - _exact_monomial(a, 6 - a)) for a in range(7)]
    assert max(errs) > 1e-6


def test_weights_and_points():
    assert quad.WEIGHTS.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(quad.BARY.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(quad.BARY > 0)  # interior points only
