"""Pins of the test's exact Riemann solver (Toro ch. 4) before it is used to
pin the scheme: published star states and jump conditions."""
import math

import pytest

from exact_riemann import sample, star_state


def test_sod_star_state_textbook():
    # Toro, Table 4.3, test 1: p* = 0.30313, u* = 0.92745
    p, u = star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert p == pytest.approx(0.30313, abs=1e-5)
    assert u == pytest.approx(0.92745, abs=1e-5)


def test_123_problem_star_state_textbook():
    # Toro, Table 4.3, test 2: p* = 0.00189, u* = 0.0
    p, u = star_state((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 1.4)
    assert p == pytest.approx(0.00189, abs=1e-5)
    assert abs(u) < 1e-12


def test_rankine_hugoniot_across_right_shock():
    g = 1.4
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    p, u = star_state(L, R, g)
    cr = math.sqrt(g * R[2] / R[0])
    S = R[1] + cr * math.sqrt((g + 1) / (2 * g) * p / R[2] + (g - 1) / (2 * g))
    rs, us, ps = sample(L, R, g, S - 1e-9)
    rr, ur, pr = R
    # mass, momentum, energy jump conditions in the shock frame
    def flux(r, v, pp):
        E = pp / (g - 1) + 0.5 * r * v * v
        return (r * v - S * r, r * v * v + pp - S * r * v, v * (E + pp) - S * E)
    a, b = flux(rs, us, ps), flux(rr, ur, pr)
    for x, y in zip(a, b):
        assert abs(x - y) < 1e-9


def test_vacuum_opens_for_fast_double_rarefaction():
    # the paper's double rarefaction (u = -+2, p = 0.1) opens a vacuum
    assert star_state((1.0, -2.0, 0.1), (1.0, 2.0, 0.1), 1.4) is None
    r, u, p = sample((1.0, -2.0, 0.1), (1.0, 2.0, 0.1), 1.4, 0.0)
    assert r == 0.0 and p == 0.0
