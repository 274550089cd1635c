"""Pins for the closed forms in oracle/analytic.py.

Each profile is checked against the boundary-value problem it solves, not
against a retyped copy of itself:
  * Chang-Lundgren (Sec. VIII): u'' + Ha B' + 1 = 0, B'' + Ha u' = 0,
    u(+-1) = 0, -B'(-1) + B(-1)/c = 0 and B'(1) + B(1)/c = 0.
  * Hartmann-Couette (App. C): u'' + Ha B' = 0, B'' + Ha u' = 0, u(-1) = 0,
    u(1) = 1, -B'(-1) + B(-1)/c_l = 0, B'(1) + B(1)/c_u = 0.
Derivatives by fourth-order central differences.
"""
import math

import numpy as np
import pytest

from oracle import analytic

H = 1e-3


def d1(fn, x):
    return (-fn(x + 2 * H) + 8 * fn(x + H) - 8 * fn(x - H) + fn(x - 2 * H)) / (12 * H)


def d2(fn, x):
    return (-fn(x + 2 * H) + 16 * fn(x + H) - 30 * fn(x) + 16 * fn(x - H) - fn(x - 2 * H)) / (12 * H * H)


def robin(B, dB, c, side):
    """Shercliff condition residual in nondimensional form (Sec. III)."""
    sgn = -1.0 if side == "lo" else 1.0
    if math.isinf(c):
        return dB
    if c == 0.0:
        return B
    return sgn * dB + B / c


CL_CASES = [(ha, c) for ha in (0.5, 5.0, 20.0) for c in (0.0, 0.1, 0.5, 1.0, 1e4, math.inf)]


@pytest.mark.parametrize("ha,c", CL_CASES)
def test_chang_lundgren_solves_bvp(ha, c):
    u = lambda x: analytic.chang_lundgren(x, ha, c)[0]
    b = lambda x: analytic.chang_lundgren(x, ha, c)[1]
    xi = np.linspace(-0.99, 0.99, 41)
    scale = max(np.abs(u(xi)).max(), np.abs(b(xi)).max(), 1e-3)
    assert np.abs(d2(u, xi) + ha * d1(b, xi) + 1.0).max() < 1e-5 * max(1.0, ha * ha)
    assert np.abs(d2(b, xi) + ha * d1(u, xi)).max() < 1e-5 * max(1.0, ha * ha)
    for side, x in (("lo", -1.0), ("hi", 1.0)):
        assert abs(u(np.array([x]))[0]) < 1e-13
        r = robin(b(np.array([x]))[0], d1(b, np.array([x]))[0], c, side)
        assert abs(r) < 1e-6 * max(1.0, scale * ha), (side, r)


CP_CASES = [(ha, cl, cu) for ha in (5.0, 20.0)
            for (cl, cu) in ((0.0, 0.0), (0.5, 0.5), (0.5, 0.0), (0.0, 0.5), (0.0, 0.1),
                             (0.0, 1.0), (0.0, 1e4), (0.0, math.inf), (math.inf, 0.3),
                             (0.2, 3.0))]


@pytest.mark.parametrize("ha,cl,cu", CP_CASES)
def test_hartmann_couette_solves_bvp(ha, cl, cu):
    u = lambda x: analytic.hartmann_couette(x, ha, cl, cu)[0]
    b = lambda x: analytic.hartmann_couette(x, ha, cl, cu)[1]
    xi = np.linspace(-0.99, 0.99, 41)
    tol = 1e-5 * max(1.0, ha * ha) * max(1.0, np.abs(b(xi)).max())
    assert np.abs(d2(u, xi) + ha * d1(b, xi)).max() < tol
    assert np.abs(d2(b, xi) + ha * d1(u, xi)).max() < tol
    assert abs(u(np.array([-1.0]))[0]) < 1e-12
    assert abs(u(np.array([1.0]))[0] - 1.0) < 1e-12
    for side, x, c in (("lo", -1.0, cl), ("hi", 1.0, cu)):
        r = robin(b(np.array([x]))[0], d1(b, np.array([x]))[0], c, side)
        assert abs(r) < 1e-6 * max(1.0, ha) * max(1.0, abs(b(np.array([x]))[0])), (side, r)


def test_couette_equal_walls_velocity_independent_of_c():
    """App. C: with c_wl = c_wu the velocity does not depend on c."""
    xi = np.linspace(-1, 1, 51)
    ref = analytic.hartmann_couette(xi, 5.0, 0.0, 0.0)[0]
    for c in (0.1, 0.5, 3.0, 1e4):
        assert np.abs(analytic.hartmann_couette(xi, 5.0, c, c)[0] - ref).max() < 1e-13
    assert np.abs(ref - 0.5 * (1 + np.sinh(5 * xi) / np.sinh(5.0))).max() < 1e-13


def test_couette_insulated_reduces_to_closed_form():
    """App. C, insulated walls: B* = (1 - cosh(Ha xi)/cosh(Ha)) / (2 tanh Ha)."""
    xi = np.linspace(-1, 1, 51)
    b = analytic.hartmann_couette(xi, 5.0, 0.0, 0.0)[1]
    ref = (1 - np.cosh(5 * xi) / np.cosh(5.0)) / (2 * np.tanh(5.0))
    assert np.abs(b - ref).max() < 1e-13


def test_chang_lundgren_small_ha_is_poiseuille():
    xi = np.linspace(-1, 1, 21)
    u, b = analytic.chang_lundgren(xi, 1e-4, 0.3)
    assert np.abs(u - 0.5 * (1 - xi ** 2)).max() < 1e-6
    assert np.abs(b).max() < 1e-4


def test_infinite_c_is_limit_of_large_c():
    xi = np.linspace(-1, 1, 21)
    for ha in (5.0, 20.0):
        u1, b1 = analytic.chang_lundgren(xi, ha, 1e12)
        u2, b2 = analytic.chang_lundgren(xi, ha, math.inf)
        assert np.abs(u1 - u2).max() < 1e-10 and np.abs(b1 - b2).max() < 1e-10
        u1, b1 = analytic.hartmann_couette(xi, ha, 0.3, 1e12)
        u2, b2 = analytic.hartmann_couette(xi, ha, 0.3, math.inf)
        assert np.abs(u1 - u2).max() < 1e-10 and np.abs(b1 - b2).max() < 1e-9
