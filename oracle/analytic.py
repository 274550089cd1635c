"""Closed-form steady profiles used to pin the oracle (TEST INFRASTRUCTURE).

* Chang-Lundgren Hartmann flow between thin conducting walls (Sec. VIII,
  first subsection): body-force-driven, equal wall conductance c_w on both
  walls, nondimensional u*(xi) = u/U_ref and B*(xi) = B_x/B_ref, xi = y/a.
* Hartmann-Couette flow with different wall conductance ratios (App. C,
  Eqs. 1DMHDmovingwallfinalsolution and 1DMHDmovingwallintconstants): the upper
  wall moves at U_w, u* = u/U_w, B* = B_x / (U_w sqrt(rho nu sigma) mu_m).

Conductance ratios may be ``inf``.  App. C writes its constants with
phi = c_wl / c_wu, which is undefined at c_wu = 0 although (c_wu, c_wl) =
(0, 0.5) is one of the paper's cases; the constants are therefore evaluated in
the equivalent form (1 + phi) c_wu = c_wu + c_wl and phi c_wu^2 = c_wu c_wl,
identical wherever phi is defined.
"""
from __future__ import annotations

import math

import numpy as np


def chang_lundgren(xi, ha: float, c: float):
    """(u*, B*) of the conducting-wall Hartmann flow at xi in [-1, 1].

    u* = (1/Ha) K [1 - cosh(Ha xi)/cosh(Ha)],
    B* = -xi/Ha + (1/Ha) K sinh(Ha xi)/cosh(Ha),
    K  = (c + 1)/(Ha c + tanh Ha)   (-> 1/Ha as c -> inf).
    Ha -> 0 reduces to plane Poiseuille u* = (1 - xi^2)/2, B* = 0.
    """
    xi = np.asarray(xi, dtype=np.float64)
    if ha == 0.0:
        return 0.5 * (1.0 - xi ** 2), np.zeros_like(xi)
    t = math.tanh(ha)
    K = 1.0 / ha if math.isinf(c) else (c + 1.0) / (ha * c + t)
    ch = math.cosh(ha)
    u = (K / ha) * (1.0 - np.cosh(ha * xi) / ch)
    b = -xi / ha + (K / ha) * np.sinh(ha * xi) / ch
    return u, b


def chang_lundgren_centre(ha: float, c: float) -> float:
    """u*(0), used to set F_x from a target centreline velocity."""
    return float(chang_lundgren(np.array([0.0]), ha, c)[0][0])


def couette_constants(ha: float, c_lo: float, c_hi: float):
    """(K1, K2) of App. C with phi = c_lo/c_hi eliminated.

    K1 = (t + c_u H) / (2 t + (c_u + c_l) H)
    K2 = (1 + (c_u + c_l)/2 H (t + 1/t) + c_u c_l H^2) / (2 t + (c_u + c_l) H)
    with H = Ha, t = tanh(Ha).  Infinite ratios take the limits; with both walls
    perfectly conducting B* is fixed only up to a constant and K2 is NaN.
    """
    H = ha
    t = math.tanh(H)
    s = t + 1.0 / t
    if math.isinf(c_hi) and math.isinf(c_lo):
        return 0.5, float("nan")
    if math.isinf(c_hi):
        return 1.0, 0.5 * s + c_lo * H
    if math.isinf(c_lo):
        return 0.0, 0.5 * s + c_hi * H
    den = 2.0 * t + (c_hi + c_lo) * H
    K1 = (t + c_hi * H) / den
    K2 = (1.0 + 0.5 * (c_hi + c_lo) * H * s + c_hi * c_lo * H * H) / den
    return K1, K2


def hartmann_couette(xi, ha: float, c_lo: float, c_hi: float):
    """(u*, B*) of the shear-driven flow, upper wall moving (App. C)."""
    xi = np.asarray(xi, dtype=np.float64)
    K1, K2 = couette_constants(ha, c_lo, c_hi)
    ch, sh = math.cosh(ha), math.sinh(ha)
    u = K1 + (0.5 - K1) * np.cosh(ha * xi) / ch + 0.5 * np.sinh(ha * xi) / sh
    b = K2 - (0.5 - K1) * np.sinh(ha * xi) / ch - 0.5 * np.cosh(ha * xi) / sh
    return u, b


def node_xi(ny: int, bc: int) -> np.ndarray:
    """xi = y/a of the lattice rows.

    Link-based walls sit half-way between the wall row and the ghost row
    (Sec. VI), so a = ny/2 and xi_j = (j + 1/2)/a - 1; moment-based walls sit
    on the wall rows (Sec. VII), so a = (ny-1)/2 and xi_j = j/a - 1.
    """
    j = np.arange(ny, dtype=np.float64)
    if bc == 0:
        a = ny / 2.0
        return (j + 0.5) / a - 1.0
    a = (ny - 1) / 2.0
    return j / a - 1.0
