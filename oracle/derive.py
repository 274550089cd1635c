"""Lattice parameters from the physical problem statement (TEST INFRASTRUCTURE).

Lattice units: dx = dt = 1, rho0 = 1, mu_m = 1.
  nu  = cs2 (tau_f - 1/2)                       (Sec. V)
  eta = cs2m (tau_m - 1/2)                      (Sec. IV)
  Ha  = B0 a sqrt(sigma/(rho nu)), sigma = 1/(eta mu_m)   (Sec. VIII)
      => B0 = Ha sqrt(rho nu eta) / a
  U_ref = a^2 F_x / (rho nu)                    (Sec. VIII) => F_x from u_max
  B_ref = a^2 F_x mu_m sqrt(sigma/(rho nu))     (Sec. VIII)
  Couette scale of B: U_w sqrt(rho nu sigma) mu_m         (App. C)
"""
from __future__ import annotations

import math

from . import LINK, Params
from .analytic import chang_lundgren_centre


def nu_of(tau_f: float) -> float:
    return (tau_f - 0.5) / 3.0


def eta_of(tau_m: float) -> float:
    return (tau_m - 0.5) / 3.0


def trt_times(tau_f: float, tau_m: float, lambda_f: float, lambda_m: float):
    """The free TRT relaxation times from the magic parameters.

    Lambda = (tau+ - 1/2)(tau- - 1/2) for each distribution.  For f, tau_f is
    the even-part time (it sets nu) and the odd-part time tau_fm follows; for
    g, tau_m is the odd-part time (it sets eta) and the even-part time tau_mp
    follows.  Returns (tau_fm, tau_mp).
    """
    return 0.5 + lambda_f / (tau_f - 0.5), 0.5 + lambda_m / (tau_m - 0.5)


def mrt_rates(tau_f: float, tau_m: float, lambda_f: float, lambda_m: float,
              s_e: float = 1.64, s_eps: float = 1.54):
    """MRT rates (s_fe, s_feps, s_fq, s_me, s_md).  The energy modes of f take
    s_e and s_eps (defaults: Lallemand & Luo 2000's stability choice); the
    odd q modes of f and both second-order modes of g take the TRT rates of
    the magic parameters, so that s_e = s_eps = 1/tau_f makes MRT the TRT of
    (lambda_f, lambda_m)."""
    tau_fm, tau_mp = trt_times(tau_f, tau_m, lambda_f, lambda_m)
    return s_e, s_eps, 1.0 / tau_fm, 1.0 / tau_mp, 1.0 / tau_mp


def half_width(ny: int, bc: int) -> float:
    return ny / 2.0 if bc == LINK else (ny - 1) / 2.0


def b0_of(ha: float, tau_f: float, tau_m: float, a: float, rho: float = 1.0) -> float:
    return ha * math.sqrt(rho * nu_of(tau_f) * eta_of(tau_m)) / a


def fx_for_umax(u_max: float, ha: float, c: float, tau_f: float, a: float,
                rho: float = 1.0) -> float:
    """Body force whose Chang-Lundgren centreline velocity is u_max."""
    return u_max * rho * nu_of(tau_f) / (a * a * chang_lundgren_centre(ha, c))


def b_ref_hartmann(fx: float, tau_f: float, tau_m: float, a: float, rho: float = 1.0) -> float:
    return a * a * fx / math.sqrt(rho * nu_of(tau_f) * eta_of(tau_m))


def u_ref_hartmann(fx: float, tau_f: float, a: float, rho: float = 1.0) -> float:
    return a * a * fx / (rho * nu_of(tau_f))


def b_ref_couette(u_w: float, tau_f: float, tau_m: float, rho: float = 1.0) -> float:
    return u_w * math.sqrt(rho * nu_of(tau_f) / eta_of(tau_m))


def hartmann_params(nx: int, ny: int, bc: int, tau_f: float, tau_m: float,
                    ha: float, c: float, u_max: float) -> Params:
    """Body-force-driven Hartmann channel with equal wall conductance c."""
    a = half_width(ny, bc)
    return Params(nx=nx, ny=ny, bc=bc, tau_f=tau_f, tau_m=tau_m,
                  b0=b0_of(ha, tau_f, tau_m, a),
                  fx=fx_for_umax(u_max, ha, c, tau_f, a),
                  c_lo=c, c_hi=c, a=a, extra={"ha": ha, "u_max": u_max})


def couette_params(nx: int, ny: int, bc: int, tau_f: float, tau_m: float,
                   ha: float, c_lo: float, c_hi: float, u_w: float) -> Params:
    """Shear-driven Hartmann-Couette channel, upper wall moving at u_w."""
    a = half_width(ny, bc)
    return Params(nx=nx, ny=ny, bc=bc, tau_f=tau_f, tau_m=tau_m,
                  b0=b0_of(ha, tau_f, tau_m, a), fx=0.0,
                  c_lo=c_lo, c_hi=c_hi, u_lo=0.0, u_hi=u_w, a=a,
                  extra={"ha": ha, "u_w": u_w})
