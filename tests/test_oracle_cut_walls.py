"""Pins of the oracle's link-based Hartmann walls at a cut distance q != 1/2
(the wall q nodes beyond the wall row; orc_link_closure_q).

* Continuity: as q -> 1/2 the closure becomes the paper's half-way closure
  (the interpolations, the curvature and shear corrections and the mass
  correction all vanish there), so runs at q = 1/2 +- 1e-7 differ from the
  half-way run by O(1e-7).
* Exact solutions: steady Hartmann flow (Chang-Lundgren) and
  Hartmann-Couette flow with a moving wall and unequal conductances, with the
  half-width a = (ny - 1)/2 + q and nodes at y = q - a + j, converge to the
  closed forms under refinement (error ratios near 4 per doubling:
  2.8-4.9 from 16 to 32 and 64 rows), for q = 0.25, 0.75 and 1 and
  insulating and conducting walls.
* Mass: the interpolated bounce-back alone lets mass through a wall when
  the populations are asymmetric about its normal (the Lorentz force's
  normal part does that); the correction returns it, so mass is exact.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, Params, analytic, derive


def steady(p, tol=1e-11, chunk=2000, max_steps=600_000):
    s = oracle.init_state(p)
    prev, n = None, 0
    while n < max_steps:
        oracle.run(p, s, chunk, nthreads=8)
        n += chunk
        o = oracle.observe(p, s)
        if prev is not None and max(np.linalg.norm(o[k] - prev[k]) / np.linalg.norm(o[k])
                                    for k in ("ux", "bx")) < tol:
            return o
        prev = o
    raise AssertionError("no steady state")


def hartmann_errors(ny, q, ha, c, tau=0.8):
    a = (ny - 1) / 2.0 + q
    nu = eta = (tau - 0.5) / 3.0
    fx = derive.fx_for_umax(0.02, ha, c, tau, a)
    p = Params(nx=1, ny=ny, bc=LINK, tau_f=tau, tau_m=tau, b0=ha * math.sqrt(nu * eta) / a,
               fx=fx, c_lo=c, c_hi=c, q_lo=q, q_hi=q)
    assert p.half_width() == a
    o = steady(p)
    us, bs = analytic.chang_lundgren((np.arange(ny) + q - a) / a, ha, c)
    U, B = a * a * fx / nu, a * a * fx / math.sqrt(nu * eta)
    return (np.linalg.norm(o["ux"][:, 0] - U * us) / np.linalg.norm(U * us),
            np.linalg.norm(o["bx"][:, 0] - B * bs) / np.linalg.norm(B * bs))


def couette_errors(ny, q, ha, cl, ch, tau=0.8, U=0.02):
    a = (ny - 1) / 2.0 + q
    nu = eta = (tau - 0.5) / 3.0
    p = Params(nx=1, ny=ny, bc=LINK, tau_f=tau, tau_m=tau, b0=ha * math.sqrt(nu * eta) / a,
               c_lo=cl, c_hi=ch, u_hi=U, q_lo=q, q_hi=q)
    o = steady(p)
    us, bs = analytic.hartmann_couette((np.arange(ny) + q - a) / a, ha, cl, ch)
    B = U * math.sqrt(nu / eta)
    return (np.linalg.norm(o["ux"][:, 0] - U * us) / np.linalg.norm(U * us),
            np.linalg.norm(o["bx"][:, 0] - B * bs) / np.linalg.norm(B * bs))


@pytest.mark.parametrize("q", [0.25, 0.75, 1.0])
@pytest.mark.parametrize("ha,c", [(5.0, 0.0), (5.0, 0.5), (5.0, 2.0)])
def test_hartmann_flow_between_cut_walls_converges(q, ha, c):
    e16, e32 = hartmann_errors(16, q, ha, c), hartmann_errors(32, q, ha, c)
    for k in range(2):
        assert e32[k] < 5e-2 and e16[k] / e32[k] > 2.7, (e16, e32)


@pytest.mark.parametrize("q", [0.25, 0.75, 1.0])
@pytest.mark.parametrize("ha,cl,ch", [(5.0, 0.5, 2.0), (4.0, 0.0, 1.0)])
def test_hartmann_couette_flow_between_cut_walls_converges(q, ha, cl, ch):
    e16, e32 = couette_errors(16, q, ha, cl, ch), couette_errors(32, q, ha, cl, ch)
    for k in range(2):
        assert e32[k] < 2e-2 and e16[k] / e32[k] > 2.7, (e16, e32)


def random_state(p, seed):
    from paper_2112_13930_amd.workloads import random_populations
    return random_populations(p.nx, p.ny, seed=seed, b0=p.b0)


@pytest.mark.parametrize("c", [0.0, 0.6, math.inf])
def test_cut_closure_tends_to_the_half_way_closure(c):
    kw = dict(nx=9, ny=12, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=c, c_hi=c,
              u_lo=-0.02, u_hi=0.03)
    s0 = random_state(Params(**kw), seed=13)
    half = oracle.run(Params(**kw), s0.copy(), 20)
    for dq in (1e-7, -1e-7):
        near = oracle.run(Params(**kw, q_lo=0.5 + dq, q_hi=0.5 + dq), s0.copy(), 20)
        d = np.abs(near - half).max()
        assert 1e-12 < d < 1e-5, d


def test_cut_walls_conserve_mass():
    p = Params(nx=10, ny=12, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=0.3,
               c_hi=math.inf, u_lo=-0.02, u_hi=0.04, q_lo=0.3, q_hi=0.85)
    s = random_state(p, seed=17)
    m0 = s[:9].sum()
    oracle.run(p, s, 50)
    assert abs(s[:9].sum() - m0) / m0 < 1e-14
