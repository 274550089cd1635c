"""Pins of the 3D oracle's rectangular duct: stationary link-closed Shercliff
side walls at z = -1/2 and nz - 1/2 besides the Hartmann walls.

* Continuum limit: x-invariant steady duct flow converges at second order to
  an independent finite-difference solution of the fully developed
  equations of Sec. II with the thin-wall condition on every wall
  (tests/duct_fd.py, itself checked against the Chang-Lundgren profile), for
  insulating, finitely and perfectly conducting Hartmann and side walls.
* y <-> z exchange: without an imposed field and with equal conductances on
  all walls, a square duct is symmetric under exchanging y and z (and the
  y and z components); this maps the side-wall closure onto the pinned
  Hartmann-wall link closure, edges included.
* z mirror: exchanging the two side walls mirrors the run (u_z, B_z odd).
* Conservation: mass with every wall stationary; sum B_x when every wall
  is perfectly conducting.
* Limits of the side closure: perfectly conducting walls bounce back the
  tangential field populations, insulating walls anti-bounce-back them.
"""
import math

import numpy as np
import pytest

from oracle import LINK, d3
from tests import duct_fd
from tests.test_oracle3d import random_state_3d


def duct_params(N, ha, cH, cS, nx=1, tau=0.8, fx_scale=1e-6, **kw):
    """cS: one conductance for both side walls, or (z = 0 side, z = nz-1 side)."""
    a = N / 2.0
    nu = eta = (tau - 0.5) / 3.0
    cs_lo, cs_hi = cS if isinstance(cS, tuple) else (cS, cS)
    return d3.Params3(nx=nx, ny=N, nz=N, bc=LINK, tau_f=tau, tau_m=tau,
                      b0=ha * math.sqrt(nu * eta) / a, fx=fx_scale * (16.0 / a) ** 2,
                      c_lo=cH, c_hi=cH, side_walls=True, cs_lo=cs_lo, cs_hi=cs_hi, **kw)


def steady(p, tol=1e-9, chunk=2000, max_steps=300_000):
    s = d3.init_state(p)
    prev, n = None, 0
    while n < max_steps:
        d3.run(p, s, chunk, nthreads=8)
        n += chunk
        o = d3.observe(p, s)
        if prev is not None and max(np.linalg.norm(o[k] - prev[k]) / np.linalg.norm(o[k])
                                    for k in ("ux", "bx")) < tol:
            return o
        prev = o
    raise AssertionError("no steady state")


def fd_errors(N, ha, cH, cS):
    p = duct_params(N, ha, cH, cS)
    o = steady(p)
    nu = eta = (p.tau_f - 0.5) / 3.0
    u, b = duct_fd.solve(N, N, nu, eta, p.b0, p.fx, cH, cH, p.cs_lo, p.cs_hi, m=9)
    ux, bx = o["ux"][:, :, 0], o["bx"][:, :, 0]
    return (np.linalg.norm(ux - u) / np.linalg.norm(u),
            np.linalg.norm(bx - b) / np.linalg.norm(b))


def test_fd_reference_matches_chang_lundgren():
    from oracle import analytic
    ny, nu, eta = 32, 0.1, 0.1
    a = ny / 2
    for ha, c in ((5.0, 0.1), (8.0, math.inf)):
        b0, fx = ha * math.sqrt(nu * eta) / a, 1e-6
        u, b = duct_fd.solve(ny, None, nu, eta, b0, fx, c, c, m=15)
        us, bs = analytic.chang_lundgren((np.arange(ny) + 0.5 - a) / a, ha, c)
        U, B = a * a * fx / nu, a * a * fx / math.sqrt(nu * eta)
        assert np.linalg.norm(u - U * us) / np.linalg.norm(U * us) < 1e-4
        db, ds = (b - b.mean(), B * (bs - bs.mean())) if math.isinf(c) else (b, B * bs)
        assert np.linalg.norm(db - ds) / np.linalg.norm(ds) < 1e-4


@pytest.mark.parametrize("ha,cH,cS", [(5.0, 0.1, 0.5), (5.0, 0.0, 0.0), (8.0, math.inf, 0.0),
                                      (5.0, 1.0, math.inf), (5.0, 0.3, (0.0, math.inf))])
def test_duct_converges_to_fd_solution_at_second_order(ha, cH, cS):
    e8 = fd_errors(8, ha, cH, cS)
    e16 = fd_errors(16, ha, cH, cS)
    for k in range(2):
        assert e16[k] < 0.05, (e8, e16)
        assert 3.2 < e8[k] / e16[k] < 4.4, (e8, e16)


def swap_yz(state):
    """The state with y and z exchanged: coordinates, velocities, field."""
    permf = [next(r for r in range(19) if (d3.EF[r] == d3.EF[q][[0, 2, 1]]).all()) for q in range(19)]
    permg = [next(r for r in range(7) if (d3.EG[r] == d3.EG[q][[0, 2, 1]]).all()) for q in range(7)]
    out = np.empty_like(state)
    t = np.transpose(state, (0, 2, 1, 3))  # [plane][z][y][x] -> [plane][y][z][x]
    for q in range(19):
        out[permf[q]] = t[q]
    for comp, comp2 in ((0, 0), (1, 2), (2, 1)):
        for q in range(7):
            out[19 + 7 * comp2 + permg[q]] = t[19 + 7 * comp + q]
    return out


@pytest.mark.parametrize("c", [0.0, 0.3, math.inf])
def test_square_duct_without_field_is_symmetric_under_y_z_exchange(c):
    p = d3.Params3(nx=5, ny=8, nz=8, bc=LINK, tau_f=0.75, tau_m=0.85, b0=0.0, fx=3e-5,
                   c_lo=c, c_hi=c, side_walls=True, cs_lo=c, cs_hi=c)
    s = random_state_3d(p, seed=21)
    a = d3.run(p, s.copy(), 12)
    b = swap_yz(d3.run(p, swap_yz(s), 12))
    assert np.abs(a - b).max() < 1e-15


def mirror_z(state):
    permf = [next(r for r in range(19) if (d3.EF[r] == d3.EF[q] * [1, 1, -1]).all()) for q in range(19)]
    permg = [next(r for r in range(7) if (d3.EG[r] == d3.EG[q] * [1, 1, -1]).all()) for q in range(7)]
    out = np.empty_like(state)
    t = state[:, ::-1]
    for q in range(19):
        out[permf[q]] = t[q]
    for comp in range(3):
        sign = -1.0 if comp == 2 else 1.0
        for q in range(7):
            out[19 + 7 * comp + permg[q]] = sign * t[19 + 7 * comp + q]
    return out


def test_exchanging_the_side_walls_mirrors_the_run():
    kw = dict(nx=4, ny=9, nz=7, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=0.2,
              c_hi=math.inf, u_hi=0.03, side_walls=True)
    p = d3.Params3(cs_lo=0.0, cs_hi=1.5, **kw)
    q = d3.Params3(cs_lo=1.5, cs_hi=0.0, **kw)
    s = random_state_3d(p, seed=5)
    a = d3.run(p, s.copy(), 10)
    b = mirror_z(d3.run(q, mirror_z(s), 10))
    assert np.abs(a - b).max() < 1e-15


def test_duct_conservation():
    p = d3.Params3(nx=4, ny=7, nz=6, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5,
                   c_lo=math.inf, c_hi=math.inf, side_walls=True, cs_lo=math.inf,
                   cs_hi=math.inf)
    s = random_state_3d(p, seed=3)
    m0 = s[:19].sum()
    bx0 = d3.observe(p, s)["bx"].sum()
    d3.run(p, s, 30)
    assert abs(s[:19].sum() - m0) / m0 < 1e-14
    bx = d3.observe(p, s)["bx"]
    assert abs(bx.sum() - bx0) < 1e-13 * max(1.0, np.abs(bx).sum())
    # with insulating side walls B_x is not conserved
    q = d3.Params3(**{**p.__dict__, "cs_lo": 0.0})
    s = random_state_3d(q, seed=3)
    d3.run(q, s, 30)
    assert abs(d3.observe(q, s)["bx"].sum() - bx0) > 1e-8


def test_side_closure_limits():
    rng = np.random.default_rng(7)
    own = rng.uniform(-0.1, 0.1, 40)
    f0, g0 = rng.uniform(0, 0.1, 19), rng.uniform(-0.1, 0.1, (7, 3))
    b0 = 0.05
    for wall, ez_in in ((0, 1), (1, -1)):
        q_in = [q for q in range(7) if d3.EG[q, 2] == ez_in][0]
        q_out = [q for q in range(7) if d3.EG[q, 2] == -ez_in][0]
        for cs, sign in ((math.inf, 1.0), (0.0, -1.0)):
            p = d3.Params3(nx=1, ny=4, nz=4, bc=LINK, tau_m=0.9, b0=b0, side_walls=True,
                           cs_lo=cs, cs_hi=cs)
            f, g = d3.side_closure(p, wall, own, f0, g0)
            w = 1.0 / 6.0
            assert g[q_in, 0] == sign * own[19 + q_out]
            assert math.isclose(g[q_in, 1] - w * b0, sign * (own[26 + q_out] - w * b0),
                                rel_tol=1e-15, abs_tol=1e-17)
            assert g[q_in, 2] == -own[33 + q_out]                 # B_z = 0 at any c
            for q in range(19):
                if d3.EF[q, 2] == ez_in:
                    r = [r for r in range(19) if (d3.EF[r] == -d3.EF[q]).all()][0]
                    assert f[q] == own[r]
                else:
                    assert f[q] == f0[q]
