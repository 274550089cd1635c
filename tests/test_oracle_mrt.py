"""Pins of the oracle's multiple-relaxation-time (MRT) collision.

The paper names multiple-relaxation-time collisions as a replacement for its
BGK operators (Secs. V and IX) without fixing a basis.  The reading: f in
the orthogonal D2Q9 basis of Lallemand & Luo (Phys. Rev. E 61 (2000) 6546)
with p_xx and p_xy at 1/tau_f (viscosity) and e, epsilon and q at free rates;
each component of g in the orthogonal D2Q5 basis (B, Lambda_x, Lambda_y,
epsilon, d) with Lambda at 1/tau_m (magnetic diffusivity) and epsilon, d at
free rates; each source moment with the weight 1 - s/2 of its rate.

* Reductions: with the even rates equal to TRT's (s_fe = s_feps = 1/tau_f,
  s_me = s_md = 1/tau_mp) and q at TRT's odd rate, MRT is the TRT step, a
  separately written and pinned operator; with every rate at 1/tau it is
  the BGK step.
* Poiseuille flow with half-way bounce-back at the magic parameter
  (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16: exact to round-off when s_e = s_nu, for
  any s_eps; with s_e != s_nu the energy mode, which the force feeds through
  u.F, leaves a deviation of relative size O(u^2) (it grows with fx^2).
* Exact solutions: steady Hartmann flow converges to the Chang-Lundgren
  profile at second order, with link and moment walls, insulating and
  conducting, for the default rates and for an arbitrary set.  A rate put
  on the wrong moment changes nu or eta and misses the profile by O(1).
* Uniform modes: in a uniform state at rest streaming is the identity away
  from the walls, so a non-equilibrium part put into one moment alone
  decays geometrically at that moment's rate, (1 - s)^n after n steps, and
  leaves every other moment at equilibrium.  Each free rate is checked on
  its own moment (e, epsilon, q_x, q_y, p_xx, p_xy of f; epsilon and d of
  each component of g).
* Conservation: mass with link walls.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, MRT, TRT, Params, analytic, derive


def mrt_params(tau_f=0.7, tau_m=0.9, rates=None, **kw):
    if rates is None:
        rates = derive.mrt_rates(tau_f, tau_m, 3.0 / 16.0, 0.25)
    s_fe, s_feps, s_fq, s_me, s_md = rates
    return Params(tau_f=tau_f, tau_m=tau_m, collision=MRT, s_fe=s_fe, s_feps=s_feps, s_fq=s_fq,
                  s_me=s_me, s_md=s_md, **kw)


def random_state(p, seed):
    from paper_2112_13930_amd.workloads import random_populations
    return random_populations(p.nx, p.ny, seed=seed, b0=p.b0)


KW = dict(nx=9, ny=12, b0=0.05, fx=2e-5, fy=-1e-5, c_lo=0.3, c_hi=math.inf, u_hi=0.03)


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_mrt_with_trt_rates_is_trt(bc):
    tfm, tmp = derive.trt_times(0.7, 0.9, 3.0 / 16.0, 0.25)
    t = Params(bc=bc, tau_f=0.7, tau_m=0.9, collision=TRT, tau_fm=tfm, tau_mp=tmp, **KW)
    m = mrt_params(bc=bc, rates=(1 / 0.7, 1 / 0.7, 1 / tfm, 1 / tmp, 1 / tmp), **KW)
    s0 = random_state(t, seed=21)
    st = oracle.run(t, s0.copy(), 30)
    assert np.abs(oracle.run(m, s0.copy(), 30) - st).max() < 1e-14
    # each free rate matters
    for k in range(5):
        r = [1 / 0.7, 1 / 0.7, 1 / tfm, 1 / tmp, 1 / tmp]
        r[k] += 0.1
        d = np.abs(oracle.run(mrt_params(bc=bc, rates=tuple(r), **KW), s0.copy(), 30) - st).max()
        assert d > 1e-9, (k, d)


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_mrt_with_equal_rates_is_bgk(bc):
    b = Params(bc=bc, tau_f=0.7, tau_m=0.9, **KW)
    m = mrt_params(bc=bc, rates=(1 / 0.7, 1 / 0.7, 1 / 0.7, 1 / 0.9, 1 / 0.9), **KW)
    s0 = random_state(b, seed=22)
    assert np.abs(oracle.run(m, s0.copy(), 30) - oracle.run(b, s0.copy(), 30)).max() < 1e-14


def poiseuille_error(tau_f, fx, s_e, s_eps, ny=16, steps=40000):
    rates = derive.mrt_rates(tau_f, 0.9, 3.0 / 16.0, 0.25, s_e=s_e, s_eps=s_eps)
    p = mrt_params(tau_f=tau_f, rates=rates, nx=1, ny=ny, bc=LINK, fx=fx)
    s = oracle.init_state(p)
    oracle.run(p, s, steps)
    ux = oracle.observe(p, s)["ux"][:, 0]
    a = ny / 2.0
    y = np.arange(ny) + 0.5 - a
    exact = fx / (2 * derive.nu_of(tau_f)) * (a * a - y * y)
    return np.abs(ux - exact).max() / exact.max()


@pytest.mark.parametrize("tau_f", [0.6, 1.5])
def test_mrt_poiseuille_exact_when_the_energy_mode_takes_the_viscous_rate(tau_f):
    assert poiseuille_error(tau_f, 1e-5, 1 / tau_f, 1.54) < 1e-10
    assert poiseuille_error(tau_f, 1e-5, 1 / tau_f, 1.1) < 1e-10


def test_mrt_poiseuille_deviation_is_second_order_in_the_velocity():
    e1, e2 = poiseuille_error(0.8, 1e-5, 1.64, 1.54), poiseuille_error(0.8, 1e-4, 1.64, 1.54)
    assert 1e-9 < e1 < 1e-7 and 90 < e2 / e1 < 110, (e1, e2)


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


def hartmann_errors(ny, bc, ha, c, rates, tau=0.8):
    a = ny / 2.0 if bc == LINK else (ny - 1) / 2.0
    nu = eta = (tau - 0.5) / 3.0
    fx = derive.fx_for_umax(0.02, ha, c, tau, a)
    p = mrt_params(tau_f=tau, tau_m=tau, rates=rates, nx=1, ny=ny, bc=bc,
                   b0=ha * math.sqrt(nu * eta) / a, fx=fx, c_lo=c, c_hi=c)
    o = steady(p)
    y = (np.arange(ny) + (0.5 if bc == LINK else 0.0) - a) / a
    us, bs = analytic.chang_lundgren(y, ha, c)
    U, B = a * a * fx / nu, a * a * fx / math.sqrt(nu * eta)
    return (np.linalg.norm(o["ux"][:, 0] - U * us) / np.linalg.norm(U * us),
            np.linalg.norm(o["bx"][:, 0] - B * bs) / np.linalg.norm(B * bs))


@pytest.mark.parametrize("rates", [None, (1.2, 1.7, 1.3, 1.0, 1.6)], ids=["default", "other"])
@pytest.mark.parametrize("c", [0.0, 0.5])
@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_mrt_hartmann_flow_converges_to_the_closed_form(bc, c, rates):
    r = derive.mrt_rates(0.8, 0.8, 3.0 / 16.0, 0.25) if rates is None else rates
    e16, e32 = hartmann_errors(16, bc, 5.0, c, r), hartmann_errors(32, bc, 5.0, c, r)
    for k in range(2):
        assert e32[k] < 2.5e-2 and e16[k] / e32[k] > 3.4, (e16, e32)


def test_mrt_conserves_mass():
    p = mrt_params(nx=11, ny=10, bc=LINK, b0=0.05, fx=2e-5, c_lo=0.2, c_hi=math.inf,
                   u_lo=-0.02, u_hi=0.03)
    s = random_state(p, seed=4)
    m0 = s[:9].sum()
    oracle.run(p, s, 40)
    assert abs(s[:9].sum() - m0) / m0 < 1e-14


def test_mrt_rates_are_validated():
    with pytest.raises(AssertionError):
        mrt_params(nx=4, ny=4, rates=(1.64, 1.54, 2.0, 1.0, 1.0)).c_struct()


# Moment rows (the orthogonal bases named above) in the velocity order of the
# state planes.
F_ROWS = {"e": [-4, -1, -1, -1, -1, 2, 2, 2, 2], "eps": [4, -2, -2, -2, -2, 1, 1, 1, 1],
          "qx": [0, -2, 0, 2, 0, 1, -1, -1, 1], "qy": [0, 0, -2, 0, 2, 1, 1, -1, -1],
          "pxx": [0, 1, -1, 1, -1, 0, 0, 0, 0], "pxy": [0, 0, 0, 0, 0, 1, -1, 1, -1]}
G_ROWS = {"eps": [-4, 1, 1, 1, 1], "d": [0, 1, -1, 1, -1]}


@pytest.mark.parametrize("plane0,rows", [(0, F_ROWS), (9, G_ROWS), (14, G_ROWS)],
                         ids=["f", "g_x", "g_y"])
def test_mrt_uniform_modes_decay_at_their_own_rates(plane0, rows):
    rates = (1.21, 1.37, 1.53, 0.77, 1.66)
    tau_f, tau_m = 0.8, 0.9
    rate_of = {0: {"e": rates[0], "eps": rates[1], "qx": rates[2], "qy": rates[2],
                   "pxx": 1 / tau_f, "pxy": 1 / tau_f},
               9: {"eps": rates[3], "d": rates[4]}, 14: {"eps": rates[3], "d": rates[4]}}[plane0]
    n, amp = 4, 1e-3
    for name, row in rows.items():
        p = mrt_params(tau_f=tau_f, tau_m=tau_m, rates=rates, nx=4, ny=16, bc=LINK)
        s = oracle.init_state(p)
        row = np.asarray(row, dtype=float)
        s[plane0:plane0 + len(row)] += (amp * row / (row @ row))[:, None, None]
        eq = oracle.init_state(p)
        oracle.run(p, s, n)
        for y in (7, 8):   # beyond the walls' reach after n steps
            d = s[plane0:plane0 + len(row), y, 1] - eq[plane0:plane0 + len(row), y, 1]
            for other, orow in rows.items():
                got = np.asarray(orow, dtype=float) @ d
                want = amp * (1 - rate_of[name]) ** n if other == name else 0.0
                assert abs(got - want) < 1e-14, (name, other, got, want)
            assert abs(d.sum()) < 1e-14


@pytest.mark.parametrize("walls", [dict(x_walls=True, cx_lo=0.5, cx_hi=math.inf),
                                   dict(q_lo=0.3, q_hi=0.8)], ids=["enclosure", "cut"])
def test_mrt_with_trt_rates_is_trt_in_enclosures_and_at_cut_walls(walls):
    tfm, tmp = derive.trt_times(0.7, 0.9, 3.0 / 16.0, 0.25)
    kw = dict(KW, bc=LINK, **walls)
    t = Params(tau_f=0.7, tau_m=0.9, collision=TRT, tau_fm=tfm, tau_mp=tmp, **kw)
    m = mrt_params(rates=(1 / 0.7, 1 / 0.7, 1 / tfm, 1 / tmp, 1 / tmp), **kw)
    s0 = random_state(t, seed=23)
    assert np.abs(oracle.run(m, s0.copy(), 20) - oracle.run(t, s0.copy(), 20)).max() < 1e-14
