"""Whole-step pins of the oracle: conservation laws, symmetries, transport
coefficients and x-streaming, none of which restate the code under test.

  * Mass: collisions conserve it (sum f^eq = rho, sum S = 0, Sec. V) and
    half-way bounce-back with Ladd's moving-wall terms (+-U/6 in pairs,
    App. B.1) conserves it, so the link-based total mass is constant to
    round-off, for any (even x- and y-random) state.
  * Magnetic flux: with perfectly conducting stationary link walls (pure
    bounce-back of g_x, Sec. VI limit (b)) sum B_x is conserved.
  * x-invariance, y-mirror symmetry of Hartmann flow (Sec. VIII: B_x odd,
    u even about the centreline), and the mirror map between a moving upper
    wall and a moving lower wall (the lower-wall forms are mirror images of
    the printed upper-wall ones).
  * Viscosity nu = cs2 (tau - 1/2) (Sec. V) and resistivity
    eta = cs2m (tau_m - 1/2) (Sec. IV) from the decay of an x-dependent shear
    wave and of a B_y wave, and the direction of x-streaming from their
    advection by a uniform flow.
  * Thread-count independence of the oracle (bitwise).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params, derive

rng = np.random.default_rng(99)


def random_state(p, eps=0.02):
    """Random x- and y-dependent populations near a rest state."""
    s = oracle.init_state(p)
    s *= 1.0 + eps * rng.uniform(-1, 1, s.shape)
    s[9:] += eps * 0.05 * rng.uniform(-1, 1, s[9:].shape)
    return s


@pytest.mark.parametrize("u_lo,u_hi", [(0.0, 0.0), (0.03, -0.05)])
def test_link_mass_conservation(orc, u_lo, u_hi):
    p = Params(nx=7, ny=11, bc=LINK, tau_f=0.65, tau_m=0.9, b0=0.04, fx=2e-5, fy=-1e-5,
               c_lo=0.2, c_hi=3.0, u_lo=u_lo, u_hi=u_hi)
    s = random_state(p)
    m0 = s[:9].sum()
    orc.run(p, s, 60)
    assert abs(s[:9].sum() - m0) / m0 < 2e-14


def test_conducting_link_walls_conserve_bx_flux(orc):
    p = Params(nx=5, ny=9, bc=LINK, tau_f=0.7, tau_m=0.8, b0=0.05, fx=1e-4,
               c_lo=math.inf, c_hi=math.inf)
    s = random_state(p)
    f0 = s[9:14].sum()
    orc.run(p, s, 60)
    assert abs(s[9:14].sum() - f0) < 1e-15 * s.size


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_x_invariance_and_uniform_by(orc, bc):
    p = derive.hartmann_params(4, 12, bc, 0.8, 0.7, 5.0, 0.3, 0.05)
    s = oracle.init_state(p)
    orc.run(p, s, 200)
    for x in range(1, 4):
        assert np.array_equal(s[:, :, x], s[:, :, 0])
    o = orc.observe(p, s)
    assert np.abs(o["by"] - p.b0).max() < 1e-14


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_hartmann_mirror_symmetry(orc, bc):
    p = derive.hartmann_params(1, 20, bc, 0.8, 0.7, 8.0, 0.4, 0.05)
    s = oracle.init_state(p)
    orc.run(p, s, 3000)
    o = orc.observe(p, s)
    u, b = o["ux"][:, 0], o["bx"][:, 0]
    assert np.abs(u - u[::-1]).max() < 1e-13 * np.abs(u).max()
    assert np.abs(b + b[::-1]).max() < 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("c1,c2", [(0.0, 0.5), (0.2, math.inf), (1.0, 1.0)])
def test_moving_lower_wall_is_mirror_of_moving_upper_wall(orc, bc, c1, c2):
    """y -> -y with B_x -> -B_x maps (lower c1 at rest, upper c2 moving) onto
    (lower c2 moving, upper c1 at rest)."""
    pa = derive.couette_params(3, 14, bc, 0.75, 0.9, 6.0, c1, c2, 0.05)
    pb = Params(**{**pa.__dict__, "c_lo": c2, "c_hi": c1, "u_lo": 0.05, "u_hi": 0.0})
    sa, sb = oracle.init_state(pa), oracle.init_state(pb)
    orc.run(pa, sa, 1500)
    orc.run(pb, sb, 1500)
    oa, ob = orc.observe(pa, sa), orc.observe(pb, sb)
    assert np.abs(oa["ux"] - ob["ux"][::-1]).max() < 1e-14
    assert np.abs(oa["bx"] + ob["bx"][::-1]).max() < 1e-14
    assert np.abs(oa["uy"] + ob["uy"][::-1]).max() < 1e-14


def _wave_state(p, U0, eps, b):
    s = np.empty((19, p.ny, p.nx))
    k = 2 * np.pi / p.nx
    for x in range(p.nx):
        uy, by = eps * np.sin(k * x), b * np.sin(k * x)
        fe = oracle.feq(1.0, U0, uy)
        gx, gy = oracle.geq(0.0, by, U0, uy)
        s[:9, :, x] = fe[:, None]
        s[9:14, :, x] = gx[:, None]
        s[14:, :, x] = gy[:, None]
    return s


def _mode(o, key, p):
    k = 2 * np.pi / p.nx
    x = np.arange(p.nx)
    row = o[key][p.ny // 2 - 2:p.ny // 2 + 2].mean(axis=0)
    c, s = 2 * (row * np.cos(k * x)).mean(), 2 * (row * np.sin(k * x)).mean()
    return math.hypot(c, s), math.atan2(-c, s)


@pytest.mark.parametrize("U0", [0.0, 0.05, -0.05])
def test_wave_decay_and_advection(orc, U0):
    """u_y = eps sin(kx) decays at nu k^2 and B_y = b sin(kx) at eta k^2, and
    both are carried at U0 by a uniform flow (walls moving at U0, B0 = 0)."""
    tau_f, tau_m = 0.8, 0.9
    # The no-slip walls launch sound at t = 0; the window [t1, t2] ends before
    # it can cross half the channel (c_s t2 < ny/2) to the rows measured.
    p = Params(nx=32, ny=256, bc=LINK, tau_f=tau_f, tau_m=tau_m, b0=0.0, u_lo=U0, u_hi=U0)
    s = _wave_state(p, U0, 1e-4, 1e-4)
    k = 2 * np.pi / p.nx
    t1, t2 = 10, 110
    assert t2 / math.sqrt(3.0) < p.ny / 2 - 4
    orc.run(p, s, t1)
    o1 = orc.observe(p, s)
    orc.run(p, s, t2 - t1)
    o2 = orc.observe(p, s)
    for key, coef in (("uy", derive.nu_of(tau_f)), ("by", derive.eta_of(tau_m))):
        (a1, ph1), (a2, ph2) = _mode(o1, key, p), _mode(o2, key, p)
        rate = math.log(a1 / a2) / (t2 - t1) / k ** 2
        assert abs(rate / coef - 1) < 0.02, (key, rate, coef)
        dphase = ph2 - ph1
        assert abs(dphase - k * U0 * (t2 - t1)) < 0.02 * max(abs(k * U0 * (t2 - t1)), 0.05), (key, dphase)


def test_thread_count_independent(orc):
    p = Params(nx=9, ny=13, bc=MOMENT, tau_f=0.7, tau_m=0.8, b0=0.03, fx=1e-5,
               c_lo=0.1, c_hi=math.inf, u_hi=0.02)
    s = random_state(p)
    a = orc.step(p, s, nthreads=1)
    b = orc.step(p, s, nthreads=4)
    assert np.array_equal(a, b)


def test_limits_of_c_in_whole_run(orc):
    """c = 1e-12 matches c = 0 and c = 1e12 matches c = inf over many steps
    (Sec. VI limits (a), (b); Sec. VII limits)."""
    for bc in (LINK, MOMENT):
        for small, lim in ((1e-12, 0.0), (1e12, math.inf)):
            pa = derive.couette_params(2, 10, bc, 0.8, 0.8, 4.0, small, small, 0.05)
            pb = derive.couette_params(2, 10, bc, 0.8, 0.8, 4.0, lim, lim, 0.05)
            sa, sb = oracle.init_state(pa), oracle.init_state(pb)
            orc.run(pa, sa, 500)
            orc.run(pb, sb, 500)
            assert np.abs(sa - sb).max() < 1e-9


def test_steady_driver_reports_blow_up(orc):
    """An unstable parameter set (strong forcing at a tiny viscosity) must be
    reported, not mistaken for a steady state."""
    from oracle import steady
    p = Params(nx=1, ny=16, bc=LINK, tau_f=0.5005, tau_m=0.5005, b0=0.8, fx=0.02)
    with pytest.raises(FloatingPointError):
        steady.run_to_steady(p, tol=1e-12, check_every=100, max_steps=200_000)
