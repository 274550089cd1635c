"""Pins of the 2D oracle's enclosure: stationary link-closed Shercliff walls
at x = -1/2 and nx - 1/2 besides the Hartmann walls.

The paper's closures are for walls normal to the imposed field; the walls
parallel to it and the corners are a reading (the enclosure-wall closure in
oracle/lks_oracle.c).  What pins it:

* x <-> y exchange: without an imposed field, with stationary walls of one
  conductance, a square enclosure is symmetric under exchanging x and y
  (and the components); this maps the x-wall closure onto the pinned
  Hartmann-wall link closure, corners included.
* x mirror: exchanging the two x-walls mirrors the run (u_x and B_x odd,
  the lid velocity and F_x reversed).
* Mass: conserved with a moving lid (the corner links take the Hartmann
  closure with its moving-wall term, whose terms cancel pairwise).
* Closure limits: perfectly conducting walls bounce back the tangential
  field population, insulating ones anti-bounce-back it; the normal one is
  always anti-bounced (B_x = 0).
* Free magnetic decay (exact): with the fluid at rest and no imposed field,
  each field component diffuses on its own, and its slowest mode in the box
  decays at eta (k_x^2 + k_y^2).  Along walls where the component is normal,
  k = pi / (2 a_w) (B_n = 0); along walls where it is tangential, k is the
  smallest root of tan(k a_w) = 1 / (c a k), the thin-wall condition
  c a db/dn + b = 0 (k = 0 for c = inf).  The decay rates converge to these
  eigenvalues at second order for both components and insulating, finitely
  and perfectly conducting enclosure and Hartmann walls.
* Consistency of the flow: the lid-driven cavity converges under
  refinement, at first order as the lid's velocity jump at the two upper
  corners allows.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, Params

EX9 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY9 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
EX5 = np.array([0, 1, 0, -1, 0])
EY5 = np.array([0, 0, 1, 0, -1])


def random_state(p, seed):
    from paper_2112_13930_amd.workloads import random_populations
    return random_populations(p.nx, p.ny, seed=seed, b0=p.b0)


def _perm(ex, ey, fx, fy):
    return [next(r for r in range(len(ex)) if ex[r] == fx(ex[q], ey[q]) and ey[r] == fy(ex[q], ey[q]))
            for q in range(len(ex))]


def swap_xy(state):
    p9 = _perm(EX9, EY9, lambda a, b: b, lambda a, b: a)
    p5 = _perm(EX5, EY5, lambda a, b: b, lambda a, b: a)
    t = np.transpose(state, (0, 2, 1))
    out = np.empty(t.shape)
    for q in range(9):
        out[p9[q]] = t[q]
    for q in range(5):
        out[9 + p5[q]] = t[14 + q]   # B_x <- B_y
        out[14 + p5[q]] = t[9 + q]
    return out


def mirror_x(state):
    p9 = _perm(EX9, EY9, lambda a, b: -a, lambda a, b: b)
    p5 = _perm(EX5, EY5, lambda a, b: -a, lambda a, b: b)
    t = state[:, :, ::-1]
    out = np.empty(t.shape)
    for q in range(9):
        out[p9[q]] = t[q]
    for q in range(5):
        out[9 + p5[q]] = -t[9 + q]
        out[14 + p5[q]] = t[14 + q]
    return out


@pytest.mark.parametrize("c", [0.0, 0.3, math.inf])
def test_square_enclosure_without_field_is_symmetric_under_x_y_exchange(c):
    kw = dict(nx=9, ny=9, bc=LINK, tau_f=0.75, tau_m=0.85, b0=0.0, c_lo=c, c_hi=c,
              x_walls=True, cx_lo=c, cx_hi=c)
    p = Params(fx=2e-5, fy=-1e-5, **kw)
    q = Params(fx=-1e-5, fy=2e-5, **kw)
    s = random_state(p, seed=31)
    a = oracle.run(p, s.copy(), 15)
    b = swap_xy(oracle.run(q, swap_xy(s), 15))
    assert np.abs(a - b).max() < 1e-15


def test_exchanging_the_x_walls_mirrors_the_run():
    kw = dict(nx=11, ny=8, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fy=1e-5, c_lo=0.2,
              c_hi=math.inf, x_walls=True)
    p = Params(fx=2e-5, u_hi=0.03, cx_lo=0.0, cx_hi=1.5, **kw)
    q = Params(fx=-2e-5, u_hi=-0.03, cx_lo=1.5, cx_hi=0.0, **kw)
    s = random_state(p, seed=8)
    a = oracle.run(p, s.copy(), 12)
    b = mirror_x(oracle.run(q, mirror_x(s), 12))
    assert np.abs(a - b).max() < 1e-15


def test_enclosure_with_moving_lid_conserves_mass():
    p = Params(nx=10, ny=9, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, c_lo=0.3, c_hi=2.0,
               u_lo=-0.02, u_hi=0.04, x_walls=True, cx_lo=0.0, cx_hi=math.inf)
    s = random_state(p, seed=12)
    m0 = s[:9].sum()
    oracle.run(p, s, 40)
    assert abs(s[:9].sum() - m0) / m0 < 1e-14


def test_xwall_closure_limits():
    rng = np.random.default_rng(3)
    own = rng.uniform(-0.1, 0.1, 19)
    f0, gx0, gy0 = rng.uniform(0, 0.1, 9), rng.uniform(-0.1, 0.1, 5), rng.uniform(-0.1, 0.1, 5)
    b0, w = 0.05, 1.0 / 6.0
    for wall, ex_in in ((0, 1), (1, -1)):
        qi = int(np.where((EX5 == ex_in) & (EY5 == 0))[0][0])
        qo = int(np.where((EX5 == -ex_in) & (EY5 == 0))[0][0])
        for c, sign in ((math.inf, 1.0), (0.0, -1.0)):
            p = Params(nx=4, ny=4, bc=LINK, tau_m=0.9, b0=b0, x_walls=True, cx_lo=c, cx_hi=c)
            f, gx, gy = oracle.xwall_closure(p, wall, own, f0, gx0, gy0)
            assert gx[qi] == -own[9 + qo]
            assert math.isclose(gy[qi] - w * b0, sign * (own[14 + qo] - w * b0), rel_tol=1e-15,
                                abs_tol=1e-17)
            for q in range(9):
                if EX9[q] == ex_in:
                    r = int(np.where((EX9 == -EX9[q]) & (EY9 == -EY9[q]))[0][0])
                    assert f[q] == own[r]
                else:
                    assert f[q] == f0[q]


def cavity(N, b0_ha, c=0.5, lid=1e-4, tau=0.8):
    """Steady lid-driven square cavity, N x N, upper wall moving at `lid`."""
    nu = eta = (tau - 0.5) / 3.0
    a = N / 2.0
    p = Params(nx=N, ny=N, bc=LINK, tau_f=tau, tau_m=tau, b0=b0_ha * math.sqrt(nu * eta) / a,
               c_lo=c, c_hi=c, u_hi=lid, x_walls=True, cx_lo=c, cx_hi=c)
    s = oracle.init_state(p)
    prev, n = None, 0
    while n < 400_000:
        oracle.run(p, s, 2000, nthreads=8)
        n += 2000
        o = oracle.observe(p, s)
        if prev is not None and max(np.linalg.norm(o[k] - prev[k]) / np.linalg.norm(o[k])
                                    for k in ("ux", "uy")) < 1e-10:
            return o
        prev = o
    raise AssertionError("no steady state")


def restrict(v):
    """2x2 averages: the coarse cell centres of a grid twice as fine."""
    return 0.25 * (v[0::2, 0::2] + v[1::2, 0::2] + v[0::2, 1::2] + v[1::2, 1::2])


def test_lid_driven_cavity_converges():
    sols = [cavity(N, 4.0) for N in (12, 24, 48)]
    for k in ("ux", "uy", "bx", "by"):
        v12, v24, v48 = (s[k] - (s[k].mean() if k == "by" else 0.0) for s in sols)
        d1 = np.linalg.norm(v12 - restrict(v24))
        d2 = np.linalg.norm(restrict(v24 - restrict(v48)))
        assert 1.6 < d1 / d2 < 2.8, (k, d1, d2)


def robin_k(c, a_w, a):
    """Smallest k > 0 with tan(k a_w) = 1/(c a k); pi/(2 a_w) for c = 0,
    0 for c = inf."""
    from scipy.optimize import brentq
    if c == 0.0:
        return math.pi / (2 * a_w)
    if math.isinf(c):
        return 0.0
    hi = math.pi / (2 * a_w) * (1 - 1e-12)
    return brentq(lambda k: math.tan(k * a_w) - 1.0 / (c * a * k), 1e-12, hi)


def decay_rate_error(N, comp, cx, cy, tau=0.8, amp=1e-6):
    p = Params(nx=N, ny=N, bc=LINK, tau_f=tau, tau_m=tau, b0=0.0, c_lo=cy, c_hi=cy,
               x_walls=True, cx_lo=cx, cx_hi=cx)
    s = oracle.init_state(p)
    a = N / 2.0
    xy = np.arange(N) + 0.5 - a
    prof = amp * np.outer(np.cos(math.pi * xy / (2 * a)), np.cos(math.pi * xy / (2 * a)))
    base = 9 if comp == "x" else 14
    for q, w in enumerate((1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6)):
        s[base + q] += w * prof
    eta = (tau - 0.5) / 3.0
    lam_est = 2 * eta * (math.pi / (2 * a)) ** 2
    t1, dt = int(5 / lam_est), int(2 / lam_est)   # the slowest mode dominates
    oracle.run(p, s, t1)
    n1 = np.linalg.norm(oracle.observe(p, s)["b" + comp])
    oracle.run(p, s, dt)
    n2 = np.linalg.norm(oracle.observe(p, s)["b" + comp])
    lam = -math.log(n2 / n1) / dt
    if comp == "y":   # tangential at the enclosure walls, normal at the Hartmann walls
        k2 = robin_k(cx, a, a) ** 2 + (math.pi / (2 * a)) ** 2
    else:             # normal at the enclosure walls, tangential at the Hartmann walls
        k2 = (math.pi / (2 * a)) ** 2 + robin_k(cy, a, a) ** 2
    return abs(lam - eta * k2) / (eta * k2)


@pytest.mark.parametrize("comp", ["x", "y"])
@pytest.mark.parametrize("cx,cy", [(0.5, 0.2), (0.0, 1.0), (math.inf, 0.3), (2.0, math.inf)])
def test_free_magnetic_decay_converges_to_the_box_eigenvalue(comp, cx, cy):
    e8, e16 = decay_rate_error(8, comp, cx, cy), decay_rate_error(16, comp, cx, cy)
    assert e16 < 3e-3 and 3.7 < e8 / e16 < 4.3, (e8, e16)


def test_each_enclosure_wall_takes_its_own_conductance():
    """c_x,lo closes the x = 0 side and c_x,hi the x = nx-1 side: with an
    insulating lower and a perfectly conducting upper wall, the tangential
    population entering at x = 0 is anti-bounced (b_y = 0) and the one
    entering at x = nx-1 bounced back."""
    p = Params(nx=6, ny=5, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, x_walls=True, cx_lo=0.0,
               cx_hi=math.inf)
    s = random_state(p, seed=2)
    wb0 = p.b0 / 6.0
    for y in (1, 2, 3):
        lo = oracle.gather(p, s, 0, y)
        hi = oracle.gather(p, s, p.nx - 1, y)
        # D2Q5: 1 = +x, 3 = -x; g_y planes start at 14
        assert math.isclose(lo[14 + 1] - wb0, -(s[14 + 3, y, 0] - wb0), rel_tol=1e-14)
        assert hi[14 + 3] == s[14 + 1, y, p.nx - 1]
