"""Node-level pins of the oracle: each building block against the moment
relations the paper defines it by.

  f^eq (Sec. V):  sum = rho, sum e = rho u, sum e e = rho (cs2 I + u u)
  g^eq (Sec. IV): sum = B, sum_alpha e_j g^eq_i = u_j B_i - B_j u_i
  S    (Sec. V):  sum S = 0, sum e S = F
  u/J solve:      rho u = sum f e + F/2 with F = F_ext + J x B (Secs. II, V) and
                  J_z from the non-equilibrium Lambda (Sec. IV), simultaneously
  link closure:   Eq. (constraintrelationmovingwall) and the Dirichlet relation
                  of Eq. (magneticfieldanditsgradientrelation1); limits of
                  Sec. VI / App. B.1; Ladd's moving bounce-back (App. B.1)
  moment closure: the constraints it is solved from (App. A, App. B.2,
                  Eqs. momentconstraintgx/gy) and the limits printed after them
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params

EX9 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY9 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
EX5 = np.array([0, 1, 0, -1, 0])
EY5 = np.array([0, 0, 1, 0, -1])
rng = np.random.default_rng(1234)


@pytest.mark.parametrize("trial", range(5))
def test_feq_moments(orc, trial):
    rho, ux, uy = 0.8 + 0.4 * rng.random(), 0.2 * rng.standard_normal(), 0.2 * rng.standard_normal()
    f = orc.feq(rho, ux, uy)
    assert abs(f.sum() - rho) < 1e-15
    assert abs((f * EX9).sum() - rho * ux) < 1e-15
    assert abs((f * EY9).sum() - rho * uy) < 1e-15
    assert abs((f * EX9 * EX9).sum() - rho * (1 / 3 + ux * ux)) < 1e-15
    assert abs((f * EY9 * EY9).sum() - rho * (1 / 3 + uy * uy)) < 1e-15
    assert abs((f * EX9 * EY9).sum() - rho * ux * uy) < 1e-15


@pytest.mark.parametrize("trial", range(5))
def test_geq_moments(orc, trial):
    bx, by, ux, uy = rng.standard_normal(4) * 0.1
    gx, gy = orc.geq(bx, by, ux, uy)
    u, b = np.array([ux, uy]), np.array([bx, by])
    g = np.stack([gx, gy])  # [i][alpha]
    e = np.stack([EX5, EY5])  # [j][alpha]
    assert np.allclose(g.sum(axis=1), b, atol=1e-16, rtol=0)
    lam = e @ g.T  # Lambda_ji = sum_a e_aj g_ai
    lam0 = np.outer(u, b) - np.outer(b, u)  # u_j B_i - B_j u_i
    assert np.abs(lam - lam0).max() < 1e-16


@pytest.mark.parametrize("trial", range(5))
def test_source_moments(orc, trial):
    rho, ux, uy, Fx, Fy = 1 + 0.1 * rng.random(), *(0.1 * rng.standard_normal(4))
    fe = orc.feq(rho, ux, uy)
    S = orc.source(rho, ux, uy, Fx, Fy, fe)
    assert abs(S.sum()) < 1e-16
    assert abs((S * EX9).sum() - Fx) < 1e-15
    assert abs((S * EY9).sum() - Fy) < 1e-15


@pytest.mark.parametrize("trial", range(8))
def test_local_solve_satisfies_definitions(orc, trial):
    rho = 0.9 + 0.2 * rng.random()
    mx, my, bx, by, lxy, lyx, fex, fey = rng.standard_normal(8) * np.array(
        [0.05, 0.05, 0.3, 0.5, 0.05, 0.05, 1e-3, 1e-3])
    tau_m = 0.55 + rng.random()
    ux, uy, jz = orc.local_solve(rho, mx, my, bx, by, lxy, lyx, tau_m, fex, fey)
    k = 3.0 / tau_m
    Fx, Fy = fex - jz * by, fey + jz * bx
    assert abs(rho * ux - (mx + Fx / 2)) < 1e-15
    assert abs(rho * uy - (my + Fy / 2)) < 1e-15
    l0xy, l0yx = ux * by - bx * uy, uy * bx - by * ux
    jz_def = -k * ((lxy - l0xy) - (lyx - l0yx))
    assert abs(jz - jz_def) < 1e-14 * max(1.0, abs(jz))


def _p(bc, c_lo, c_hi, u_lo=0.0, u_hi=0.0, b0=0.05, tau_m=0.8, a=16.0):
    return Params(nx=4, ny=8, bc=bc, tau_f=0.7, tau_m=tau_m, b0=b0, c_lo=c_lo,
                  c_hi=c_hi, u_lo=u_lo, u_hi=u_hi, a=a)


@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("c", [0.0, 0.03, 0.5, 7.0, math.inf])
@pytest.mark.parametrize("U", [0.0, 0.04])
def test_link_closure(orc, wall, c, U):
    p = _p(LINK, c, c, u_lo=U if wall == 0 else 0.0, u_hi=U if wall == 1 else 0.0)
    own = 0.1 + 0.05 * rng.random(19)
    f, gx, gy = (np.full(n, np.nan) for n in (9, 5, 5))
    f, gx, gy = orc.link_closure(p, wall, own, f, gx, gy)
    ein = 1 if wall == 0 else -1
    q_in, q_out = (2, 4) if wall == 0 else (4, 2)
    W = 1.0 / 6.0
    # g_y: (g_in + g~_out)/2 = W B0
    assert abs(0.5 * (gy[q_in] + own[14 + q_out]) - W * p.b0) < 1e-16
    gbar = own[9 + q_out]
    if math.isinf(c):
        assert gx[q_in] == gbar - 2 * W * (ein * 3.0) * p.b0 * U
    elif c == 0.0:
        assert gx[q_in] == -gbar
    else:
        theta = c * p.a / (p.tau_m - 0.5)
        lhs = (1 + theta) * gx[q_in] + (1 - theta) * gbar + 2 * theta * W * ein * 3.0 * p.b0 * U
        assert abs(lhs) < 1e-15 * max(1.0, theta)
    # f: Ladd's moving-wall bounce-back, f_a = f~_abar + 2 w_a e_ax U / cs2
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    for q in range(9):
        if EY9[q] == ein:
            assert abs(f[q] - (own[opp[q]] + 2 * w[q] * EX9[q] * U * 3.0)) < 1e-16
        else:
            assert np.isnan(f[q])


@pytest.mark.parametrize("wall", [0, 1])
@pytest.mark.parametrize("c", [0.0, 0.03, 0.5, 7.0, math.inf])
@pytest.mark.parametrize("U", [0.0, 0.04])
def test_moment_closure_constraints(orc, wall, c, U):
    p = _p(MOMENT, c, c, u_lo=U if wall == 0 else 0.0, u_hi=U if wall == 1 else 0.0)
    f = 0.1 + 0.02 * rng.random(9)
    gx = 0.01 * rng.standard_normal(5)
    gy = p.b0 / 5 + 0.01 * rng.standard_normal(5)
    f2, gx2, gy2 = orc.moment_closure(p, wall, f, gx, gy)
    unknown = [2, 5, 6] if wall == 0 else [4, 7, 8]
    known = [q for q in range(9) if q not in unknown]
    assert np.array_equal(f2[known], f[known])
    rho = f2.sum()
    assert abs((f2 * EX9).sum() - rho * U) < 1e-15
    assert abs((f2 * EY9).sum()) < 1e-15
    assert abs((f2 * EX9 * EX9).sum() - rho * (1 / 3 + U * U)) < 1e-15
    # g_y: sum = B0
    assert abs(gy2.sum() - p.b0) < 1e-16
    q_in = 2 if wall == 0 else 4
    assert np.array_equal(np.delete(gx2, q_in), np.delete(gx, q_in))
    lam_yx = gx2[2] - gx2[4]
    A = 3.0 / p.tau_m
    if c == 0.0:
        assert abs(gx2.sum()) < 1e-16  # B_x = 0 at an insulating wall
    elif math.isinf(c):
        assert abs(lam_yx + p.b0 * U) < 1e-16  # dB_x/dy = 0
    else:
        C = 1.0 / (c * p.a)
        sgn = 1.0 if wall == 0 else -1.0
        assert abs(sgn * A * (lam_yx + p.b0 * U) + C * gx2.sum()) < 1e-14


def test_closure_limits_continuous(orc):
    """The general formulas tend to the printed limiting closures (Sec. VI,
    Sec. VII, App. B): c -> 0 and c -> inf."""
    own = 0.1 + 0.05 * rng.random(19)
    f0, gx0, gy0 = 0.1 + 0.02 * rng.random(9), 0.01 * rng.standard_normal(5), 0.01 + 0.01 * rng.random(5)
    for bc in (LINK, MOMENT):
        for wall in (0, 1):
            for small, lim in ((1e-13, 0.0), (1e13, math.inf)):
                pa = _p(bc, small, small, 0.03, 0.03)
                pb = _p(bc, lim, lim, 0.03, 0.03)
                if bc == LINK:
                    ra = orc.link_closure(pa, wall, own, f0, gx0, gy0)
                    rb = orc.link_closure(pb, wall, own, f0, gx0, gy0)
                else:
                    ra = orc.moment_closure(pa, wall, f0, gx0, gy0)
                    rb = orc.moment_closure(pb, wall, f0, gx0, gy0)
                for x, y in zip(ra, rb):
                    assert np.allclose(x, y, rtol=0, atol=1e-11)
