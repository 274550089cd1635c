"""Pins of the oracle's two-relaxation-time (TRT) collision.

The paper names multiple-relaxation-time collisions as a drop-in
replacement for its BGK operators (Secs. V and IX); TRT is the smallest such
model.  Its reading: the even part of f relaxes at tau_f (viscosity) and its
odd part at tau_fm; the odd part of g relaxes at tau_m (magnetic
diffusivity) and its even part at tau_mp.

* Moment algebra (complete): for every moment of a basis of the D2Q9 (D2Q5)
  population space, the post-collision moment equals the pre-collision one
  relaxed towards the equilibrium's at the rate of its parity, plus the
  source's moment with the weight 1 - 1/(2 tau) of that parity.  The bases
  span the whole space, so this fixes the operator.
* Equal rates: TRT with tau_fm = tau_f and tau_mp = tau_m is the BGK step.
* Poiseuille flow with half-way bounce-back is reproduced exactly (to
  round-off) at the magic parameter Lambda_f = (tau_f - 1/2)(tau_fm - 1/2)
  = 3/16 for every tau_f (Ginzburg, Verhaeghe and d'Humieres, Commun. Comput.
  Phys. 3 (2008) 427); BGK, whose Lambda is (tau_f - 1/2)^2, is exact only at
  tau_f = 1/2 + sqrt(3)/4.
* Conservation: mass with link-based walls, and sum B_x with perfectly
  conducting stationary link walls, under TRT.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import BGK, LINK, MOMENT, TRT, Params, derive

EX9 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY9 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
EX5 = np.array([0, 1, 0, -1, 0], dtype=float)
EY5 = np.array([0, 0, 1, 0, -1], dtype=float)

# Moment bases, split by parity under e -> -e.
EVEN9 = np.array([np.ones(9), EX9**2, EY9**2, EX9 * EY9, EX9**2 * EY9**2])
ODD9 = np.array([EX9, EY9, EX9 * EY9**2, EX9**2 * EY9])
EVEN5 = np.array([np.ones(5), EX5**2, EY5**2])
ODD5 = np.array([EX5, EY5])


def test_moment_bases_span_the_population_spaces():
    assert np.linalg.matrix_rank(np.vstack([EVEN9, ODD9])) == 9
    assert np.linalg.matrix_rank(np.vstack([EVEN5, ODD5])) == 5


@pytest.mark.parametrize("seed", range(6))
def test_trt_collision_moment_algebra(seed):
    rng = np.random.default_rng(seed)
    tau_f, tau_fm, tau_m, tau_mp = rng.uniform(0.55, 2.0, 4)
    p = Params(nx=1, ny=3, tau_f=tau_f, tau_m=tau_m, collision=TRT, tau_fm=tau_fm,
               tau_mp=tau_mp)
    f = rng.uniform(0.0, 0.5, 9)
    gx, gy = rng.uniform(-0.05, 0.05, 5), rng.uniform(-0.05, 0.05, 5)
    rho = 1 + 0.1 * rng.uniform(-1, 1)
    ux, uy, bx, by = 0.05 * rng.uniform(-1, 1, 4)
    Fx, Fy = 1e-3 * rng.uniform(-1, 1, 2)
    out = oracle.collide(p, f, gx, gy, rho, ux, uy, bx, by, Fx, Fy)
    feq = oracle.feq(rho, ux, uy)
    S = oracle.source(rho, ux, uy, Fx, Fy, feq)
    gex, gey = oracle.geq(bx, by, ux, uy)

    def relaxed(M, h, heq, tau, src=None):
        v = M @ h - (M @ h - M @ heq) / tau
        return v if src is None else v + (1 - 1 / (2 * tau)) * (M @ src)

    assert np.allclose(EVEN9 @ out[:9], relaxed(EVEN9, f, feq, tau_f, S), rtol=0, atol=1e-15)
    assert np.allclose(ODD9 @ out[:9], relaxed(ODD9, f, feq, tau_fm, S), rtol=0, atol=1e-15)
    for h, he, o in ((gx, gex, out[9:14]), (gy, gey, out[14:19])):
        assert np.allclose(EVEN5 @ o, relaxed(EVEN5, h, he, tau_mp), rtol=0, atol=1e-16)
        assert np.allclose(ODD5 @ o, relaxed(ODD5, h, he, tau_m), rtol=0, atol=1e-16)
    # momentum gains exactly F at any pair of rates (rho u = m + F/2)
    m = np.array([EX9 @ f, EY9 @ f])
    u_consistent = (m + 0.5 * np.array([Fx, Fy])) / (f.sum())
    out2 = oracle.collide(p, f, gx, gy, f.sum(), *u_consistent, bx, by, Fx, Fy)
    assert np.allclose([EX9 @ out2[:9], EY9 @ out2[:9]], m + [Fx, Fy], rtol=0, atol=1e-15)


def random_state(p, seed):
    from paper_2112_13930_amd.workloads import random_populations
    return random_populations(p.nx, p.ny, seed=seed, b0=p.b0)


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_trt_with_equal_rates_is_bgk(bc):
    kw = dict(nx=9, ny=12, bc=bc, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=0.3,
              c_hi=math.inf, u_hi=0.03)
    a = Params(**kw)
    b = Params(**kw, collision=TRT, tau_fm=0.7, tau_mp=0.9)
    s0 = random_state(a, seed=21)
    sa = oracle.run(a, s0.copy(), 30)
    sb = oracle.run(b, s0.copy(), 30)
    assert np.abs(sa - sb).max() < 1e-15
    c = Params(**kw, collision=TRT, tau_fm=0.8, tau_mp=0.9)
    assert np.abs(oracle.run(c, s0.copy(), 30) - sa).max() > 1e-8  # the odd rate matters


def poiseuille_error(tau_f, collision, ny=16, fx=1e-5, steps=40000):
    tau_fm, tau_mp = derive.trt_times(tau_f, 0.9, 3.0 / 16.0, 0.25)
    p = Params(nx=1, ny=ny, bc=LINK, tau_f=tau_f, tau_m=0.9, fx=fx, collision=collision,
               tau_fm=tau_fm, tau_mp=tau_mp)
    s = oracle.init_state(p)
    oracle.run(p, s, steps)
    ux = oracle.observe(p, s)["ux"][:, 0]
    a = ny / 2.0
    y = np.arange(ny) + 0.5 - a  # walls half-way, at y = -a and +a
    exact = fx / (2 * derive.nu_of(tau_f)) * (a * a - y * y)
    return np.abs(ux - exact).max() / exact.max()


@pytest.mark.parametrize("tau_f", [0.6, 0.8, 1.5])
def test_trt_magic_parameter_makes_bounce_back_poiseuille_exact(tau_f):
    assert poiseuille_error(tau_f, TRT) < 1e-10


def test_bgk_poiseuille_exact_only_at_its_magic_time():
    assert poiseuille_error(0.5 + math.sqrt(3.0) / 4.0, BGK) < 1e-10
    assert poiseuille_error(0.8, BGK) > 1e-3


def test_trt_conservation():
    tau_fm, tau_mp = derive.trt_times(0.7, 0.9, 3.0 / 16.0, 0.25)
    p = Params(nx=11, ny=10, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=math.inf,
               c_hi=math.inf, u_lo=-0.02, u_hi=0.03, collision=TRT, tau_fm=tau_fm,
               tau_mp=tau_mp)
    s = random_state(p, seed=4)
    m0 = s[:9].sum()
    oracle.run(p, s, 40)
    assert abs(s[:9].sum() - m0) / m0 < 1e-14
    q = Params(**{**p.__dict__, "u_lo": 0.0, "u_hi": 0.0})
    s = random_state(q, seed=5)
    b0x = oracle.observe(q, s)["bx"].sum()
    oracle.run(q, s, 40)
    bx = oracle.observe(q, s)["bx"]
    assert abs(bx.sum() - b0x) < 1e-13 * max(1.0, np.abs(bx).sum())
