"""Pins of the three-dimensional channel oracle (oracle/lks_oracle3.c).

* Local relations: moments of f^eq, g^eq and the source; the coupled u/J
  solve satisfies its six defining relations.
* Reduction to two dimensions: a z-invariant 3D state evolves exactly as the
  independent two-dimensional oracle does on its e_z-summed populations, for
  both wall treatments, finite, zero and infinite conductance, moving walls
  and forcing.  This pins streaming in x and y, both closures, the moments
  and the solve.
* x <-> z exchange: a random x-, y- and z-dependent state driven along x
  equals the exchanged state driven along z, exchanged back.  This maps the
  x handling, pinned above, onto z (streaming, J_x and J_y, the tangential
  g_z closure).
* Conservation: the link-based walls conserve mass for random 3D states.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params
from oracle import d3

RNG = np.random.default_rng(2024)


def test_feq_geq_source_moments():
    rho, u = 1.07, np.array([0.031, -0.022, 0.017])
    f = d3.feq(rho, u)
    E = d3.EF
    assert math.isclose(f.sum(), rho, rel_tol=1e-15)
    assert np.allclose(E.T @ f, rho * u, atol=1e-16)
    Pi = np.einsum("q,qi,qj->ij", f, E, E)
    assert np.allclose(Pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-16)
    b = np.array([0.012, 0.05, -0.008])
    g = d3.geq(b, u)
    assert np.allclose(g.sum(axis=0), b, atol=1e-17)
    lam = np.einsum("qj,qi->ji", d3.EG, g)
    assert np.allclose(lam, np.outer(u, b) - np.outer(b, u), atol=1e-17)
    assert g[0].tolist() == [0.0, 0.0, 0.0]  # zero rest weight
    F = np.array([1e-4, -2e-5, 3e-5])
    S = d3.source(rho, u, F, f)
    assert abs(S.sum()) < 1e-18
    assert np.allclose(E.T @ S, F, atol=1e-18)


def test_local_solve_satisfies_definitions():
    for _ in range(20):
        rho = 1 + 0.05 * RNG.uniform(-1, 1)
        m = 0.05 * RNG.uniform(-1, 1, 3)
        b = RNG.uniform(-0.1, 0.1, 3)
        lam = 0.01 * RNG.uniform(-1, 1, (3, 3))
        fext = 1e-4 * RNG.uniform(-1, 1, 3)
        tau_m = 0.6 + 0.5 * RNG.uniform()
        u, J = d3.local_solve(rho, m, b, lam, tau_m, fext)
        k = 3.0 / tau_m
        F = fext + np.cross(J, b)
        assert np.allclose(rho * u, m + F / 2, atol=1e-16)
        L0 = np.outer(u, b) - np.outer(b, u)  # L0[j][i] = u_j B_i - B_j u_i
        N = lam - L0
        curl = np.array([N[1, 2] - N[2, 1], N[2, 0] - N[0, 2], N[0, 1] - N[1, 0]])
        assert np.allclose(J, -k * curl, atol=1e-15)


def random_state_2d(p, seed):
    from paper_2112_13930_amd.workloads import random_populations
    return random_populations(p.nx, p.ny, seed=seed, b0=p.b0)


CASES_2D = [
    # bc, c_lo, c_hi, u_lo, u_hi, fx, fy
    (LINK, 0.3, 2.0, 0.0, 0.04, 1e-5, 0.0),
    (LINK, 0.0, math.inf, -0.03, 0.02, 2e-5, -1e-5),
    (MOMENT, 0.3, 2.0, 0.0, 0.04, 1e-5, 0.0),
    (MOMENT, math.inf, 0.0, 0.02, -0.01, 0.0, 1e-5),
]


@pytest.mark.parametrize("case", CASES_2D)
def test_z_invariant_run_reproduces_2d_oracle(case):
    bc, cl, cu, ul, uu, fx, fy = case
    p2 = Params(nx=7, ny=10, bc=bc, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=fy, c_lo=cl,
                c_hi=cu, u_lo=ul, u_hi=uu)
    s2 = random_state_2d(p2, seed=11)
    for nz in (1, 3):
        p3 = d3.Params3.from_2d(p2, nz)
        s3 = d3.lift_from_2d(s2, nz)
        assert np.allclose(d3.project_to_2d(s3), s2, rtol=0, atol=1e-16)
        a2 = s2.copy()
        oracle.run(p2, a2, 15)
        d3.run(p3, s3, 15)
        # every layer identical, and the e_z sums equal the 2D state
        assert np.array_equal(s3, np.repeat(s3[:, :1], nz, axis=1))
        assert np.abs(d3.project_to_2d(s3) - a2).max() < 1e-14
        o3 = d3.observe(p3, s3)
        o2 = oracle.observe(p2, a2)
        for k in ("rho", "ux", "uy", "bx", "by", "jz"):
            assert np.abs(o3[k][0] - o2[k]).max() < 1e-14, k
        for k in ("uz", "bz", "jx", "jy"):
            assert np.abs(o3[k]).max() < 1e-16, k


def random_state_3d(p, seed):
    """Near-rest equilibrium with random x-, y- and z-dependent perturbations
    (g_z nonzero; the zero-weight rest population of g stays zero)."""
    rng = np.random.default_rng(seed)
    s = d3.init_state(p)
    shape = (p.nz, p.ny, p.nx)
    s[:19] *= 1 + 0.02 * rng.uniform(-1, 1, (19,) + shape)
    for comp in range(3):
        base = 19 + 7 * comp
        s[base + 1:base + 7] += 0.002 * rng.uniform(-1, 1, (6,) + shape)
    return s


def swap_xz(state):
    """The state with the x and z axes exchanged: coordinates, velocity
    components and field components."""
    permf = [next(r for r in range(19) if (d3.EF[r] == d3.EF[q][[2, 1, 0]]).all()) for q in range(19)]
    permg = [next(r for r in range(7) if (d3.EG[r] == d3.EG[q][[2, 1, 0]]).all()) for q in range(7)]
    out = np.empty_like(state)
    t = np.transpose(state, (0, 3, 2, 1))  # [plane][x][y][z] -> read as [plane][z'][y][x']
    for q in range(19):
        out[permf[q]] = t[q]
    for comp, comp2 in ((0, 2), (1, 1), (2, 0)):
        for q in range(7):
            out[19 + 7 * comp2 + permg[q]] = t[19 + 7 * comp + q]
    return out


@pytest.mark.parametrize("bc,c", [(LINK, 0.4), (MOMENT, 0.4), (LINK, math.inf), (MOMENT, 0.0)])
def test_x_z_exchange(bc, c):
    n = 6
    p = d3.Params3(nx=n, ny=8, nz=n, bc=bc, tau_f=0.75, tau_m=0.85, b0=0.04, fx=3e-5,
                   c_lo=c, c_hi=c)
    q = d3.Params3(nx=n, ny=8, nz=n, bc=bc, tau_f=0.75, tau_m=0.85, b0=0.04, fz=3e-5,
                   c_lo=c, c_hi=c)
    s = random_state_3d(p, seed=5)
    a = d3.run(p, s.copy(), 12)
    b = swap_xz(d3.run(q, swap_xz(s), 12))
    assert np.abs(a - b).max() < 1e-15


def test_link_walls_conserve_mass_3d():
    p = d3.Params3(nx=5, ny=9, nz=4, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5,
                   fz=-1e-5, c_lo=0.3, c_hi=math.inf, u_lo=-0.02, u_hi=0.03)
    s = random_state_3d(p, seed=9)
    m0 = s[:19].sum()
    d3.run(p, s, 25)
    assert abs(s[:19].sum() - m0) / m0 < 1e-14


def test_thread_count_does_not_change_result():
    p = d3.Params3(nx=5, ny=7, nz=3, bc=MOMENT, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5,
                   c_lo=0.3, c_hi=2.0, u_hi=0.03)
    s = random_state_3d(p, seed=4)
    a = d3.run(p, s.copy(), 6, nthreads=1)
    b = d3.run(p, s.copy(), 6, nthreads=4)
    assert np.array_equal(a, b)


# ---- two-relaxation-time collision ----

def _basis3():
    ex, ey, ez = (d3.EF[:, i].astype(float) for i in range(3))
    even = [np.ones(19), ex**2, ey**2, ez**2, ex * ey, ex * ez, ey * ez, ex**2 * ey**2,
            ex**2 * ez**2, ey**2 * ez**2]
    odd = [ex, ey, ez, ex * ey**2, ex * ez**2, ey * ex**2, ey * ez**2, ez * ex**2, ez * ey**2]
    gx, gy, gz = (d3.EG[:, i].astype(float) for i in range(3))
    return (np.array(even), np.array(odd), np.array([np.ones(7), gx**2, gy**2, gz**2]),
            np.array([gx, gy, gz]))


def test_trt_moment_bases_span_d3q19_and_d3q7():
    e9, o9, e7, o7 = _basis3()
    assert np.linalg.matrix_rank(np.vstack([e9, o9])) == 19
    assert np.linalg.matrix_rank(np.vstack([e7, o7])) == 7


@pytest.mark.parametrize("seed", range(4))
def test_trt_collision_moment_algebra_3d(seed):
    """Every basis moment relaxes at the rate of its parity (the bases span
    the population spaces, so this fixes the operator)."""
    rng = np.random.default_rng(100 + seed)
    tau_f, tau_fm, tau_m, tau_mp = rng.uniform(0.55, 2.0, 4)
    p = d3.Params3(nx=1, ny=3, nz=1, tau_f=tau_f, tau_m=tau_m, collision=d3.TRT,
                   tau_fm=tau_fm, tau_mp=tau_mp)
    f = rng.uniform(0.0, 0.3, 19)
    g = rng.uniform(-0.05, 0.05, (7, 3))
    rho = 1 + 0.1 * rng.uniform(-1, 1)
    u, b, F = 0.05 * rng.uniform(-1, 1, 3), 0.05 * rng.uniform(-1, 1, 3), 1e-3 * rng.uniform(-1, 1, 3)
    out = d3.collide(p, f, g, rho, u, b, F)
    feq = d3.feq(rho, u)
    S = d3.source(rho, u, F, feq)
    geq = d3.geq(b, u)  # [7][3]
    e9, o9, e7, o7 = _basis3()

    def relaxed(M, h, heq, tau, src=None):
        v = M @ h - (M @ h - M @ heq) / tau
        return v if src is None else v + (1 - 1 / (2 * tau)) * (M @ src)

    assert np.allclose(e9 @ out[:19], relaxed(e9, f, feq, tau_f, S), rtol=0, atol=1e-15)
    assert np.allclose(o9 @ out[:19], relaxed(o9, f, feq, tau_fm, S), rtol=0, atol=1e-15)
    for i in range(3):
        o = out[19 + 7 * i:26 + 7 * i]
        assert np.allclose(e7 @ o, relaxed(e7, g[:, i], geq[:, i], tau_mp), rtol=0, atol=1e-16)
        assert np.allclose(o7 @ o, relaxed(o7, g[:, i], geq[:, i], tau_m), rtol=0, atol=1e-16)


def _trt3(p, lf=3 / 16, lm=1 / 4):
    from oracle import derive
    tfm, tmp = derive.trt_times(p.tau_f, p.tau_m, lf, lm)
    return tfm, tmp


@pytest.mark.parametrize("case", CASES_2D)
def test_trt_z_invariant_run_reproduces_2d_trt_oracle(case):
    """The even/odd split commutes with the e_z sums, so a z-invariant TRT run
    is the 2D TRT run (the independent 2D oracle)."""
    bc, cl, cu, ul, uu, fx, fy = case
    p2 = Params(nx=7, ny=10, bc=bc, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=fy, c_lo=cl,
                c_hi=cu, u_lo=ul, u_hi=uu)
    tfm, tmp = _trt3(p2, 1 / 4, 1 / 12)
    p2 = Params(**{**p2.__dict__, "collision": oracle.TRT, "tau_fm": tfm, "tau_mp": tmp})
    s2 = random_state_2d(p2, seed=12)
    p3 = d3.Params3.from_2d(p2, 3)
    assert p3.collision == d3.TRT
    s3 = d3.lift_from_2d(s2, 3)
    a2 = oracle.run(p2, s2.copy(), 15)
    d3.run(p3, s3, 15)
    assert np.abs(d3.project_to_2d(s3) - a2).max() < 1e-14
    o3, o2 = d3.observe(p3, s3), oracle.observe(p2, a2)
    for k in ("rho", "ux", "uy", "bx", "by", "jz"):
        assert np.abs(o3[k][0] - o2[k]).max() < 1e-14, k


@pytest.mark.parametrize("bc,c", [(LINK, 0.4), (MOMENT, math.inf)])
def test_trt_x_z_exchange(bc, c):
    n = 6
    kw = dict(nx=n, ny=8, nz=n, bc=bc, tau_f=0.75, tau_m=0.85, b0=0.04, c_lo=c, c_hi=c,
              collision=d3.TRT, tau_fm=0.9, tau_mp=1.1)
    p = d3.Params3(fx=3e-5, **kw)
    q = d3.Params3(fz=3e-5, **kw)
    s = random_state_3d(p, seed=6)
    a = d3.run(p, s.copy(), 12)
    b = swap_xz(d3.run(q, swap_xz(s), 12))
    assert np.abs(a - b).max() < 1e-15


def test_trt_equal_rates_is_bgk_3d():
    kw = dict(nx=5, ny=7, nz=4, bc=MOMENT, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, fz=1e-5,
              c_lo=0.3, c_hi=math.inf, u_hi=0.03)
    s = random_state_3d(d3.Params3(**kw), seed=8)
    a = d3.run(d3.Params3(**kw), s.copy(), 10)
    b = d3.run(d3.Params3(**kw, collision=d3.TRT, tau_fm=0.7, tau_mp=0.9), s.copy(), 10)
    assert np.abs(a - b).max() < 1e-15
    c = d3.run(d3.Params3(**kw, collision=d3.TRT, tau_fm=0.8, tau_mp=0.9), s.copy(), 10)
    assert np.abs(c - a).max() > 1e-8
