"""Pins of the 3D oracle's multiple-relaxation-time (MRT) collision.

The reading follows the 2D one: f in the orthogonal D3Q19 basis of
d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo (Phil. Trans. R. Soc. A
360 (2002) 437) with the five stresses at 1/tau_f, e at s_fe, epsilon and
the fourth-order pi_xx, pi_ww at s_feps, and q and the third-order m at
s_fq; each component of g (D3Q7) with Lambda at 1/tau_m and its two
traceless second moments at s_md (its isotropic second moment has no
non-equilibrium part: the rest weight is zero).

* Reductions: with s_fe = s_feps = 1/tau_f and s_md = TRT's even rate, MRT
  is the separately written and pinned 3D TRT step; with every rate at
  1/tau it is BGK.
* x <-> z exchange: the basis is isotropic, so the exchange that holds for
  BGK and TRT holds for MRT with distinct rates; a wrong row or a rate on
  the wrong component of a moment breaks it.
* Uniform modes: away from the walls, a non-equilibrium part put into one
  moment of a uniform state at rest decays as (1 - s)^n and leaves the
  others at equilibrium, for every free moment of f and g.
* Exact solution: steady Hartmann flow (x- and z-invariant) converges to the
  Chang-Lundgren profile at second order with distinct rates.
* Conservation: mass with link walls.
"""
import math

import numpy as np
import pytest

from oracle import LINK, MOMENT, analytic, derive
from oracle import d3
from tests.test_oracle3d import random_state_3d, swap_xz

RATES = dict(s_fe=1.19, s_feps=1.4, s_fq=1.2, s_md=1.6)


def mrt3(**kw):
    r = {**RATES, **{k: kw.pop(k) for k in list(kw) if k in RATES}}
    return d3.Params3(collision=d3.MRT, **r, **kw)


KW = dict(nx=5, ny=7, nz=4, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, fz=1e-5, c_lo=0.3,
          c_hi=math.inf, u_hi=0.03)


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_mrt3_with_trt_rates_is_trt(bc):
    tfm, tmp = derive.trt_times(0.7, 0.9, 3.0 / 16.0, 0.25)
    t = d3.Params3(bc=bc, collision=d3.TRT, tau_fm=tfm, tau_mp=tmp, **KW)
    m = mrt3(bc=bc, s_fe=1 / 0.7, s_feps=1 / 0.7, s_fq=1 / tfm, s_md=1 / tmp, **KW)
    s = random_state_3d(t, seed=31)
    st = d3.run(t, s.copy(), 10)
    assert np.abs(d3.run(m, s.copy(), 10) - st).max() < 1e-14
    for k, v in RATES.items():   # each free rate matters
        r = dict(s_fe=1 / 0.7, s_feps=1 / 0.7, s_fq=1 / tfm, s_md=1 / tmp)
        r[k] = v
        assert np.abs(d3.run(mrt3(bc=bc, **r, **KW), s.copy(), 10) - st).max() > 1e-9, k


def test_mrt3_side_walls_with_trt_rates_is_trt():
    kw = dict(KW, nz=5, side_walls=True, cs_lo=0.5, cs_hi=math.inf)
    tfm, tmp = derive.trt_times(0.7, 0.9, 3.0 / 16.0, 0.25)
    t = d3.Params3(bc=LINK, collision=d3.TRT, tau_fm=tfm, tau_mp=tmp, **kw)
    m = mrt3(bc=LINK, s_fe=1 / 0.7, s_feps=1 / 0.7, s_fq=1 / tfm, s_md=1 / tmp, **kw)
    s = random_state_3d(t, seed=32)
    assert np.abs(d3.run(m, s.copy(), 10) - d3.run(t, s.copy(), 10)).max() < 1e-14


def test_mrt3_with_equal_rates_is_bgk():
    b = d3.Params3(bc=MOMENT, **KW)
    m = mrt3(bc=MOMENT, s_fe=1 / 0.7, s_feps=1 / 0.7, s_fq=1 / 0.7, s_md=1 / 0.9, **KW)
    s = random_state_3d(b, seed=33)
    assert np.abs(d3.run(m, s.copy(), 10) - d3.run(b, s.copy(), 10)).max() < 1e-14


@pytest.mark.parametrize("bc,c", [(LINK, 0.4), (MOMENT, math.inf)])
def test_mrt3_x_z_exchange(bc, c):
    n = 6
    kw = dict(nx=n, ny=8, nz=n, bc=bc, tau_f=0.75, tau_m=0.85, b0=0.04, c_lo=c, c_hi=c)
    p = mrt3(fx=3e-5, **kw)
    q = mrt3(fz=3e-5, **kw)
    s = random_state_3d(p, seed=34)
    a = d3.run(p, s.copy(), 12)
    b = swap_xz(d3.run(q, swap_xz(s), 12))
    assert np.abs(a - b).max() < 1e-15


def _rows_f():
    E = d3.EF.astype(float)
    ex, ey, ez = E[:, 0], E[:, 1], E[:, 2]
    e2 = ex * ex + ey * ey + ez * ez
    return {"e": 19 * e2 - 30, "eps": (21 * e2 * e2 - 53 * e2 + 24) / 2,
            "qx": (5 * e2 - 9) * ex, "qy": (5 * e2 - 9) * ey, "qz": (5 * e2 - 9) * ez,
            "3pxx": 3 * ex * ex - e2, "3pixx": (3 * e2 - 5) * (3 * ex * ex - e2),
            "pww": ey * ey - ez * ez, "piww": (3 * e2 - 5) * (ey * ey - ez * ez),
            "pxy": ex * ey, "pyz": ey * ez, "pxz": ex * ez,
            "mx": (ey * ey - ez * ez) * ex, "my": (ez * ez - ex * ex) * ey,
            "mz": (ex * ex - ey * ey) * ez}


def _rows_g():
    E = d3.EG.astype(float)
    ex, ey, ez = E[:, 0], E[:, 1], E[:, 2]
    return {"a": 2 * ex * ex - ey * ey - ez * ez, "w": ey * ey - ez * ez}


def test_mrt3_uniform_modes_decay_at_their_own_rates():
    tau_f, tau_m = 0.8, 0.9
    snu = 1 / tau_f
    rate = {"e": RATES["s_fe"], "eps": RATES["s_feps"], "3pixx": RATES["s_feps"],
            "piww": RATES["s_feps"], "qx": RATES["s_fq"], "qy": RATES["s_fq"],
            "qz": RATES["s_fq"], "mx": RATES["s_fq"], "my": RATES["s_fq"], "mz": RATES["s_fq"],
            "3pxx": snu, "pww": snu, "pxy": snu, "pyz": snu, "pxz": snu,
            "a": RATES["s_md"], "w": RATES["s_md"]}
    n, amp = 3, 1e-3
    for plane0, rows in ((0, _rows_f()), (19, _rows_g()), (26, _rows_g()), (33, _rows_g())):
        for name, row in rows.items():
            p = mrt3(nx=3, ny=12, nz=3, bc=LINK, tau_f=tau_f, tau_m=tau_m)
            s = d3.init_state(p)
            eq = d3.init_state(p)
            s[plane0:plane0 + len(row)] += (amp * row / (row @ row))[:, None, None, None]
            d3.run(p, s, n)
            for y in (5, 6):
                d = s[plane0:plane0 + len(row), 1, y, 1] - eq[plane0:plane0 + len(row), 1, y, 1]
                for other, orow in rows.items():
                    got = orow @ d
                    want = amp * (1 - rate[name]) ** n if other == name else 0.0
                    assert abs(got - want) < 2e-13, (plane0, name, other, got, want)
                assert abs(d.sum()) < 2e-13


def test_mrt3_hartmann_flow_converges_to_the_closed_form():
    def errors(ny, ha=5.0, c=0.5, tau=0.8):
        a = ny / 2.0
        nu = eta = (tau - 0.5) / 3.0
        fx = derive.fx_for_umax(0.02, ha, c, tau, a)
        p = mrt3(nx=1, ny=ny, nz=1, bc=LINK, tau_f=tau, tau_m=tau,
                 b0=ha * math.sqrt(nu * eta) / a, fx=fx, c_lo=c, c_hi=c)
        s = d3.init_state(p)
        prev = None
        for _ in range(300):
            d3.run(p, s, 2000, nthreads=8)
            o = d3.observe(p, s)
            if prev is not None and np.linalg.norm(o["ux"] - prev) < 1e-11 * np.linalg.norm(o["ux"]):
                break
            prev = o["ux"].copy()
        y = (np.arange(ny) + 0.5 - a) / a
        us, bs = analytic.chang_lundgren(y, ha, c)
        U, B = a * a * fx / nu, a * a * fx / math.sqrt(nu * eta)
        ux, bx = o["ux"][0, :, 0], o["bx"][0, :, 0]
        return (np.linalg.norm(ux - U * us) / np.linalg.norm(U * us),
                np.linalg.norm(bx - B * bs) / np.linalg.norm(B * bs))
    e16, e32 = errors(16), errors(32)
    for k in range(2):
        assert e32[k] < 2.5e-2 and e16[k] / e32[k] > 3.4, (e16, e32)


def test_mrt3_conserves_mass():
    p = mrt3(nx=5, ny=8, nz=4, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, c_lo=0.2,
             c_hi=math.inf, u_lo=-0.02, u_hi=0.03)
    s = random_state_3d(p, seed=35)
    m0 = s[:19].sum()
    d3.run(p, s, 20)
    assert abs(s[:19].sum() - m0) / m0 < 1e-14
