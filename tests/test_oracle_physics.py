"""Steady-state pins of the oracle against the paper's closed forms.

* Body-force Hartmann flow vs Chang-Lundgren (Sec. VIII, experiments with
  both closures) and the paper's grid-convergence study: Ha = 20, tau = 0.9,
  tau_m = 0.95, N = 50, 100, 200, c_w = 0, 0.1, 0.5, 1, diffusive scaling,
  RMS error of Sec. VIII, observed order ~ 2.
* Shear-driven Hartmann-Couette flow vs App. C, with unequal wall
  conductances, both closures (paper's tau = 0.6, tau_m = 0.65).
* Ha = 0 Couette: both wall treatments reproduce the linear profile exactly.
* Equal wall conductances: the Couette velocity does not depend on c (App. C),
  up to the discretisation error.

The paper's own figures are not available as numbers, so closeness is
measured against the closed forms, and the order of convergence is the check.
"""
import math

import numpy as np
import pytest

from oracle import LINK, MOMENT, analytic, derive, steady


def hartmann_errors(bc, ny, tau_f, tau_m, ha, c, u_max, tol=1e-12):
    p = derive.hartmann_params(1, ny, bc, tau_f, tau_m, ha, c, u_max)
    _, obs, n, r = steady.run_to_steady(p, tol=tol, check_every=1000, max_steps=3_000_000)
    assert r < tol
    xi = analytic.node_xi(ny, bc)
    ua, ba = analytic.chang_lundgren(xi, ha, c)
    u = obs["ux"][:, 0] / derive.u_ref_hartmann(p.fx, tau_f, p.a)
    b = obs["bx"][:, 0] / derive.b_ref_hartmann(p.fx, tau_f, tau_m, p.a)
    return math.sqrt(np.mean((u - ua) ** 2)), math.sqrt(np.mean((b - ba) ** 2))


def couette_errors(bc, ny, tau_f, tau_m, ha, cl, cu, u_w, tol=1e-12):
    p = derive.couette_params(1, ny, bc, tau_f, tau_m, ha, cl, cu, u_w)
    _, obs, n, r = steady.run_to_steady(p, tol=tol, check_every=1000, max_steps=3_000_000)
    assert r < tol
    xi = analytic.node_xi(ny, bc)
    ua, ba = analytic.hartmann_couette(xi, ha, cl, cu)
    u = obs["ux"][:, 0] / u_w
    b = obs["bx"][:, 0] / derive.b_ref_couette(u_w, tau_f, tau_m)
    return math.sqrt(np.mean((u - ua) ** 2)), math.sqrt(np.mean((b - ba) ** 2)), obs


def orders(errs, ns=None, bc=LINK):
    """Observed orders between successive grids, measured in the half-width a."""
    if ns is None:
        return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    a = [derive.half_width(n, bc) for n in ns]
    return [math.log(errs[i] / errs[i + 1]) / math.log(a[i + 1] / a[i]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("c", [0.0, 0.1, 1.0, math.inf])
def test_hartmann_second_order(bc, c):
    # The moment-based errors mix terms of both signs until the Hartmann
    # layer is well resolved, so its order is read on the finer pair of three
    # grids at a smaller Ha (it rises towards 2 with refinement).
    ns, ha = ((32, 64), 10.0) if bc == LINK else ((32, 64, 128), 5.0)
    e = [hartmann_errors(bc, n, 0.8, 0.8, ha, c, 0.05 * 32 / n) for n in ns]
    ou, ob = orders([x[0] for x in e], ns, bc)[-1], orders([x[1] for x in e], ns, bc)[-1]
    lo = 1.9 if bc == LINK else 1.8
    assert ou > lo and ob > lo, (ou, ob, e)
    assert e[-1][0] < 2e-3 and e[-1][1] < 2e-3


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("c", [0.0, 0.1, 0.5, 1.0])
def test_paper_grid_convergence_study(bc, c):
    """Ha = 20, tau = 0.9, tau_m = 0.95, N = 50, 100 (and 200 for c <= 0.1)."""
    ns = (50, 100, 200) if c <= 0.1 else (50, 100)
    e = [hartmann_errors(bc, n, 0.9, 0.95, 20.0, c, 0.05 * 50 / n) for n in ns]
    ou, ob = orders([x[0] for x in e], ns, bc), orders([x[1] for x in e], ns, bc)
    if bc == LINK:
        assert min(ou + ob) > 1.9, (ou, ob)
    else:
        # the moment-based velocity is still pre-asymptotic at N = 50
        assert ou[-1] > 1.5 and min(ob) > 1.9, (ou, ob)
        if len(ou) > 1:
            assert ou[-1] > 1.85


COUETTE = [(5.0, 0.0, 0.0), (8.0, 0.5, 0.5), (5.0, 0.0, 0.5), (5.0, 0.5, 0.0),
           (5.0, 0.0, 0.1), (5.0, 0.0, 1.0), (5.0, 0.0, 1e4), (5.0, 0.0, math.inf),
           (5.0, math.inf, 0.3)]
# Both walls perfectly conducting with one moving has no steady state: the
# induction flux gives d/dt int B_x dy = B0 (U_u - U_l) when dB_x/dy = 0 on both
# walls, and App. C's K2 diverges accordingly.


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("ha,cl,cu", COUETTE)
def test_couette_second_order(bc, ha, cl, cu):
    ns = (26, 51)
    e = [couette_errors(bc, n, 0.6, 0.65, ha, cl, cu, 0.05 * 26 / n)[:2] for n in ns]
    ou = orders([x[0] for x in e], ns, bc)[0]
    ob = orders([x[1] for x in e], ns, bc)[0]
    lo = 1.85 if bc == LINK else 1.6
    assert ou > lo and ob > lo, (ou, ob, e)


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_ha0_couette_is_exactly_linear(bc, tau):
    p = derive.couette_params(1, 20, bc, tau, 0.7, 0.0, 0.3, 0.3, 0.05)
    _, obs, _, _ = steady.run_to_steady(p, tol=1e-14, check_every=1000)
    xi = analytic.node_xi(20, bc)
    assert np.abs(obs["ux"][:, 0] - 0.05 * 0.5 * (1 + xi)).max() < 5e-13


@pytest.mark.parametrize("bc", [LINK, MOMENT])
def test_couette_velocity_independent_of_equal_c(bc):
    """The c-dependence of the computed velocity is discretisation error: it
    is small and shrinks at second order under refinement."""
    diffs = []
    for n in (21, 41):
        u_w = 0.05 * 21 / n
        us = [couette_errors(bc, n, 0.6, 0.65, 5.0, c, c, u_w)[2]["ux"][:, 0] / u_w
              for c in (0.0, 0.5, 5.0)]
        diffs.append(max(np.abs(u - us[0]).max() for u in us[1:]))
    assert diffs[-1] < 1e-2
    assert diffs[0] / diffs[1] > 3.0, diffs
