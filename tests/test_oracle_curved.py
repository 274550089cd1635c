"""Pins of the oracle's curved walls (solid bodies closed by interpolated
bounce-back of f and anti-bounce-back of g on every link they cut; the paper
names such walls as future work, Sec. IX).

* q = 1/2: half-planes whose edges lie half-way between rows give every cut
  link q = 1/2, where the closure must be the paper's link-based Hartmann
  closure of an insulating wall (Sec. VI), moving wall included: the channel
  with solid rows above and below matches the plain channel row for row.
* mass: exact where every cut is at q = 1/2 (bounce-back); interpolated
  bounce-back at other q leaks a little, bounded here.
* second order: circular Couette flow between a rotating inner cylinder and
  a still outer one (no field) against its closed form u_theta = A r + B / r;
  the error falls about four-fold per doubling of the radii.
* mirror symmetry of a Hartmann channel with a disc on its axis.
* the cut distances against bisection along each link.
"""
import math

import numpy as np
import pytest

import oracle as O

NT = 8


def test_half_way_bodies_reduce_to_the_straight_link_walls():
    ny, nx, U = 12, 6, 0.03
    base = dict(nx=nx, bc=O.LINK, tau_f=0.8, tau_m=0.9, b0=0.02, fx=2e-6, c_lo=0.0, c_hi=0.0)
    straight = O.Params(ny=ny, u_hi=U, **base)
    bodies = O.Params(ny=ny + 4, a=ny / 2.0,
                      solids=((O.BELOW, 0.0, 1.5, 0.0, 0.0, 0.0),
                              (O.ABOVE, 0.0, ny + 1.5, 0.0, 0.0, U)), **base)
    s0, s1 = O.init_state(straight), O.init_state(bodies)
    # a non-trivial start: the same perturbation on the fluid rows
    rng = np.random.default_rng(3)
    pert = 1.0 + 0.01 * (rng.random(s0.shape) - 0.5)
    s0 *= pert
    s1[:, 2:ny + 2, :] *= pert
    O.run(straight, s0, 300, NT)
    O.run(bodies, s1, 300, NT)
    m0 = s1[:9].sum()
    diff = np.abs(s1[:, 2:ny + 2, :] - s0).max()
    assert diff < 1e-14, diff
    O.run(bodies, s1, 300, NT)
    assert abs(s1[:9].sum() - m0) / m0 < 1e-13  # bounce-back: no mass crosses (round-off)
    # the solid rows stay at rest
    rest = O.init_state(O.Params(ny=ny + 4, **base))[:, :2, :]
    assert np.abs(s1[:, :2, :] - rest).max() == 0.0


@pytest.mark.parametrize("omega,bound", [(0.0, 2e-6), (0.004, 4e-4)])
def test_disc_mass_leak_is_small(omega, bound):
    p = O.Params(nx=48, ny=32, bc=O.LINK, tau_f=0.8, tau_m=0.9, b0=0.03, fx=3e-6, c_lo=0.5,
                 c_hi=math.inf, solids=((O.DISC, 20.3, 15.7, 7.4, omega, 0.0),))
    s = O.init_state(p)
    m0 = s[:9].sum()
    O.run(p, s, 1000, NT)
    assert np.isfinite(s).all()
    drift = abs(s[:9].sum() - m0) / m0
    print("relative mass change", drift)
    assert drift < bound
    o = O.observe(p, s)
    assert np.abs(o["ux"]).max() > 1e-5  # the flow did develop


def _couette(n):
    """Circular Couette flow, inner radius n rotating, outer radius 2n at
    rest; returns the relative L2 error of u_theta and the largest |u_r|
    relative to the wall speed."""
    r1, r2, u0 = float(n), 2.0 * n, 0.01
    omega = u0 / r1
    size = 2 * int(math.ceil(r2)) + 6
    c = (size - 1) / 2.0
    tau = 0.8
    p = O.Params(nx=size, ny=size, bc=O.LINK, tau_f=tau, tau_m=0.8, b0=0.0,
                 solids=((O.BORE, c, c, r2, 0.0, 0.0), (O.DISC, c, c, r1, omega, 0.0)))
    s = O.init_state(p)
    nu = (tau - 0.5) / 3.0
    O.run(p, s, int(6 * (r2 - r1) ** 2 / nu), NT)
    o = O.observe(p, s)
    solid = O.solid_mask(p)
    y, x = np.mgrid[0:size, 0:size].astype(float)
    dx, dy = x - c, y - c
    r = np.hypot(dx, dy)
    A = -omega * r1 ** 2 / (r2 ** 2 - r1 ** 2)
    B = omega * r1 ** 2 * r2 ** 2 / (r2 ** 2 - r1 ** 2)
    fluid = ~solid
    ut = (-dy * o["ux"] + dx * o["uy"]) / np.where(r > 0, r, 1.0)
    ur = (dx * o["ux"] + dy * o["uy"]) / np.where(r > 0, r, 1.0)
    exact = A * r + B / np.where(r > 0, r, 1.0)
    err = np.sqrt(((ut - exact)[fluid] ** 2).sum() / (exact[fluid] ** 2).sum())
    return err, np.abs(ur[fluid]).max() / u0


def test_circular_couette_converges_at_second_order():
    e = [_couette(n) for n in (6, 12, 24)]
    errs = [v[0] for v in e]
    print("relative L2 errors", errs, "max |u_r|/u0", [v[1] for v in e])
    assert errs[0] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert a / b > 3.0, errs  # order > 1.58 per doubling, close to 2


def test_disc_on_the_axis_keeps_the_mirror_symmetry():
    ny = 31
    p = O.Params(nx=40, ny=ny, bc=O.LINK, tau_f=0.7, tau_m=0.9, b0=0.02, fx=2e-6, c_lo=0.3,
                 c_hi=0.3, solids=((O.DISC, 17.2, (ny - 1) / 2.0, 5.6, 0.0, 0.0),))
    s = O.init_state(p)
    O.run(p, s, 400, NT)
    o = O.observe(p, s)
    flip = lambda a: a[::-1, :]
    scale = np.abs(o["ux"]).max()
    assert np.abs(o["ux"] - flip(o["ux"])).max() < 1e-12 * scale + 1e-18
    assert np.abs(o["uy"] + flip(o["uy"])).max() < 1e-12 * scale + 1e-18
    bs = np.abs(o["bx"]).max()
    assert bs > 0
    assert np.abs(o["bx"] + flip(o["bx"])).max() < 1e-12 * bs + 1e-18


def test_cut_distances_match_bisection():
    p = O.Params(nx=30, ny=26, solids=((O.DISC, 13.37, 12.81, 5.9, 0.01, 0.0),
                                       (O.BELOW, 0.0, 2.3, 0.0, 0.0, 0.02)))
    solid = O.solid_mask(p)
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    cx, cy, r = 13.37, 12.81, 5.9
    inside = lambda X, Y: (X - cx) ** 2 + (Y - cy) ** 2 < r * r or Y < 2.3
    n = 0
    for y in range(1, p.ny - 1):
        for x in range(1, p.nx - 1):
            if solid[y, x]:
                continue
            for a in range(1, 9):
                ux, uy = x - ex[a], y - ey[a]
                cut = O.link_cut(p, x, y, a)
                assert (cut is not None) == bool(solid[uy, ux])
                if cut is None:
                    continue
                lo, hi = 0.0, 1.0  # bisection for the first point inside
                for _ in range(60):
                    mid = 0.5 * (lo + hi)
                    if inside(x - mid * ex[a], y - mid * ey[a]):
                        hi = mid
                    else:
                        lo = mid
                q, uwx, uwy = cut
                assert abs(q - hi) < 1e-9, (x, y, a, q, hi)
                if inside(x - hi * ex[a], y - hi * ey[a]) and (y - hi * ey[a]) >= 2.3:
                    # on the disc: rotation about its centre
                    wx, wy = x - q * ex[a] - cx, y - q * ey[a] - cy
                    assert abs(uwx + 0.01 * wy) < 1e-12 and abs(uwy - 0.01 * wx) < 1e-12
                n += 1
    assert n > 50
