"""FP64 CPU oracle for the lattice-kinetic MHD step (arXiv 2112.13930).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or executes anything here, and this package imports nothing from it.

Contents
  lks_oracle.c   plain C reference step (pull stream, wall closures, moments,
                 coupled u/J solve, BGK, TRT or MRT collisions) -- built into
                 liblks_oracle.so by :func:`build`.
  analytic.py    closed-form Hartmann (Chang-Lundgren) and Hartmann-Couette
                 profiles of Sec. VIII and App. C.
  derive.py      lattice parameters (nu, eta, a, B0, F_x, theta) from the
                 physical ones, per Secs. IV, V, VI and VIII.
  steady.py      run-to-steady driver with the residual used for stopping.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lks_oracle.c")
LIB = os.path.join(HERE, "liblks_oracle.so")

LINK, MOMENT = 0, 1
BGK, TRT, MRT = 0, 1, 2
NPLANES = 19


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


DISC, BORE, BELOW, ABOVE = 1, 2, 3, 4  # solid bodies (curved walls)


class _Solid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("r", ctypes.c_double), ("omega", ctypes.c_double),
                ("u", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("tau_f", ctypes.c_double), ("tau_m", ctypes.c_double),
        ("b0", ctypes.c_double), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
        ("c_lo", ctypes.c_double), ("c_hi", ctypes.c_double),
        ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double),
        ("a", ctypes.c_double),
        ("tau_fm", ctypes.c_double), ("tau_mp", ctypes.c_double),
        ("x_walls", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("cx_lo", ctypes.c_double), ("cx_hi", ctypes.c_double),
        ("q_lo", ctypes.c_double), ("q_hi", ctypes.c_double),
        ("s_fe", ctypes.c_double), ("s_feps", ctypes.c_double), ("s_fq", ctypes.c_double),
        ("s_me", ctypes.c_double), ("s_md", ctypes.c_double),
        ("nsolid", ctypes.c_int32), ("pad2_", ctypes.c_int32),
        ("solid", _Solid * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        L.orc_feq.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_geq.argtypes = [ctypes.c_double] * 4 + [dp, dp]
        L.orc_source.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        L.orc_local_solve.argtypes = [ctypes.c_double] * 10 + [dp]
        L.orc_link_closure.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp]
        L.orc_moment_closure.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        L.orc_init.argtypes = [pp, ctypes.c_double, dp]
        L.orc_step.argtypes = [pp, dp, dp, ctypes.c_int]
        L.orc_run.argtypes = [pp, dp, dp, ctypes.c_int64, ctypes.c_int]
        L.orc_observe.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_gather.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_collide.argtypes = [pp, dp, dp, dp] + [ctypes.c_double] * 7 + [dp]
        L.orc_xwall_closure.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp]
        L.orc_is_solid.argtypes = [pp, ctypes.c_int, ctypes.c_int]
        L.orc_is_solid.restype = ctypes.c_int
        L.orc_link_cut.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_link_cut.restype = ctypes.c_int
        for fn in ("orc_feq", "orc_geq", "orc_source", "orc_local_solve",
                   "orc_link_closure", "orc_moment_closure", "orc_init",
                   "orc_step", "orc_run", "orc_observe", "orc_gather", "orc_collide",
                   "orc_xwall_closure"):
            getattr(L, fn).restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Lattice parameters of one channel (lattice units, rho0 = 1).

    ``c_lo``/``c_hi`` may be ``math.inf``; ``a`` is the half-width H = a used in
    the wall-conductance terms.  Use :mod:`oracle.derive` to obtain them from
    (Ha, c_w, u_max) the way Sec. VIII defines the problem.

    ``collision`` selects BGK (the paper's operator) or TRT.  Under TRT,
    ``tau_f`` relaxes the even part of f and ``tau_fm`` its odd part, ``tau_m``
    the odd part of g and ``tau_mp`` its even part
    (:func:`oracle.derive.trt_times` gives them from the magic parameters).
    Under MRT, f's moments p_xx and p_xy relax at 1/tau_f and e, epsilon and q
    at ``s_fe``, ``s_feps`` and ``s_fq``; g's Lambda moments at 1/tau_m and its
    epsilon and d moments at ``s_me`` and ``s_md`` (:func:`oracle.derive.mrt_rates`).
    """
    nx: int
    ny: int
    bc: int = LINK
    tau_f: float = 0.8
    tau_m: float = 0.8
    b0: float = 0.0
    fx: float = 0.0
    fy: float = 0.0
    c_lo: float = 0.0
    c_hi: float = 0.0
    u_lo: float = 0.0
    u_hi: float = 0.0
    a: float = float("nan")
    rho0: float = 1.0
    collision: int = BGK
    tau_fm: float = float("nan")
    tau_mp: float = float("nan")
    x_walls: bool = False  # enclosure: stationary Shercliff walls bound x
    cx_lo: float = 0.0     # their conductance ratios (x = 0 side, x = nx-1 side)
    cx_hi: float = 0.0
    q_lo: float = 0.5      # link scheme: Hartmann wall distance from its wall row
    q_hi: float = 0.5
    s_fe: float = float("nan")    # MRT rates (collision == MRT)
    s_feps: float = float("nan")
    s_fq: float = float("nan")
    s_me: float = float("nan")
    s_md: float = float("nan")
    # solid bodies (curved walls): (kind, cx, cy, r, omega, u) with kind DISC
    # (solid inside the circle), BORE (solid outside), BELOW (y < cy) or
    # ABOVE (y > cy); omega the circle's surface angular velocity, u a
    # half-plane's velocity along x
    solids: tuple = ()
    extra: dict = field(default_factory=dict)

    def half_width(self) -> float:
        if not math.isnan(self.a):
            return self.a
        if self.bc == LINK:
            return (self.ny - 1 + self.q_lo + self.q_hi) / 2.0
        return (self.ny - 1) / 2.0

    def c_struct(self) -> _Params:
        if self.collision == TRT:
            assert self.tau_fm > 0.5 and self.tau_mp > 0.5, "TRT needs tau_fm and tau_mp > 1/2"
        if self.collision == MRT:
            assert all(0 < r < 2 for r in (self.s_fe, self.s_feps, self.s_fq, self.s_me,
                                           self.s_md)), "MRT needs rates in (0, 2)"
        if self.x_walls:
            assert self.bc == LINK and self.nx >= 2, "enclosure walls need link-based closures"
        if (self.q_lo, self.q_hi) != (0.5, 0.5):
            assert self.bc == LINK and 0 < self.q_lo <= 1 and 0 < self.q_hi <= 1
        assert len(self.solids) <= 4, "at most four solid bodies"
        if self.solids:
            assert not self.x_walls and (self.q_lo, self.q_hi) == (0.5, 0.5), \
                "solid bodies need an x-periodic channel with half-way Hartmann walls"
        bodies = (_Solid * 4)()
        for k, b in enumerate(self.solids):
            kind, cx, cy, r, omega, u = b
            bodies[k] = _Solid(int(kind), 0, cx, cy, r, omega, u)
        return _Params(self.nx, self.ny, self.bc, self.collision, self.tau_f, self.tau_m,
                       self.b0, self.fx, self.fy, self.c_lo, self.c_hi,
                       self.u_lo, self.u_hi, self.half_width(), self.tau_fm, self.tau_mp,
                       int(self.x_walls), 0, self.cx_lo, self.cx_hi, self.q_lo, self.q_hi,
                       self.s_fe, self.s_feps, self.s_fq, self.s_me, self.s_md,
                       len(self.solids), 0, bodies)


def init_state(p: Params) -> np.ndarray:
    s = np.empty((NPLANES, p.ny, p.nx), dtype=np.float64)
    cp = p.c_struct()
    lib().orc_init(ctypes.byref(cp), p.rho0, _dp(s))
    return s


def step(p: Params, state: np.ndarray, nthreads: int = 1) -> np.ndarray:
    out = np.empty_like(state)
    cp = p.c_struct()
    lib().orc_step(ctypes.byref(cp), _dp(state), _dp(out), nthreads)
    return out


def run(p: Params, state: np.ndarray, nsteps: int, nthreads: int = 1,
        scratch: np.ndarray | None = None) -> np.ndarray:
    """Advance ``state`` in place by ``nsteps`` steps and return it."""
    assert state.shape == (NPLANES, p.ny, p.nx)
    if scratch is None:
        scratch = np.empty_like(state)
    cp = p.c_struct()
    lib().orc_run(ctypes.byref(cp), _dp(state), _dp(scratch), int(nsteps), nthreads)
    return state


def observe(p: Params, state: np.ndarray) -> dict:
    """rho, ux, uy, bx, by, jz of the state (the fields the next step uses)."""
    out = {k: np.empty((p.ny, p.nx), dtype=np.float64)
           for k in ("rho", "ux", "uy", "bx", "by", "jz")}
    cp = p.c_struct()
    lib().orc_observe(ctypes.byref(cp), _dp(state), *(_dp(out[k]) for k in
                      ("rho", "ux", "uy", "bx", "by", "jz")))
    return out


def gather(p: Params, state: np.ndarray, x: int, y: int) -> np.ndarray:
    """Post-streaming, post-closure populations of node (x, y)."""
    out = np.empty(NPLANES, dtype=np.float64)
    cp = p.c_struct()
    lib().orc_gather(ctypes.byref(cp), _dp(state), x, y, _dp(out))
    return out


def feq(rho, ux, uy) -> np.ndarray:
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, _dp(out))
    return out


def geq(bx, by, ux, uy):
    gx, gy = np.empty(5), np.empty(5)
    lib().orc_geq(bx, by, ux, uy, _dp(gx), _dp(gy))
    return gx, gy


def source(rho, ux, uy, Fx, Fy, feq_):
    out = np.empty(9)
    lib().orc_source(rho, ux, uy, Fx, Fy, _dp(np.ascontiguousarray(feq_, dtype=np.float64)), _dp(out))
    return out


def local_solve(rho, mx, my, bx, by, lxy, lyx, tau_m, fex=0.0, fey=0.0):
    out = np.empty(3)
    lib().orc_local_solve(rho, mx, my, bx, by, lxy, lyx, tau_m, fex, fey, _dp(out))
    return out


def link_closure(p: Params, wall: int, own: np.ndarray, f, gx, gy):
    f, gx, gy = (np.array(v, dtype=np.float64) for v in (f, gx, gy))
    cp = p.c_struct()
    lib().orc_link_closure(ctypes.byref(cp), wall, _dp(np.ascontiguousarray(own, dtype=np.float64)),
                           _dp(f), _dp(gx), _dp(gy))
    return f, gx, gy


def moment_closure(p: Params, wall: int, f, gx, gy):
    f, gx, gy = (np.array(v, dtype=np.float64) for v in (f, gx, gy))
    cp = p.c_struct()
    lib().orc_moment_closure(ctypes.byref(cp), wall, _dp(f), _dp(gx), _dp(gy))
    return f, gx, gy


def collide(p: Params, f, gx, gy, rho, ux, uy, bx, by, Fx, Fy) -> np.ndarray:
    """Post-collision values (19, plane order) of one node's populations."""
    f, gx, gy = (np.ascontiguousarray(v, dtype=np.float64) for v in (f, gx, gy))
    out = np.empty(NPLANES)
    cp = p.c_struct()
    lib().orc_collide(ctypes.byref(cp), _dp(f), _dp(gx), _dp(gy), rho, ux, uy, bx, by, Fx,
                      Fy, _dp(out))
    return out


def xwall_closure(p: Params, wall: int, own, f, gx, gy):
    """Apply the enclosure-wall closure (wall 0: x = 0 side, 1: x = nx-1
    side) to one node's pulled populations; own: its 19 previous
    post-collision values."""
    f, gx, gy = (np.array(v, dtype=np.float64) for v in (f, gx, gy))
    cp = p.c_struct()
    lib().orc_xwall_closure(ctypes.byref(cp), wall,
                            _dp(np.ascontiguousarray(own, dtype=np.float64)), _dp(f), _dp(gx),
                            _dp(gy))
    return f, gx, gy


def solid_mask(p: Params) -> np.ndarray:
    """(ny, nx) bool array of the solid nodes."""
    cp = p.c_struct()
    L = lib()
    return np.array([[bool(L.orc_is_solid(ctypes.byref(cp), x, y)) for x in range(p.nx)]
                     for y in range(p.ny)])


def link_cut(p: Params, x: int, y: int, a: int):
    """(q, u_wall_x, u_wall_y) of the link of fluid node (x, y) towards its
    upstream node (x, y) - e_a (D2Q9 numbering) if a body contains that
    node, else None."""
    cp = p.c_struct()
    q, ux, uy = (np.zeros(1) for _ in range(3))
    if lib().orc_link_cut(ctypes.byref(cp), x, y, a, _dp(q), _dp(ux), _dp(uy)):
        return float(q[0]), float(ux[0]), float(uy[0])
    return None
