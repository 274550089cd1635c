"""Three-dimensional channel oracle (TEST INFRASTRUCTURE ONLY).

ctypes wrapper of lks_oracle3.c: D3Q19 flow distribution with the Lorentz
force, three-component D3Q7 magnetic distribution (zero rest weight), both
Shercliff closures on the Hartmann walls y = 0 and y = ny-1, x and z
periodic.  The lattice choices and why a z-invariant run reproduces the
two-dimensional scheme exactly are given in the C file's header.

State: FP64 array [40][nz][ny][nx]: f_0..f_18, then g_x, g_y, g_z with
seven populations each (rest first).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lks_oracle3.c")
LIB = os.path.join(HERE, "liblks_oracle3.so")

LINK, MOMENT = 0, 1
BGK, TRT, MRT = 0, 1, 2
NPLANES = 40
NF, NG = 19, 7


def build(force: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("tau_f", ctypes.c_double), ("tau_m", ctypes.c_double), ("b0", ctypes.c_double),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("fz", ctypes.c_double),
        ("c_lo", ctypes.c_double), ("c_hi", ctypes.c_double),
        ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double), ("a", ctypes.c_double),
        ("collision", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("tau_fm", ctypes.c_double), ("tau_mp", ctypes.c_double),
        ("side_walls", ctypes.c_int32), ("pad2_", ctypes.c_int32),
        ("cs_lo", ctypes.c_double), ("cs_hi", ctypes.c_double),
        ("s_fe", ctypes.c_double), ("s_feps", ctypes.c_double), ("s_fq", ctypes.c_double),
        ("s_md", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params3)
        L.orc3_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc3_geq.argtypes = [dp, dp, dp]
        L.orc3_source.argtypes = [ctypes.c_double, dp, dp, dp, dp]
        L.orc3_local_solve.argtypes = [ctypes.c_double, dp, dp, dp, ctypes.c_double, dp, dp]
        L.orc3_link_closure.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        L.orc3_moment_closure.argtypes = [pp, ctypes.c_int, dp, dp]
        L.orc3_init.argtypes = [pp, ctypes.c_double, dp]
        L.orc3_step.argtypes = [pp, dp, dp, ctypes.c_int]
        L.orc3_run.argtypes = [pp, dp, dp, ctypes.c_int64, ctypes.c_int]
        L.orc3_observe.argtypes = [pp, dp, dp]
        L.orc3_gather.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc3_collide.argtypes = [pp, dp, dp, ctypes.c_double, dp, dp, dp, dp]
        L.orc3_side_closure.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        for name in ("orc3_feq", "orc3_geq", "orc3_source", "orc3_local_solve",
                     "orc3_link_closure", "orc3_moment_closure", "orc3_init", "orc3_step",
                     "orc3_run", "orc3_observe", "orc3_gather", "orc3_collide",
                     "orc3_side_closure"):
            getattr(L, name).restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params3:
    nx: int
    ny: int
    nz: int
    bc: int = LINK
    tau_f: float = 0.8
    tau_m: float = 0.8
    b0: float = 0.0
    fx: float = 0.0
    fy: float = 0.0
    fz: float = 0.0
    c_lo: float = 0.0
    c_hi: float = 0.0
    u_lo: float = 0.0
    u_hi: float = 0.0
    a: float | None = None
    collision: int = BGK
    tau_fm: float = float("nan")
    tau_mp: float = float("nan")
    side_walls: bool = False   # duct: stationary Shercliff walls bound z
    cs_lo: float = 0.0         # their conductance ratios (z = 0 side, z = nz-1 side)
    cs_hi: float = 0.0
    s_fe: float = float("nan")     # MRT (collision == MRT): e at s_fe, epsilon and pi at
    s_feps: float = float("nan")   # s_feps, q and m at s_fq; g's traceless second moments
    s_fq: float = float("nan")     # at s_md
    s_md: float = float("nan")

    def half_width(self) -> float:
        if self.a is not None:
            return self.a
        return self.ny / 2.0 if self.bc == LINK else (self.ny - 1) / 2.0

    def c_struct(self) -> _Params3:
        if self.collision == TRT:
            assert self.tau_fm > 0.5 and self.tau_mp > 0.5, "TRT needs tau_fm and tau_mp > 1/2"
        if self.collision == MRT:
            assert all(0 < r < 2 for r in (self.s_fe, self.s_feps, self.s_fq, self.s_md)), \
                "MRT needs rates in (0, 2)"
        if self.side_walls:
            assert self.bc == LINK and self.nz >= 2, "side walls need link-based closures"
        return _Params3(self.nx, self.ny, self.nz, self.bc, self.tau_f, self.tau_m, self.b0,
                        self.fx, self.fy, self.fz, self.c_lo, self.c_hi, self.u_lo, self.u_hi,
                        self.half_width(), self.collision, 0, self.tau_fm, self.tau_mp,
                        int(self.side_walls), 0, self.cs_lo, self.cs_hi, self.s_fe,
                        self.s_feps, self.s_fq, self.s_md)

    @classmethod
    def from_2d(cls, p, nz: int) -> "Params3":
        """The 3D channel with the 2D parameter set p (oracle.Params) and nz
        periodic layers."""
        return cls(nx=p.nx, ny=p.ny, nz=nz, bc=p.bc, tau_f=p.tau_f, tau_m=p.tau_m, b0=p.b0,
                   fx=p.fx, fy=p.fy, fz=0.0, c_lo=p.c_lo, c_hi=p.c_hi, u_lo=p.u_lo,
                   u_hi=p.u_hi, a=p.half_width(), collision=p.collision, tau_fm=p.tau_fm,
                   tau_mp=p.tau_mp, s_fe=p.s_fe, s_feps=p.s_feps, s_fq=p.s_fq, s_md=p.s_md)


def init_state(p: Params3, rho0: float = 1.0) -> np.ndarray:
    s = np.empty((NPLANES, p.nz, p.ny, p.nx), dtype=np.float64)
    ps = p.c_struct()
    lib().orc3_init(ctypes.byref(ps), rho0, _dp(s))
    return s


def step(p: Params3, state: np.ndarray, nthreads: int = 1) -> np.ndarray:
    out = np.empty_like(state)
    ps = p.c_struct()
    lib().orc3_step(ctypes.byref(ps), _dp(state), _dp(out), nthreads)
    return out


def run(p: Params3, state: np.ndarray, nsteps: int, nthreads: int = 1,
        scratch: np.ndarray | None = None) -> np.ndarray:
    """nsteps steps in place on state; returns state."""
    if scratch is None:
        scratch = np.empty_like(state)
    ps = p.c_struct()
    lib().orc3_run(ctypes.byref(ps), _dp(state), _dp(scratch), int(nsteps), nthreads)
    return state


OBS = ("rho", "ux", "uy", "uz", "bx", "by", "bz", "jx", "jy", "jz")


def observe(p: Params3, state: np.ndarray) -> dict:
    out = np.empty((10, p.nz, p.ny, p.nx), dtype=np.float64)
    ps = p.c_struct()
    lib().orc3_observe(ctypes.byref(ps), _dp(state), _dp(out))
    return {k: out[i] for i, k in enumerate(OBS)}


def gather(p: Params3, state: np.ndarray, x: int, y: int, z: int) -> np.ndarray:
    out = np.empty(NPLANES, dtype=np.float64)
    ps = p.c_struct()
    lib().orc3_gather(ctypes.byref(ps), _dp(state), x, y, z, _dp(out))
    return out


def feq(rho, u) -> np.ndarray:
    out = np.empty(NF)
    lib().orc3_feq(rho, _dp(np.asarray(u, dtype=np.float64)), _dp(out))
    return out


def geq(b, u) -> np.ndarray:
    """[7, 3] array g^eq_{alpha i}."""
    out = np.empty(NG * 3)
    lib().orc3_geq(_dp(np.asarray(b, dtype=np.float64)), _dp(np.asarray(u, dtype=np.float64)),
                   _dp(out))
    return out.reshape(NG, 3)


def source(rho, u, F, feq_) -> np.ndarray:
    out = np.empty(NF)
    lib().orc3_source(rho, _dp(np.asarray(u, dtype=np.float64)),
                      _dp(np.asarray(F, dtype=np.float64)),
                      _dp(np.ascontiguousarray(feq_, dtype=np.float64)), _dp(out))
    return out


def local_solve(rho, m, b, lam, tau_m, fext=(0.0, 0.0, 0.0)):
    """(u[3], J[3]); lam is the 3x3 array Lambda[j][i]."""
    out = np.empty(6)
    lib().orc3_local_solve(rho, _dp(np.asarray(m, dtype=np.float64)),
                           _dp(np.asarray(b, dtype=np.float64)),
                           _dp(np.ascontiguousarray(lam, dtype=np.float64).reshape(9)), tau_m,
                           _dp(np.asarray(fext, dtype=np.float64)), _dp(out))
    return out[:3], out[3:]


def collide(p: Params3, f, g, rho, u, b, F) -> np.ndarray:
    """The 40 post-collision values of one node (g given as [7][3])."""
    out = np.empty(NPLANES)
    lib().orc3_collide(ctypes.byref(p.c_struct()),
                       _dp(np.ascontiguousarray(f, dtype=np.float64)),
                       _dp(np.ascontiguousarray(g, dtype=np.float64).reshape(21)), rho,
                       _dp(np.asarray(u, dtype=np.float64)), _dp(np.asarray(b, dtype=np.float64)),
                       _dp(np.asarray(F, dtype=np.float64)), _dp(out))
    return out


def side_closure(p: Params3, wall: int, own, f, g):
    """Apply the side-wall closure (wall 0: z = 0 side, 1: z = nz-1 side) to
    one node's pulled populations f[19], g[7][3]; own are its 40 previous
    post-collision values."""
    f = np.array(f, dtype=np.float64)
    g = np.array(g, dtype=np.float64).reshape(21)
    lib().orc3_side_closure(ctypes.byref(p.c_struct()), wall,
                            _dp(np.ascontiguousarray(own, dtype=np.float64)), _dp(f), _dp(g))
    return f, g.reshape(7, 3)


# Velocity sets, typed here for the tests only (the C file has its own).
EF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [1, 1, 0], [-1, 1, 0],
               [-1, -1, 0], [1, -1, 0], [0, 0, 1], [0, 0, -1], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
EG = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])


def project_to_2d(state3: np.ndarray) -> np.ndarray:
    """Sum a z-invariant 3D state over e_z into the 2D layout [19][ny][nx]
    (one z layer): f by (e_x, e_y) groups into D2Q9, g by (e_x, e_y) groups
    into D2Q5 per in-plane component."""
    s = state3[:, 0]
    d2q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    d2q5 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)]
    out = np.zeros((19,) + s.shape[1:])
    for q, (ex, ey) in enumerate(d2q9):
        for r in range(NF):
            if EF[r, 0] == ex and EF[r, 1] == ey:
                out[q] += s[r]
    for comp in range(2):
        for q, (ex, ey) in enumerate(d2q5):
            for r in range(NG):
                if EG[r, 0] == ex and EG[r, 1] == ey:
                    out[9 + 5 * comp + q] += s[NF + comp * NG + r]
    return out


def lift_from_2d(state2: np.ndarray, nz: int) -> np.ndarray:
    """A z-invariant 3D state whose e_z sums are the 2D state state2: each
    D2Q9 population is split over its D3Q19 group in proportion to the
    weights, each D2Q5 one over its D3Q7 group likewise (g_z = 0)."""
    W3 = np.array([1 / 3] + [1 / 18] * 4 + [1 / 36] * 4 + [1 / 18] * 2 + [1 / 36] * 8)
    WG = np.array([0.0] + [1 / 6] * 6)
    d2q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    d2q5 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)]
    ny, nx = state2.shape[1:]
    out = np.zeros((NPLANES, nz, ny, nx))
    for q, (ex, ey) in enumerate(d2q9):
        grp = [r for r in range(NF) if EF[r, 0] == ex and EF[r, 1] == ey]
        wsum = sum(W3[r] for r in grp)
        for r in grp:
            out[r] = state2[q] * (W3[r] / wsum)
    for comp in range(2):
        for q, (ex, ey) in enumerate(d2q5):
            grp = [r for r in range(NG) if EG[r, 0] == ex and EG[r, 1] == ey]
            wsum = sum(WG[r] for r in grp)
            for r in grp:
                out[NF + comp * NG + r] = state2[9 + 5 * comp + q] * (WG[r] / wsum)
    return out


def b0_of(ha: float, tau_f: float, tau_m: float, a: float, rho: float = 1.0) -> float:
    """Imposed field for a Hartmann number (Sec. VIII): Ha = B0 a / sqrt(rho nu eta)."""
    nu = (tau_f - 0.5) / 3.0
    eta = (tau_m - 0.5) / 3.0
    return ha * math.sqrt(rho * nu * eta) / a
