"""Finite-difference solution of fully developed MHD duct flow (TEST
INFRASTRUCTURE): an independent discretisation of the governing equations
of Sec. II that the lattice-kinetic duct must approach as it is refined.

For a flow along x that does not vary along x, with the imposed field B0
along y and the induced field b(y, z) along x, the momentum and induction
equations reduce to two coupled Poisson problems on the cross-section
(lattice units, rho = mu_m = 1):

    nu  (u_yy + u_zz) + B0 b_y + F = 0
    eta (b_yy + b_zz) + B0 u_y     = 0

with no slip, u = 0, on every wall and the thin-conducting-wall condition of
Sec. III on each wall, c_w a db/dn + b = 0 (n the outward normal, a the
half-width between the Hartmann walls, c_w that wall's conductance ratio;
c_w = 0 gives b = 0, c_w = inf gives db/dn = 0).

Discretisation: cell-centred second-order differences on a uniform grid with
ghost cells for the wall conditions.  With the lattice's walls half-way
between nodes and an odd refinement m, every lattice node is a cell centre of
the grid (cell index m j + (m - 1)/2), so no interpolation enters.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _ghost_factor(c: float, a: float, h: float) -> float:
    """b_ghost = factor * b_inside for c a db/dn + b = 0 at the face between
    them (face value the mean, normal derivative the difference over h)."""
    if math.isinf(c):
        return 1.0
    k = c * a / h
    return (k - 0.5) / (k + 0.5)


def solve(ny: int, nz: int | None, nu: float, eta: float, b0: float, fx: float,
          c_lo: float, c_hi: float, cs_lo: float = 0.0, cs_hi: float = 0.0, m: int = 7):
    """u and b at the lattice nodes of an ny x nz cross-section (walls
    half-way; nz None: no side walls, a channel).  Returns arrays [nz][ny]
    (or [ny] for a channel)."""
    assert m % 2 == 1
    a = ny / 2.0
    My = ny * m
    Mz = 1 if nz is None else nz * m
    h = 1.0 / m
    N = My * Mz
    gy_u = -1.0                      # u = 0 on every wall
    gy_b = (_ghost_factor(c_lo, a, h), _ghost_factor(c_hi, a, h))
    gz_b = (_ghost_factor(cs_lo, a, h), _ghost_factor(cs_hi, a, h))

    def idx(j, k):
        return k * My + j

    rows, cols, vals = [], [], []
    rhs = np.zeros(2 * N)

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    # unknown vector: [u (N), b (N)]
    for k in range(Mz):
        for j in range(My):
            i = idx(j, k)
            for var, coef, gyw, gzw in ((0, nu, (gy_u, gy_u), (gy_u, gy_u)),
                                        (1, eta, gy_b, gz_b)):
                r = var * N + i
                off = var * N
                diag = 0.0
                # d2/dy2
                for dj, side in ((-1, 0), (1, 1)):
                    jj = j + dj
                    if 0 <= jj < My:
                        add(r, off + idx(jj, k), coef / h**2)
                    else:
                        diag += coef * gyw[side] / h**2
                diag -= 2 * coef / h**2
                # d2/dz2 (duct only)
                if nz is not None:
                    for dk, side in ((-1, 0), (1, 1)):
                        kk = k + dk
                        if 0 <= kk < Mz:
                            add(r, off + idx(j, kk), coef / h**2)
                        else:
                            diag += coef * gzw[side] / h**2
                    diag -= 2 * coef / h**2
                add(r, r, diag)
                # coupling B0 d/dy of the other variable
                other = (1 - var) * N
                og = (gy_b if var == 0 else (gy_u, gy_u))
                for dj, side, sgn in ((-1, 0, -1.0), (1, 1, 1.0)):
                    jj = j + dj
                    if 0 <= jj < My:
                        add(r, other + idx(jj, k), sgn * b0 / (2 * h))
                    else:
                        add(r, other + i, sgn * b0 * og[side] / (2 * h))
            rhs[i] = -fx
    A = sp.csr_matrix((vals, (rows, cols)), shape=(2 * N, 2 * N))
    x = spla.spsolve(A.tocsc(), rhs)
    u = x[:N].reshape(Mz, My)
    b = x[N:].reshape(Mz, My)
    sel_y = np.arange(ny) * m + (m - 1) // 2
    if nz is None:
        return u[0, sel_y], b[0, sel_y]
    sel_z = np.arange(nz) * m + (m - 1) // 2
    return u[np.ix_(sel_z, sel_y)], b[np.ix_(sel_z, sel_y)]
