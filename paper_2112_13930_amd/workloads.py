"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
comparisons.  Holds no arithmetic of the method: only random numbers, the
sizes and parameter ranges of the workloads, and arrival times.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Typical magnitudes of the 19 population planes (f_0..f_8, g_0x..g_4x,
# g_0y..g_4y) near rest with unit density and unit imposed field.
_F_BASE = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
_GY_BASE = np.array([1 / 3] + [1 / 6] * 4)


def random_populations(nx: int, ny: int, seed: int, b0: float = 0.05,
                       rel_amp: float = 0.02, bx_amp: float = 0.002) -> np.ndarray:
    """FP64 [19, ny, nx] populations: typical magnitudes with uniform random
    relative perturbations (x- and y-dependent)."""
    rng = np.random.default_rng(seed)
    s = np.empty((19, ny, nx), dtype=np.float64)
    s[:9] = _F_BASE[:, None, None] * (1.0 + rel_amp * rng.uniform(-1, 1, (9, ny, nx)))
    s[9:14] = bx_amp * rng.uniform(-1, 1, (5, ny, nx))
    s[14:] = b0 * _GY_BASE[:, None, None] * (1.0 + rel_amp * rng.uniform(-1, 1, (5, ny, nx)))
    return s


# Typical magnitudes of the 40 raw planes of the three-dimensional channel
# (D3Q19 f, then the seven D3Q7 populations of each field component) near
# rest with unit density and unit imposed field along y.
_F3_BASE = np.array([1 / 3] + [1 / 18] * 4 + [1 / 36] * 4 + [1 / 18] * 2 + [1 / 36] * 8)
_G3_BASE = np.array([0.0] + [1 / 6] * 6)


def random_populations3(nx: int, ny: int, nz: int, seed: int, b0: float = 0.05,
                        rel_amp: float = 0.02, bt_amp: float = 0.002) -> np.ndarray:
    """FP64 [40, nz, ny, nx] populations: typical magnitudes with uniform
    random relative perturbations (x-, y- and z-dependent), random tangential
    field populations (x and z components), the rest populations of the
    field (weight 0) zero."""
    rng = np.random.default_rng(seed)
    s = np.zeros((40, nz, ny, nx), dtype=np.float64)
    shape = (nz, ny, nx)
    s[:19] = _F3_BASE[:, None, None, None] * (1.0 + rel_amp * rng.uniform(-1, 1, (19,) + shape))
    for comp in range(3):
        base = 19 + 7 * comp
        if comp == 1:
            s[base + 1:base + 7] = b0 * _G3_BASE[1:, None, None, None] * (
                1.0 + rel_amp * rng.uniform(-1, 1, (6,) + shape))
        else:
            s[base + 1:base + 7] = bt_amp * rng.uniform(-1, 1, (6,) + shape)
    return s


@dataclass
class ChannelDraw:
    nx: int
    ny: int
    ha: float
    c: float
    drive: str   # "body" (u_max) or "shear" (upper wall moving)
    bc: str      # "link" or "moment"
    tau_f: float = 0.8
    tau_m: float = 0.8
    u: float = 0.05

    def kwargs(self) -> dict:
        kw = dict(bc=self.bc, tau_f=self.tau_f, tau_m=self.tau_m, ha=self.ha,
                  c_lower=self.c, c_upper=self.c)
        if self.drive == "body":
            kw["u_max"] = self.u
        else:
            kw["u_upper"] = self.u
        return kw


def channel_mix(n: int, seed: int, nx_range=(4, 256), ny_range=(32, 2048),
                ha_range=(1.0, 200.0), c_range=(1e-3, 1e3), p_zero=0.1,
                p_inf=0.1) -> list[ChannelDraw]:
    """Independent channels drawn in this order per channel: Nx uniform
    integer in nx_range; Ny = round(exp(U(ln lo, ln hi))); Ha log-uniform;
    c = 0 (p_zero), inf (p_inf), else log-uniform in c_range; drive
    body/shear 50/50; wall treatment link/moment 50/50."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(round(math.exp(rng.uniform(math.log(ny_range[0]), math.log(ny_range[1])))))
        ha = float(math.exp(rng.uniform(math.log(ha_range[0]), math.log(ha_range[1]))))
        r = rng.uniform()
        if r < p_zero:
            c = 0.0
        elif r < p_zero + p_inf:
            c = math.inf
        else:
            c = float(math.exp(rng.uniform(math.log(c_range[0]), math.log(c_range[1]))))
        drive = "body" if rng.uniform() < 0.5 else "shear"
        bc = "link" if rng.uniform() < 0.5 else "moment"
        out.append(ChannelDraw(nx=nx, ny=ny, ha=ha, c=c, drive=drive, bc=bc))
    return out


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
