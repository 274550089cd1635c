"""Write the stored expected values under tests/golden/ (calls only oracle/).

config1_hartmann_link.json
    The plain body-force Hartmann channel: 8 x 64 nodes, link-based walls,
    tau_f = tau_m = 0.8, Ha = 10, c = 0.1 on both walls, F_x set for
    u_max = 0.05, 20000 steps from rest.  Stores the derived lattice
    parameters and the oracle's u_x and B_x rows after 20000 steps (every
    column is identical, so one column is stored), plus the Chang-Lundgren
    profile at the same rows for reference.

precision_case_512.json
    The binary16 precision case: 512 rows, link-based walls,
    tau_f = tau_m = 0.8, Ha = 50, c = 0.5 on both walls, F_x set for
    u_max = 0.003 (u_max = 0.05 drives the scheme non-finite at this size).
    Stores the oracle's u_x and B_x rows after 20 000 and 100 000 steps and at
    steady state (per-step relative change below 1e-12, checked every 1000
    steps), and the Chang-Lundgren profile at the same rows.

couette_256_link_1000.json
    The shear-driven Hartmann-Couette channel of the benchmark on 256 rows:
    link-based walls, tau_f = 0.7, tau_m = 0.9, Ha = 50, c = 1 on both
    walls, upper wall moving at 0.05, 1000 steps from rest.  Stores the
    oracle's u_x and B_x rows (the runs are x-invariant; the 3D benchmark
    channel is also z-invariant, so each of its nodes must match the row).

duct_256_link_1000.json
    The benchmark's shear-driven flow in a rectangular duct: the same Hartmann
    walls and physics on 256 rows, 256 layers between stationary side walls
    with c = 1, 1000 steps from rest, run by the 3D oracle with nx = 1 (the
    run is x-invariant).  Stores the u_x and B_x rows of the layers
    z = 0, 1, 4, 16, 64 and 128.

cavity_512_link_1000.json
    The lid-driven enclosure: 512 x 512 nodes, link-based Hartmann walls
    (tau_f = 0.7, tau_m = 0.9, Ha = 50, c = 1, upper wall moving at 0.05) and
    stationary x-walls with c = 1, 1000 steps from rest, 2D oracle.  Stores
    u_x, u_y and B_x at the nodes (8 + 16 i, 8 + 16 j).

Run:  python tests/golden/make_golden.py [config1] [precision] [couette256] [duct256] [cavity512]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import analytic, derive  # noqa: E402


def config1():
    p = derive.hartmann_params(8, 64, oracle.LINK, 0.8, 0.8, 10.0, 0.1, 0.05)
    s = oracle.init_state(p)
    oracle.run(p, s, 20000, nthreads=1)
    o = oracle.observe(p, s)
    xi = analytic.node_xi(64, oracle.LINK)
    ua, ba = analytic.chang_lundgren(xi, 10.0, 0.1)
    return {
        "description": "Hartmann channel 8x64, link-based, tau_f=tau_m=0.8, Ha=10, c=0.1, "
                       "u_max=0.05, 20000 steps from rest; oracle FP64 observables (one column)",
        "params": {"nx": 8, "ny": 64, "bc": "link", "tau_f": 0.8, "tau_m": 0.8, "ha": 10.0,
                   "c": 0.1, "u_max": 0.05, "steps": 20000, "a": p.a, "b0": p.b0, "fx": p.fx,
                   "theta": 0.1 * p.a / (0.8 - 0.5)},
        "ux": o["ux"][:, 0].tolist(),
        "bx": o["bx"][:, 0].tolist(),
        "rho": o["rho"][:, 0].tolist(),
        "chang_lundgren_u_star": ua.tolist(),
        "chang_lundgren_b_star": ba.tolist(),
        "u_ref": derive.u_ref_hartmann(p.fx, 0.8, p.a),
        "b_ref": derive.b_ref_hartmann(p.fx, 0.8, 0.8, p.a),
    }


def precision_case(nthreads=8):
    from oracle import steady
    p = derive.hartmann_params(1, 512, oracle.LINK, 0.8, 0.8, 50.0, 0.5, 0.003)
    out = {
        "description": "Hartmann channel, 512 rows, link-based, tau_f=tau_m=0.8, Ha=50, c=0.5, "
                       "u_max=0.003, from rest; oracle FP64 observables (one column)",
        "params": {"ny": 512, "bc": "link", "tau_f": 0.8, "tau_m": 0.8, "ha": 50.0, "c": 0.5,
                   "u_max": 0.003, "a": p.a, "b0": p.b0, "fx": p.fx},
    }
    s = oracle.init_state(p)
    done = 0
    for n in (20000, 100000):
        oracle.run(p, s, n - done, nthreads=nthreads)
        done = n
        o = oracle.observe(p, s)
        out[f"ux_{n}"] = o["ux"][:, 0].tolist()
        out[f"bx_{n}"] = o["bx"][:, 0].tolist()
    _, o, n, r = steady.run_to_steady(p, tol=1e-12, check_every=1000, max_steps=5_000_000,
                                      nthreads=nthreads)
    out["steady_steps"] = n
    out["steady_residual"] = r
    out["ux_steady"] = o["ux"][:, 0].tolist()
    out["bx_steady"] = o["bx"][:, 0].tolist()
    xi = analytic.node_xi(512, oracle.LINK)
    ua, ba = analytic.chang_lundgren(xi, 50.0, 0.5)
    out["chang_lundgren_u_star"] = ua.tolist()
    out["chang_lundgren_b_star"] = ba.tolist()
    out["u_ref"] = derive.u_ref_hartmann(p.fx, 0.8, p.a)
    out["b_ref"] = derive.b_ref_hartmann(p.fx, 0.8, 0.8, p.a)
    return out


def couette256():
    p = derive.couette_params(4, 256, oracle.LINK, 0.7, 0.9, 50.0, 1.0, 1.0, 0.05)
    s = oracle.init_state(p)
    oracle.run(p, s, 1000, nthreads=4)
    o = oracle.observe(p, s)
    return {
        "description": "Hartmann-Couette channel, 256 rows, link-based, tau_f=0.7, tau_m=0.9, "
                       "Ha=50, c=1 both walls, upper wall U=0.05, 1000 steps from rest; oracle "
                       "FP64 observables (one column)",
        "params": {"ny": 256, "bc": "link", "tau_f": 0.7, "tau_m": 0.9, "ha": 50.0, "c": 1.0,
                   "u_upper": 0.05, "steps": 1000, "a": p.a, "b0": p.b0},
        "ux": o["ux"][:, 0].tolist(),
        "bx": o["bx"][:, 0].tolist(),
    }


DUCT_LAYERS = (0, 1, 4, 16, 64, 128)


def duct256(nthreads=8):
    from oracle import d3
    p2 = derive.couette_params(1, 256, oracle.LINK, 0.7, 0.9, 50.0, 1.0, 1.0, 0.05)
    p = d3.Params3(nx=1, ny=256, nz=256, bc=oracle.LINK, tau_f=0.7, tau_m=0.9, b0=p2.b0,
                   c_lo=1.0, c_hi=1.0, u_hi=0.05, a=p2.a, side_walls=True, cs_lo=1.0, cs_hi=1.0)
    s = d3.run(p, d3.init_state(p), 1000, nthreads=nthreads)
    o = d3.observe(p, s)
    return {
        "description": "duct 256 rows x 256 layers, link-based Hartmann walls (tau_f=0.7, "
                       "tau_m=0.9, Ha=50, c=1, upper wall U=0.05) and stationary side walls "
                       "(c=1), 1000 steps from rest; 3D oracle FP64 u_x and B_x rows of the "
                       "listed layers",
        "params": {"ny": 256, "nz": 256, "bc": "link", "tau_f": 0.7, "tau_m": 0.9, "ha": 50.0,
                   "c": 1.0, "c_side": 1.0, "u_upper": 0.05, "steps": 1000, "a": p2.a,
                   "b0": p2.b0},
        "layers": list(DUCT_LAYERS),
        "ux": [o["ux"][z, :, 0].tolist() for z in DUCT_LAYERS],
        "bx": [o["bx"][z, :, 0].tolist() for z in DUCT_LAYERS],
    }


CAVITY_SAMPLE = slice(8, 512, 16)


def cavity512(nthreads=8):
    p = derive.couette_params(512, 512, oracle.LINK, 0.7, 0.9, 50.0, 1.0, 1.0, 0.05)
    p = oracle.Params(**{**p.__dict__, "x_walls": True, "cx_lo": 1.0, "cx_hi": 1.0})
    s = oracle.init_state(p)
    oracle.run(p, s, 1000, nthreads=nthreads)
    o = oracle.observe(p, s)
    return {
        "description": "lid-driven enclosure 512x512, link-based, tau_f=0.7, tau_m=0.9, Ha=50, "
                       "c=1 on all walls, upper wall U=0.05, 1000 steps from rest; oracle FP64 "
                       "u_x, u_y, B_x at rows and columns 8, 24, ..., 504",
        "params": {"nx": 512, "ny": 512, "bc": "link", "tau_f": 0.7, "tau_m": 0.9, "ha": 50.0,
                   "c": 1.0, "c_x": 1.0, "u_upper": 0.05, "steps": 1000, "a": p.a,
                   "b0": p.b0},
        "sample": [CAVITY_SAMPLE.start, CAVITY_SAMPLE.stop, CAVITY_SAMPLE.step],
        **{k: o[k][CAVITY_SAMPLE, CAVITY_SAMPLE].tolist() for k in ("ux", "uy", "bx")},
    }


if __name__ == "__main__":
    which = sys.argv[1:] or ["config1", "precision", "couette256", "duct256", "cavity512"]
    if "config1" in which:
        out = os.path.join(HERE, "config1_hartmann_link.json")
        with open(out, "w") as fh:
            json.dump(config1(), fh, indent=1)
        print("wrote", out)
    if "precision" in which:
        out = os.path.join(HERE, "precision_case_512.json")
        with open(out, "w") as fh:
            json.dump(precision_case(), fh, indent=1)
        print("wrote", out)
    if "couette256" in which:
        out = os.path.join(HERE, "couette_256_link_1000.json")
        data = couette256()
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
        print("wrote", out)
    if "duct256" in which:
        out = os.path.join(HERE, "duct_256_link_1000.json")
        data = duct256()
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
        print("wrote", out)
    if "cavity512" in which:
        out = os.path.join(HERE, "cavity_512_link_1000.json")
        data = cavity512()
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
        print("wrote", out)
