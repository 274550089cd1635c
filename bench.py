#!/usr/bin/env python3
"""Benchmark of the fused lattice-kinetic MHD step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]

A step is one fused FP32 time step (pull stream, Shercliff wall closure,
moments, coupled u/J solve, collide, store) of the shear-driven
Hartmann-Couette channel on a 4096 x 4096 grid: upper wall moving at 0.05,
Ha = 50, wall conductance ratio 1 on both walls, link-based closures,
tau_f = 0.7, tau_m = 0.9.  Inputs are synthetic (the channel starts at rest)
and resident in HBM before the timed region.  The K timed steps are bracketed
by device synchronisation; the value is nodes x K / wall time in MLUPS.

Printed as one JSON line with, besides the contract fields:
  roofline      algorithmic HBM bytes of the step kernel (152 B per node in
                FP32) over its average duration from HIP events on the stream
                it runs on, against 8 TB/s; traffic from the committed
                rocprofv3 counter summary when the kernel source is unchanged.
  cpu_baseline  the FP64 CPU oracle timed on the host cores over a bounded
                sample of the same grid.
  extras        the 30-case sweep (Ha x c x closure); binary16-storage (FP64
                and FP32 arithmetic) and FP64 rates with every reduced mode's
                error against the FP64 oracle on the 512 x 512 precision
                case; the batched launch over 256 uneven channels (FP32
                against sequential single-channel launches, and binary16);
                the continuous-batching solve service (FP32 and binary16)
                against sequential plain FP32 solves at six arrival rates;
                the headline step on a developed (random) state; the 3D
                channel (D3Q19 + D3Q7 field) on 256^3 and the duct with
                Shercliff side walls; the 2D lid-driven enclosure; link walls at
                cut distances q != 1/2; the two-relaxation-time
                collision's rates beside BGK's.
  --only LEG    run one of the extra legs alone and print it (development).

Profiling helpers (used to write profiles/*):
  --profile-run     only warm-up + timed steps of the headline, plus a copy of
                    known size for counter scaling (for rocprofv3 runs)
  --summarize DIR   turn rocprofv3 outputs into profiles/ summaries
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MHD MLUPS + % HBM roofline; batched solves/s and p99 latency vs plain"
PEAK_HBM_GBS = 8000.0
HEADLINE = dict(nx=4096, ny=4096, bc="link", precision="fp32", tau_f=0.7, tau_m=0.9,
                ha=50.0, c_lower=1.0, c_upper=1.0, u_upper=0.05)
PROFILE_DIR = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILE_DIR, "fp32_step_4096_traffic.json")
COPY_REF_BYTES = 1 << 30


def kernel_source_hash() -> str:
    """Hash of every source the FP32 step kernel is compiled from."""
    h = hashlib.sha256()
    for f in ("lks_sr.hpp", "lks_node.hpp", "lks_common.hpp", "lks_aux.hpp", "lks_single.hip"):
        with open(os.path.join(ROOT, "paper_2112_13930_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def time_channel(torch, Channel, kw, steps, warmup, shape=None, channel=None):
    """(wall seconds for `steps`, event seconds per step, channel); an open
    `channel` is timed as it is instead of a new one made from `kw`."""
    ch = Channel(**kw) if channel is None else channel
    if shape is not None:
        ch.set_launch_shape(shape)
    ch.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(ch.stream)
    ch.step(steps)
    e1.record(ch.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3 / steps, ch


def headline(torch, args):
    from paper_2112_13930_amd.channel import Channel
    wall, per_step, ch = time_channel(torch, Channel, HEADLINE, args.steps, args.warmup)
    nodes = HEADLINE["nx"] * HEADLINE["ny"]
    m = ch.moments()
    torch.cuda.synchronize()
    finite = bool(torch.isfinite(m["ux"]).all().item())
    umax = float(m["ux"].abs().max().item())
    # the weakly compressible scheme's density change (magnetic pressure
    # B_x^2/2 is taken up by the lattice density)
    drho = float((m["rho"] - 1.0).abs().max().item())
    ch.close()
    return {"wall": wall, "per_step": per_step, "nodes": nodes, "finite": finite, "umax": umax,
            "max_abs_drho": drho}


def developed_state_rate(torch, steps=200, warmup=10):
    """The headline step on an x- and y-dependent random state (every value
    away from rest, so no stored value is exact): the rate of a developed
    flow, beside the from-rest rate the workload prescribes."""
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.workloads import random_populations
    out = {}
    s0 = torch.from_numpy(random_populations(4096, 4096, seed=5, b0=0.0023))
    for prec, bpn in (("fp32", 152), ("fp16", 76)):
        ch = Channel(**dict(HEADLINE, precision=prec), stream=torch.cuda.Stream())
        ch.load_state(s0)
        ch.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ch.stream)
        ch.step(steps)
        e1.record(ch.stream)
        torch.cuda.synchronize()
        per_step = e0.elapsed_time(e1) / 1e3 / steps
        ch.close()
        gbs = bpn * 4096 * 4096 / per_step / 1e9
        out[prec] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1), "gbs": round(gbs, 1),
                     "frac_hbm": round(gbs / PEAK_HBM_GBS, 3)}
    return out


def three_d(torch, n=256, steps=200, warmup=10):
    """The three-dimensional channel (x, z periodic, Shercliff walls in y) on
    an n^3 grid with the headline physics (Ha 50, c_w 1, upper wall 0.05,
    link walls, tau_f 0.7, tau_m 0.9): rates from rest and on a developed
    random state, and the FP32 run's error against the 2D oracle (the
    from-rest run is x- and z-invariant, so every node must equal the 2D
    oracle's column)."""
    import numpy as np

    from paper_2112_13930_amd._lib import derive, make_params
    from paper_2112_13930_amd.channel3 import Channel3
    from paper_2112_13930_amd.workloads import random_populations3
    kw = dict(bc="link", tau_f=0.7, tau_m=0.9, ha=50.0, c_lower=1.0, c_upper=1.0, u_upper=0.05)
    out = {"grid": f"{n}x{n}x{n}", "steps": steps,
           "bytes_per_node": {"fp32": 296, "fp64": 592}}

    def rate(ch):
        ch.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ch.stream)
        ch.step(steps)
        e1.record(ch.stream)
        torch.cuda.synchronize()
        return n ** 3 / (e0.elapsed_time(e1) / 1e3 / steps)

    for prec, bpn in (("fp32", 296), ("fp64", 592)):
        ch = Channel3(n, n, n, precision=prec, stream=torch.cuda.Stream(), **kw)
        r0 = rate(ch)
        b0 = derive(make_params(n, n, precision=prec, **kw)).b0
        ch.load_state(torch.from_numpy(random_populations3(n, n, n, seed=1, b0=b0)))
        r1 = rate(ch)
        ch.close()
        out[prec] = {"mlups_from_rest": round(r0 / 1e6, 1),
                     "gbs_from_rest": round(bpn * r0 / 1e9, 1),
                     "frac_hbm_from_rest": round(bpn * r0 / 1e9 / PEAK_HBM_GBS, 3),
                     "mlups_developed": round(r1 / 1e6, 1),
                     "frac_hbm_developed": round(bpn * r1 / 1e9 / PEAK_HBM_GBS, 3)}
    # the two-relaxation-time collision, FP32, from rest
    ch = Channel3(n, n, n, precision="fp32", collision="trt", stream=torch.cuda.Stream(), **kw)
    r = rate(ch)
    ch.close()
    out["fp32_trt"] = {"mlups_from_rest": round(r / 1e6, 1),
                       "frac_hbm_from_rest": round(296 * r / 1e9 / PEAK_HBM_GBS, 3)}
    # the multiple-relaxation-time collision (default rates), FP32, from rest
    ch = Channel3(n, n, n, precision="fp32", collision="mrt", stream=torch.cuda.Stream(), **kw)
    r = rate(ch)
    ch.close()
    out["fp32_mrt"] = {"mlups_from_rest": round(r / 1e6, 1),
                       "frac_hbm_from_rest": round(296 * r / 1e9 / PEAK_HBM_GBS, 3)}
    # the measured FP32 workload after 1000 steps from rest against the 2D
    # oracle's columns (stored by tests/golden/make_golden.py)
    gold_path = os.path.join(ROOT, "tests", "golden", "couette_256_link_1000.json")
    if n == 256 and os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        ch = Channel3(n, n, n, precision="fp32", stream=torch.cuda.Stream(), **kw)
        ch.step(1000)
        m = ch.moments()
        g = {k: m[k].cpu().numpy() for k in ("ux", "bx")}
        del m
        ch.close()
        errs = {}
        for k in ("ux", "bx"):
            ref = np.broadcast_to(np.asarray(gold[k])[None, :, None], g[k].shape)
            errs[k] = float(np.linalg.norm(g[k] - ref) / np.linalg.norm(ref))
        out["fp32_error_vs_2d_oracle_1000_steps"] = errs
    return out


def duct_3d(torch, n=256, steps=200, warmup=10):
    """The rectangular duct: the 3D channel's Hartmann walls and physics,
    with stationary Shercliff side walls (c = 1) bounding z, on n^3 FP32:
    the rate from rest, and the FP32 run's error against the 3D oracle's
    rows stored by tests/golden/make_golden.py after 1000 steps."""
    import numpy as np

    from paper_2112_13930_amd.channel3 import Channel3
    kw = dict(bc="link", tau_f=0.7, tau_m=0.9, ha=50.0, c_lower=1.0, c_upper=1.0, u_upper=0.05,
              side_walls=True, c_side=1.0)
    ch = Channel3(n, n, n, precision="fp32", stream=torch.cuda.Stream(), **kw)
    ch.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ch.stream)
    ch.step(steps)
    e1.record(ch.stream)
    torch.cuda.synchronize()
    r = n ** 3 / (e0.elapsed_time(e1) / 1e3 / steps)
    ch.close()
    out = {"grid": f"{n}x{n}x{n}", "side_walls": "c = 1 both", "steps": steps,
           "mlups_from_rest": round(r / 1e6, 1),
           "frac_hbm_from_rest": round(296 * r / 1e9 / PEAK_HBM_GBS, 3)}
    gold_path = os.path.join(ROOT, "tests", "golden", "duct_256_link_1000.json")
    if n == 256 and os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        ch = Channel3(n, n, n, precision="fp32", stream=torch.cuda.Stream(), **kw)
        ch.step(1000)
        m = ch.moments()
        g = {k: m[k].cpu().numpy() for k in ("ux", "bx")}
        del m
        ch.close()
        errs = {}
        for k in ("ux", "bx"):
            got = np.stack([g[k][z] for z in gold["layers"]])        # [layer][y][x]
            ref = np.asarray(gold[k])[:, :, None]                    # every x equal
            errs[k] = float(np.linalg.norm(got - ref) / (np.linalg.norm(ref) * math.sqrt(n)))
        out["fp32_error_vs_3d_oracle_1000_steps"] = errs
    return out


def enclosure(torch, steps=200, warmup=20):
    """The lid-driven enclosure (x bounded by Shercliff walls with c = 1,
    the headline's Hartmann walls and physics): FP32 rates on 4096^2 from
    rest, BGK and TRT, and the FP32 run of the 512^2 cavity against the
    oracle's values stored by tests/golden/make_golden.py after 1000 steps."""
    import numpy as np

    from paper_2112_13930_amd.channel import Channel
    out = {}
    for coll in ("bgk", "trt"):
        kw = dict(HEADLINE, x_walls=True, c_x=1.0, collision=coll)
        _, per_step, ch = time_channel(torch, Channel, kw, steps, warmup)
        ch.close()
        gbs = 152 * 4096 * 4096 / per_step / 1e9
        out[f"fp32_4096_{coll}"] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1),
                                    "frac_hbm": round(gbs / PEAK_HBM_GBS, 3)}
    gold_path = os.path.join(ROOT, "tests", "golden", "cavity_512_link_1000.json")
    if os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        sl = slice(*gold["sample"])
        kw = dict(HEADLINE, nx=512, ny=512, x_walls=True, c_x=1.0)
        ch = Channel(**kw, stream=torch.cuda.Stream())
        ch.set_graph(50)
        ch.step(1000)
        m = ch.moments()
        errs = {}
        for k in ("ux", "uy", "bx"):
            got = m[k].cpu().numpy()[sl, sl]
            ref = np.asarray(gold[k])
            errs[k] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        ch.close()
        out["fp32_512_error_vs_oracle_1000_steps"] = errs
    return out


def chang_lundgren_u(xi, ha, c):
    """Chang-Lundgren centreline-normalised velocity u/U_ref at xi = y/a
    (Sec. VIII): (K/Ha)(1 - cosh(Ha xi)/cosh Ha), K = (c+1)/(Ha c + tanh Ha)."""
    import numpy as np
    K = (c + 1.0) / (ha * c + math.tanh(ha))
    return (K / ha) * (1.0 - np.cosh(ha * xi) / math.cosh(ha))


def cut_walls(torch, steps=200, warmup=20):
    """Link-based Hartmann walls at cut distances q != 1/2: the FP32 rate on
    the headline grid (q = 0.3 below, 0.8 above), and steady FP32 Hartmann
    flow (Ha 5, c 0.5, 64 rows) between walls at q = 0.25, 1/2 and 1 against
    the Chang-Lundgren profile with the half-width (ny - 1)/2 + q."""
    import numpy as np

    from paper_2112_13930_amd._lib import derive, make_params
    from paper_2112_13930_amd.channel import Channel
    out = {}
    _, per_step, ch = time_channel(torch, Channel, dict(HEADLINE, q=(0.3, 0.8)), steps, warmup)
    ch.close()
    gbs = 152 * 4096 * 4096 / per_step / 1e9
    out["fp32_4096_q_0.3_0.8"] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1),
                                  "frac_hbm": round(gbs / PEAK_HBM_GBS, 3)}
    ny, ha, c = 64, 5.0, 0.5
    errs = {}
    for q in (0.25, 0.5, 1.0):
        kw = dict(bc="link", precision="fp32", tau_f=0.8, tau_m=0.8, ha=ha, u_max=0.02,
                  c_lower=c, c_upper=c, q=q)
        d = derive(make_params(8, ny, **kw))
        ch = Channel(8, ny, stream=torch.cuda.Stream(), **kw)
        ch.set_graph(50)
        rc, n, res, _ = ch.run_to_steady(tol=1e-10, check_every=1000, max_steps=400_000)
        ux = ch.moments()["ux"].cpu().numpy()[:, 0]
        ch.close()
        xi = (np.arange(ny) + q - d.a) / d.a
        ref = d.a * d.a * d.fx / d.nu * chang_lundgren_u(xi, ha, c)
        errs[f"q={q}"] = {"steps": int(n), "status": int(rc),
                          "u_rel_l2_vs_closed_form": float(np.linalg.norm(ux - ref) / np.linalg.norm(ref))}
    out["fp32_hartmann_64_rows_vs_chang_lundgren"] = errs
    return out


def curved_walls(torch, steps=200, warmup=20):
    """Solid bodies (curved walls): the FP32 rate of the headline channel
    with a disc of radius 256 on its axis (algorithmic bytes 152 per node
    plus the 4-byte node index the kernel reads), and the steady circular
    Couette flow (inner radius 24 turning, outer 48 still, no field) against
    its closed form u_theta = A r + B / r."""
    import numpy as np

    from paper_2112_13930_amd.channel import Channel
    out = {}
    disc = (("disc", 2047.5, 2047.5, 256.0, 0.0, 0.0),)
    _, per_step, ch = time_channel(torch, Channel, dict(HEADLINE, solids=disc), steps, warmup)
    ch.close()
    gbs = 156 * 4096 * 4096 / per_step / 1e9
    out["fp32_4096_disc_r256"] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1),
                                  "gbs": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 3),
                                  "bytes_per_node": 156}
    r1, r2, u0 = 24.0, 48.0, 0.01
    size = 2 * int(r2) + 6
    c = (size - 1) / 2.0
    omega = u0 / r1
    kw = dict(bc="link", precision="fp32", tau_f=0.8, tau_m=0.8, b0=0.0,
              solids=(("bore", c, c, r2, 0.0, 0.0), ("disc", c, c, r1, omega, 0.0)))
    ch = Channel(size, size, stream=torch.cuda.Stream(), **kw)
    ch.set_graph(50)
    rc, n, res, _ = ch.run_to_steady(tol=2e-7, check_every=1000, max_steps=400_000)
    m = {k: v.cpu().numpy() for k, v in ch.moments().items()}
    ch.close()
    y, x = np.mgrid[0:size, 0:size].astype(float)
    dx, dy = x - c, y - c
    r = np.hypot(dx, dy)
    fluid = (r > r1) & (r < r2)
    A = -omega * r1 ** 2 / (r2 ** 2 - r1 ** 2)
    B = omega * r1 ** 2 * r2 ** 2 / (r2 ** 2 - r1 ** 2)
    ut = (-dy * m["ux"] + dx * m["uy"]) / np.where(r > 0, r, 1.0)
    exact = A * r + B / np.where(r > 0, r, 1.0)
    err = float(np.sqrt(((ut - exact)[fluid] ** 2).sum() / (exact[fluid] ** 2).sum()))
    out["fp32_couette_r24_r48"] = {"steps": int(n), "status": int(rc),
                                   "u_theta_rel_l2_vs_closed_form": err}
    return out


def sweep(torch, steps=100, warmup=10):
    """Config sweep: Ha in {10, 50, 100} x c in {0, 1e-2, 1, 1e2, inf} x link/moment."""
    from paper_2112_13930_amd.channel import Channel
    rows = []
    for bc in ("link", "moment"):
        for ha in (10.0, 50.0, 100.0):
            for c in (0.0, 1e-2, 1.0, 1e2, math.inf):
                kw = dict(HEADLINE, bc=bc, ha=ha, c_lower=c, c_upper=c)
                _, per_step, ch = time_channel(torch, Channel, kw, steps, warmup)
                ch.close()
                rows.append({"bc": bc, "ha": ha, "c": "inf" if math.isinf(c) else c,
                             "mlups": round(4096 * 4096 / per_step / 1e6, 1)})
    vals = [r["mlups"] for r in rows]
    return {"steps_each": steps, "cases": len(rows), "mlups_min": min(vals),
            "mlups_median": statistics.median(vals), "mlups_max": max(vals), "rows": rows}


PRECISION_CASE = os.path.join(ROOT, "tests", "golden", "precision_case_512.json")


def other_precisions(torch, steps=200, warmup=20, err_steps=100_000):
    """Rates of the other storage modes on the headline grid, and every
    reduced-precision mode's error against the FP64 oracle on the 512 x 512
    precision case (Ha = 50, c = 0.5) after err_steps steps (oracle columns
    stored by tests/golden/make_golden.py)."""
    import numpy as np

    from paper_2112_13930_amd.channel import Channel
    out = {}
    for prec, bpn, comp in (("fp16", 76, "f32 arithmetic, f64 accumulation"),
                            ("fp16_f64", 76, "f64"), ("fp64", 304, "f64")):
        _, per_step, ch = time_channel(torch, Channel, dict(HEADLINE, precision=prec), steps, warmup)
        ch.close()
        gbs = bpn * 4096 * 4096 / per_step / 1e9
        out[prec] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1), "gbs": round(gbs, 1),
                     "frac_hbm": round(gbs / PEAK_HBM_GBS, 3), "bytes_per_node": bpn,
                     "compute": comp}
    if os.path.exists(PRECISION_CASE):
        gold = json.load(open(PRECISION_CASE))
        gp = gold["params"]
        kw = dict(bc="link", tau_f=gp["tau_f"], tau_m=gp["tau_m"], ha=gp["ha"],
                  c_lower=gp["c"], c_upper=gp["c"], u_max=gp["u_max"])
        ru = np.asarray(gold[f"ux_{err_steps}"])[:, None]
        rb = np.asarray(gold[f"bx_{err_steps}"])[:, None]
        errs = {}
        for prec in ("fp32", "fp16", "fp16_f64"):
            ch = Channel(512, 512, precision=prec, stream=torch.cuda.Stream(), **kw)
            ch.set_graph(40)
            ch.step(err_steps)
            m = ch.moments()
            ux = m["ux"].cpu().numpy()
            bx = m["bx"].cpu().numpy()
            ch.close()
            errs[prec] = {"ux": float(np.linalg.norm(ux - ru) / (np.linalg.norm(ru) * math.sqrt(512))),
                          "bx": float(np.linalg.norm(bx - rb) / (np.linalg.norm(rb) * math.sqrt(512)))}
        out["error_vs_fp64_oracle"] = {
            "case": f"512x512 Hartmann channel, link, Ha=50, c=0.5, u_max=0.003, {err_steps} "
                    "steps from rest; relative L2 of u_x and B_x (binary16 modes rebase every "
                    "1000 steps)",
            **errs}
        # binary16 (the default mode: FP32 arithmetic) run to steady state
        # against the oracle's
        ch = Channel(512, 512, precision="fp16", stream=torch.cuda.Stream(), **kw)
        ch.set_graph(40)
        t0 = time.perf_counter()
        rc, steps_done, res, _ = ch.run_to_steady(tol=1e-9, check_every=1000, max_steps=3_000_000)
        dt = time.perf_counter() - t0
        m = ch.moments()
        ux = m["ux"].cpu().numpy()
        bx = m["bx"].cpu().numpy()
        ch.close()
        ru = np.asarray(gold["ux_steady"])[:, None]
        rb = np.asarray(gold["bx_steady"])[:, None]
        out["steady_state_fp16_vs_fp64_oracle"] = {
            "case": "the same channel run to steady state: binary16 through run_to_steady "
                    "(windows of 1000 steps, tol 1e-9, rebase per window) against the oracle's "
                    f"steady state ({gold['steady_steps']} steps, per-step change < 1e-12)",
            "status": int(rc), "steps": int(steps_done), "residual": float(res),
            "seconds": round(dt, 1),
            "ux": float(np.linalg.norm(ux - ru) / (np.linalg.norm(ru) * math.sqrt(512))),
            "bx": float(np.linalg.norm(bx - rb) / (np.linalg.norm(rb) * math.sqrt(512)))}
    return out


def trt_rates(torch, steps=200, warmup=20):
    """The two-relaxation-time collision on the headline grid: rates with
    link-based and moment-based walls in FP32 and binary16 storage (magic
    parameters 3/16 for f and 1/4 for g), beside BGK's."""
    from paper_2112_13930_amd.channel import Channel
    out = {}
    for prec, bpn in (("fp32", 152), ("fp16", 76)):
        for bc in ("link", "moment"):
            for coll in ("bgk", "trt"):
                kw = dict(HEADLINE, precision=prec, bc=bc, collision=coll)
                _, per_step, ch = time_channel(torch, Channel, kw, steps, warmup)
                ch.close()
                gbs = bpn * 4096 * 4096 / per_step / 1e9
                out[f"{prec}_{bc}_{coll}"] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1),
                                              "frac_hbm": round(gbs / PEAK_HBM_GBS, 3)}
    return out


def mrt_rates(torch, steps=200, warmup=20):
    """The multiple-relaxation-time collision (default rates: 1.64 and 1.54
    for f's energy modes, the TRT rates of the magic parameters for the rest)
    on the headline grid, FP32 and binary16 storage, link and moment walls,
    from rest and on a developed random state; and steady FP32 Hartmann flow
    (Ha 5, c 0.5, 64 rows, link walls) against the Chang-Lundgren profile."""
    import numpy as np

    from paper_2112_13930_amd._lib import derive, make_params
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.workloads import random_populations
    out = {}
    s0 = torch.from_numpy(random_populations(4096, 4096, seed=5, b0=0.0023))
    for prec, bpn in (("fp32", 152), ("fp16", 76)):
        for bc in ("link", "moment"):
            kw = dict(HEADLINE, precision=prec, bc=bc, collision="mrt")
            _, per_step, ch = time_channel(torch, Channel, kw, steps, warmup)
            ch.load_state(s0)
            _, per_dev, _ = time_channel(torch, Channel, kw, steps, warmup, channel=ch)
            ch.close()
            gbs = bpn * 4096 * 4096 / per_step / 1e9
            out[f"{prec}_{bc}"] = {"mlups": round(4096 * 4096 / per_step / 1e6, 1),
                                   "frac_hbm": round(gbs / PEAK_HBM_GBS, 3),
                                   "mlups_developed": round(4096 * 4096 / per_dev / 1e6, 1)}
    ny, ha, c = 64, 5.0, 0.5
    kw = dict(bc="link", precision="fp32", tau_f=0.8, tau_m=0.8, ha=ha, u_max=0.02, c_lower=c,
              c_upper=c, collision="mrt")
    d = derive(make_params(8, ny, **kw))
    ch = Channel(8, ny, stream=torch.cuda.Stream(), **kw)
    ch.set_graph(50)
    rc, n, res, _ = ch.run_to_steady(tol=1e-10, check_every=1000, max_steps=400_000)
    ux = ch.moments()["ux"].cpu().numpy()[:, 0]
    ch.close()
    xi = (np.arange(ny) + 0.5 - d.a) / d.a
    ref = d.a * d.a * d.fx / d.nu * chang_lundgren_u(xi, ha, c)
    out["fp32_hartmann_64_rows_vs_chang_lundgren"] = {
        "steps": int(n), "status": int(rc),
        "u_rel_l2_vs_closed_form": float(np.linalg.norm(ux - ref) / np.linalg.norm(ref))}
    return out


def stable_mix(n, seed):
    """Config-4 channel draws with the stability screen (serve.screened_mix
    over the full ranges).  Returns (draws, rejected)."""
    from paper_2112_13930_amd.serve import screened_mix
    return screened_mix(n, seed)


# Tile shape per width class (nx <= 8, 16, 32, 64, 128, 256, above) of the
# batched legs and their profiles: (0, h) = runs of 256 h nodes.  The shapes
# lks_mhd_batch_autotune picked most often on the 256-channel mix (fixed here
# so that the bench line and the profiles time the same launches).
BATCH_TILES = {"fp32": [(0, 2), (0, 1), (0, 1), (0, 1), (0, 1), (0, 1), (0, 1)],
               "fp16": [(0, 2), (0, 1), (0, 1), (0, 1), (0, 4), (0, 4), (0, 1)]}


def set_batch_tiles(b, precision):
    for k, (w, h) in enumerate(BATCH_TILES.get(precision, BATCH_TILES["fp32"])):
        b.set_tile(k, w, h)
    return BATCH_TILES.get(precision, BATCH_TILES["fp32"])


def batched(torch, precision="fp32", steps=1000, warmup=20, seed=2024, sequential=True):
    from paper_2112_13930_amd._lib import STORE_BYTES, make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    draws, rejected = stable_mix(256, seed)
    nodes = sum(d.nx * d.ny for d in draws)
    b = Batch(precision, max_channels=256, max_nodes=nodes + 1024)
    for d in draws:
        b.admit(make_params(d.nx, d.ny, precision=precision, **d.kwargs()))
    tiles = set_batch_tiles(b, precision)
    b.step(warmup, graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(b.stream)
    b.step(steps, graph=True)
    e1.record(b.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = e0.elapsed_time(e1) / 1e3 / steps
    b.close()
    bpn = 2 * 19 * STORE_BYTES[precision]
    gbs = bpn * nodes / per_step / 1e9
    out = {"precision": precision, "channels": len(draws), "rejected_draws": rejected,
           "nodes": nodes, "steps": steps, "ms_per_step": round(per_step * 1e3, 4),
           "mlups": round(nodes / per_step / 1e6, 1), "wall_mlups": round(nodes * steps / wall / 1e6, 1),
           "gbs": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 3), "tiles": tiles}
    if sequential:
        # baseline: the same channels advanced one after another by the plain
        # single-channel path (each its own launches), same step count
        seq_steps = max(10, steps // 10)
        chans = [Channel(d.nx, d.ny, precision=precision, stream=torch.cuda.current_stream(),
                         **d.kwargs()) for d in draws]
        for c in chans:
            c.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in chans:
            c.step(seq_steps)
        torch.cuda.synchronize()
        seq_wall = (time.perf_counter() - t0) / seq_steps
        for c in chans:
            c.close()
        out.update({"sequential_ms_per_step": round(seq_wall * 1e3, 3),
                    "sequential_mlups": round(nodes / seq_wall / 1e6, 1),
                    "speedup_vs_sequential": round(seq_wall / per_step, 2)})
    return out


def serving(torch, rates=(50.0, 100.0, 200.0, 500.0, 1000.0, 2000.0), n_requests=256, seed=5):
    """The continuous-batching service on 256 requests of the Ny <= 256
    serving workload at six arrival rates, FP32 and binary16, from a pool
    capped at a quarter of the requests' footprint, against sequential plain
    FP32 solves (serve.serve_workload_benchmark)."""
    from paper_2112_13930_amd.serve import serve_workload_benchmark
    return serve_workload_benchmark(rates=rates, n_requests=n_requests, seed=seed, log=log)


def profile_run_3d(torch, args):
    """The 3D channel's steps only (256^3, headline physics; storage
    precision --precision, FP32 or FP64; with --duct, Shercliff side walls of
    c = 1 bound z), plus a device copy of known size (counter scale)."""
    from paper_2112_13930_amd.channel3 import Channel3
    a = torch.empty(COPY_REF_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    duct = dict(side_walls=True, c_side=1.0) if args.duct else {}
    ch = Channel3(256, 256, 256, bc="link", precision=args.precision, tau_f=0.7, tau_m=0.9,
                  ha=50.0, c_lower=1.0, c_upper=1.0, u_upper=0.05, stream=torch.cuda.Stream(),
                  **duct)
    ch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(args.steps)
    torch.cuda.synchronize()
    ch.close()
    print(json.dumps({"profile_run_3d": True, "steps": args.steps,
                      "per_step_ms": (time.perf_counter() - t0) / args.steps * 1e3}))


def profile_run_batch(torch, args):
    """The 256-channel batch's steps only, in the storage precision
    --precision (the batched leg's channel mix, launched without a graph so
    that a tracer sees each step), plus a device copy of known size (counter
    scale)."""
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    a = torch.empty(COPY_REF_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    draws, _ = stable_mix(256, 2024)
    nodes = sum(d.nx * d.ny for d in draws)
    bt = Batch(args.precision, max_channels=256, max_nodes=nodes + 1024)
    for d in draws:
        bt.admit(make_params(d.nx, d.ny, precision=args.precision, **d.kwargs()))
    set_batch_tiles(bt, args.precision)
    bt.step(args.warmup, graph=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(args.steps, graph=False)
    torch.cuda.synchronize()
    bt.close()
    print(json.dumps({"profile_run_batch": True, "precision": args.precision,
                      "steps": args.steps, "nodes": nodes,
                      "per_step_ms": (time.perf_counter() - t0) / args.steps * 1e3}))


# The headline channel as the bench legs vary it (--profile-run --variant).
PROFILE_VARIANTS = {
    "headline": {},
    "moment": dict(bc="moment"),
    "trt": dict(collision="trt"),
    "mrt": dict(collision="mrt"),
    "enclosure": dict(x_walls=True, c_x=1.0),
    "cut": dict(q=(0.3, 0.8)),
    "disc": dict(solids=(("disc", 2047.5, 2047.5, 256.0, 0.0, 0.0),)),
}


def profile_run(torch, args):
    """Headline steps only (in the storage precision --precision, from rest or
    on the developed random state with --developed; with --variant, the
    scheme of another bench leg), plus a device copy of known size (counter
    scale)."""
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.workloads import random_populations
    a = torch.empty(COPY_REF_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    kw = dict(HEADLINE, precision=args.precision, **PROFILE_VARIANTS[args.variant])
    ch = Channel(**kw, stream=torch.cuda.Stream())
    if args.developed:
        ch.load_state(torch.from_numpy(random_populations(4096, 4096, seed=5, b0=0.0023)))
    _, per_step, ch = time_channel(torch, Channel, kw, args.steps, args.warmup, channel=ch)
    ch.close()
    print(json.dumps({"profile_run": True, "precision": args.precision, "variant": args.variant,
                      "developed": bool(args.developed), "steps": args.steps,
                      "per_step_ms": per_step * 1e3}))


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same grid
# ---------------------------------------------------------------------------

def cpu_baseline(target_s=15.0):
    import numpy as np

    import oracle
    from oracle import Params
    oracle.build()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    nx = ny = 4096
    p = Params(nx=nx, ny=ny, bc=oracle.LINK, tau_f=0.7, tau_m=0.9, c_lo=1.0, c_hi=1.0,
               u_hi=0.05, b0=0.0)
    from oracle import derive as od
    p.b0 = od.b0_of(50.0, 0.7, 0.9, p.half_width())
    s = oracle.init_state(p)
    scratch = np.empty_like(s)
    t0 = time.perf_counter()
    oracle.run(p, s, 1, nthreads=cores, scratch=scratch)
    one = time.perf_counter() - t0
    n_more = max(0, int(target_s / max(one, 1e-3)) - 1)
    t0 = time.perf_counter()
    oracle.run(p, s, n_more, nthreads=cores, scratch=scratch)
    dt = time.perf_counter() - t0
    steps = n_more + 1
    total = one + dt
    return {"value": round(nx * ny * steps / total / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{nx}x{ny} grid, {steps} FP64 steps of the same channel from rest "
                      f"({total:.1f} s, OpenMP over rows)"}


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------

def _read_csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def summarize(dirs, pattern=r"k_step"):
    """Kernel statistics (--kernel-trace --stats) and counters (--pmc) of the
    kernels whose names match `pattern` ("step") and of the reference copy
    ("copy"), from rocprofv3 output directories."""
    import re
    rx = re.compile(pattern)
    out = {"source_hash": kernel_source_hash(), "kernel_pattern": pattern}
    lines = []

    def kind(name):
        if rx.search(name) and "MODE" not in name:
            return "step"
        if "copy" in name.lower() or "elementwise" in name.lower():
            return "copy"
        return None

    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
            for r in _read_csv(f):
                name = r.get("Name", "")
                k = kind(name)
                if k:
                    lines.append((name[:140], r.get("Calls"), r.get("AverageNs"), r.get("Percentage")))
                if k == "step":
                    out.setdefault("step_avg_ns", float(r["AverageNs"]))
                    out.setdefault("step_calls", int(r["Calls"]))
                    out.setdefault("step_kernel", name[:200])
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            acc = {}
            for i, r in enumerate(_read_csv(f)):
                name = r.get("Kernel_Name", r.get("Kernel-Name", ""))
                cn = r.get("Counter_Name", r.get("Counter-Name", ""))
                val = float(r.get("Counter_Value", r.get("Counter-Value", "nan")))
                k = kind(name)
                if k is None:
                    continue
                # one row per dispatch and counter (summed over dimensions)
                disp = (r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id")
                        or f"row{i}")
                acc.setdefault((k, cn), {}).setdefault(disp, 0.0)
                acc[(k, cn)][disp] += val
            for (k, cn), per in acc.items():
                unit = "kib_per_dispatch" if cn in ("FETCH_SIZE", "WRITE_SIZE") else "per_dispatch"
                # the reference copy is the largest copy dispatch; the step
                # kernels take the median over their dispatches
                agg = max if k == "copy" else statistics.median
                out[f"{k}_{cn}_{unit}"] = agg(per.values())
    return out, lines


def write_summary(dirs, command, pattern=r"k_step", name="fp32_step_4096",
                  algorithmic=152 * 4096 * 4096):
    out, lines = summarize(dirs, pattern)
    fetch_s = out.get("step_FETCH_SIZE_kib_per_dispatch")
    write_s = out.get("step_WRITE_SIZE_kib_per_dispatch")
    fetch_c = out.get("copy_FETCH_SIZE_kib_per_dispatch")
    write_c = out.get("copy_WRITE_SIZE_kib_per_dispatch")
    if fetch_c and write_c:
        # a copy of COPY_REF_BYTES reads and writes that many bytes
        out["fetch_scale"] = fetch_c * 1024 / COPY_REF_BYTES
        out["write_scale"] = write_c * 1024 / COPY_REF_BYTES
    if fetch_s and write_s and "fetch_scale" in out:
        out["step_hbm_bytes_per_dispatch"] = (fetch_s * 1024 / out["fetch_scale"] +
                                              write_s * 1024 / out["write_scale"])
    out["algorithmic_bytes_per_dispatch"] = algorithmic
    out["command"] = command
    os.makedirs(PROFILE_DIR, exist_ok=True)
    if fetch_s or write_s or any(k.startswith("step_SQ_") for k in out):
        with open(os.path.join(PROFILE_DIR, f"{name}_traffic.json"), "w") as fh:
            json.dump(out, fh, indent=1)
    return out, lines


# ---------------------------------------------------------------------------

LEGS = {"developed": developed_state_rate, "sweep": sweep, "precisions": other_precisions,
        "channel_3d": three_d, "duct_3d": duct_3d, "enclosure": enclosure, "trt": trt_rates,
        "mrt": mrt_rates,
        "cut_walls": cut_walls,
        "curved_walls": curved_walls,
        "batched": lambda torch: batched(torch, "fp32"),
        "batched_fp16": lambda torch: batched(torch, "fp16", sequential=False),
        "serving": serving}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="headline only, no extras")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--precision", default="fp32", help="storage precision of --profile-run")
    ap.add_argument("--developed", action="store_true",
                    help="--profile-run on the developed random state instead of from rest")
    ap.add_argument("--variant", default="headline", choices=sorted(PROFILE_VARIANTS),
                    help="--profile-run: the headline channel with this leg's scheme")
    ap.add_argument("--profile-3d", action="store_true", help="3D steps only (profiling)")
    ap.add_argument("--duct", action="store_true", help="--profile-3d: a duct (side walls)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="256-channel batch steps only, in --precision (profiling)")
    ap.add_argument("--only", choices=sorted(LEGS), help="run one extra leg and print it")
    ap.add_argument("--summarize", nargs="*")
    ap.add_argument("--command", default="")
    ap.add_argument("--kernel-pattern", default=r"k_step",
                    help="--summarize: regular expression of the profiled kernel's name")
    ap.add_argument("--profile-name", default="fp32_step_4096",
                    help="--summarize: profiles/<name>_traffic.json is written")
    ap.add_argument("--algorithmic-bytes", type=float, default=152 * 4096 * 4096,
                    help="--summarize: algorithmic HBM bytes of one launch")
    args = ap.parse_args()

    if args.summarize:
        out, lines = write_summary(args.summarize, args.command, args.kernel_pattern,
                                   args.profile_name, args.algorithmic_bytes)
        print(json.dumps(out, indent=1))
        for ln in lines:
            print(ln)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the channel path does not "
              "shard across GPUs.", file=sys.stderr)
        return 2
    if os.environ.get("WORLD_SIZE", "1") not in ("", "1"):
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    from paper_2112_13930_amd import lib
    lib()  # fails loudly if the HIP library is not built

    if args.profile_run:
        profile_run(torch, args)
        return 0
    if args.profile_batch:
        profile_run_batch(torch, args)
        return 0
    if args.profile_3d:
        profile_run_3d(torch, args)
        return 0
    if args.only:
        print(json.dumps({args.only: LEGS[args.only](torch)}), flush=True)
        return 0

    h = headline(torch, args)
    nodes, K = h["nodes"], args.steps
    value = nodes * K / h["wall"] / 1e6
    achieved = 152 * nodes / h["per_step"] / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_hash") == kernel_source_hash() and tr.get("step_hbm_bytes_per_dispatch"):
            traffic = tr["step_hbm_bytes_per_dispatch"]
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(h["wall"] / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (channel started at rest, resident in HBM)",
        "config": {"workload": "hartmann-couette 4096x4096, link-based Shercliff walls, "
                               "Ha=50, c_w=1 both walls, upper wall U=0.05, tau_f=0.7, tau_m=0.9, "
                               "populations stored as binary32 (152 B/node), arithmetic in FP64 "
                               "with stochastic rounding to storage",
                   "nx": 4096, "ny": 4096, "precision": "fp32", "bc": "link", "ha": 50.0,
                   "c_wall": 1.0, "u_wall": 0.05, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_step<float,double,link,step,256,1>",
                     "algorithmic_bytes_per_launch": 152 * nodes,
                     "avg_launch_ms": round(h["per_step"] * 1e3, 4)},
        "finite": h["finite"],
        "max_abs_drho": h["max_abs_drho"],
    }
    if not args.quick:
        extras = {}
        log("developed state ...")
        extras["headline_on_developed_state"] = developed_state_rate(torch)
        log("sweep ...")
        extras["config_sweep_fp32"] = sweep(torch)
        log("precisions ...")
        extras["precisions"] = other_precisions(torch)
        log("3D channel ...")
        extras["channel_3d"] = three_d(torch)
        log("duct ...")
        extras["duct_3d"] = duct_3d(torch)
        log("enclosure ...")
        extras["enclosure"] = enclosure(torch)
        log("cut walls ...")
        extras["cut_walls"] = cut_walls(torch)
        log("curved walls ...")
        extras["curved_walls"] = curved_walls(torch)
        log("TRT collision ...")
        extras["trt_collision"] = trt_rates(torch)
        log("MRT collision ...")
        extras["mrt_collision"] = mrt_rates(torch)
        log("batched ...")
        extras["batched_256_channels"] = batched(torch, "fp32")
        extras["batched_256_channels_fp16"] = batched(torch, "fp16", sequential=False)
        if not args.no_serve:
            log("serving ...")
            try:
                extras["serving"] = serving(torch)
            except Exception as e:  # report, do not hide the headline
                extras["serving"] = {"error": repr(e)}
        line["extras"] = extras
    if not args.no_cpu:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
