"""Degenerate and ragged sizes against the oracle: one column, two wall rows
(link), three rows (moment, cut-distance walls), an enclosure of two
columns, rows one node longer than a 256-node block, odd widths in binary16
(no two-node vector shape), and the same channels in one batch and as a 3D
channel of one layer.  Tolerances as for the channel: relative L2 against
the FP64 oracle at equal step counts, 1e-12 (FP64), 1e-5 (FP32 storage),
2e-3 (binary16 storage)."""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params
from tests.helpers import TOL, assert_close, field_errors, lib_kwargs, to_numpy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2112_13930_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    return P


BASE = dict(tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5, fy=-1e-5, c_lo=0.3, c_hi=math.inf)
CASES = {
    "1x2_link": dict(nx=1, ny=2, bc=LINK, u_hi=0.03),
    "3x2_link": dict(nx=3, ny=2, bc=LINK, u_lo=-0.02),
    "257x5_link": dict(nx=257, ny=5, bc=LINK, u_hi=0.03),
    "1x3_moment": dict(nx=1, ny=3, bc=MOMENT, u_hi=0.03),
    "5x3_moment": dict(nx=5, ny=3, bc=MOMENT, u_lo=-0.02),
    "2x4_enclosure": dict(nx=2, ny=4, bc=LINK, u_hi=0.03, x_walls=True, cx_lo=0.3,
                          cx_hi=math.inf),
    "7x3_cut": dict(nx=7, ny=3, bc=LINK, q_lo=0.3, q_hi=0.9),
}


NSTREAMS = 16  # random streams averaged in binary16 storage


def params(name):
    return Params(**{**BASE, **CASES[name]})


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_degenerate_sizes_match_oracle(P, name, precision):
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.workloads import random_populations
    p = params(name)
    s0 = random_populations(p.nx, p.ny, seed=71, b0=p.b0)
    ch = Channel(p.nx, p.ny, **lib_kwargs(p, precision))
    if precision in ("fp16", "fp16_f64"):
        # On a grid of a few nodes the noise of binary16's stochastic
        # rounding is of the order of the bar itself in a single run (7x3,
        # cut walls: B_x error median 1.7e-3, maximum 3.2e-3, over 64 random
        # streams).  The rounding is unbiased, so the fields averaged over
        # independent streams (step-counter offsets in multiples of the
        # rebase interval, so that every stream rebases alike) are held to
        # the bar, as the average over a large grid's nodes is in one run.
        runs = []
        for k in range(NSTREAMS):
            ch.load_state(torch.from_numpy(s0), steps=1000 * k)
            ch.step(15)
            runs.append(to_numpy(ch.moments()))
        m = {f: sum(r[f] for r in runs) / NSTREAMS for f in runs[0]}
    else:
        ch.load_state(torch.from_numpy(s0))
        ch.step(15)
        m = to_numpy(ch.moments())
    s = oracle.run(p, s0.copy(), 15)
    keys = ("ux", "bx", "uy", "by", "rho") + (("jz",) if precision == "fp64" else ())
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=keys)
    if precision == "fp64":
        assert np.abs(ch.save_state().cpu().numpy() - s).max() < 1e-14


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_degenerate_channels_in_one_batch_equal_solo_runs(P, precision):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    names = ["1x2_link", "3x2_link", "257x5_link", "1x3_moment", "5x3_moment"]
    b = Batch(precision, max_channels=8, max_nodes=10_000)
    slots = [b.admit(make_params(params(n).nx, params(n).ny, **lib_kwargs(params(n), precision)))
             for n in names]
    b.step(9, graph=True)
    torch.cuda.synchronize()
    for s, n in zip(slots, names):
        p = params(n)
        solo = Channel(p.nx, p.ny, **lib_kwargs(p, precision))
        solo.set_rebase(0)
        solo.step(9)
        assert torch.equal(b.save_state(s).cpu(), solo.save_state().cpu()), n
    b.close()


@pytest.mark.parametrize("name", ["1x2_link", "1x3_moment"])
def test_one_layer_3d_channel_of_degenerate_size_matches_2d_oracle(P, name):
    from oracle import d3
    from paper_2112_13930_amd.channel3 import Channel3
    from paper_2112_13930_amd.workloads import random_populations
    p = params(name)
    s2 = random_populations(p.nx, p.ny, seed=73, b0=p.b0)
    kw = lib_kwargs(p, "fp64")
    ch = Channel3(p.nx, p.ny, 1, **kw)
    ch.load_state(torch.from_numpy(d3.lift_from_2d(s2, 1)))
    ch.step(12)
    g = {k: v.cpu().numpy()[0] for k, v in ch.moments().items()}
    ch.close()
    oracle.run(p, s2, 12)
    o = oracle.observe(p, s2)
    for k in ("ux", "bx"):
        assert np.linalg.norm(g[k] - o[k]) <= 1e-12 * np.linalg.norm(o[k]), k


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_largest_channel_matches_oracle_column(P, precision):
    """The largest channel the library accepts (nx * ny * 19 within 32-bit
    indices: 16384 x 6898, 113 M nodes, 17 GB of FP32 or 34 GB of FP64
    populations), 20 steps of a shear-driven channel from rest: sampled
    columns equal the oracle's x-invariant run; one more row is refused."""
    import ctypes

    from paper_2112_13930_amd._lib import LKS_EINVAL, lib, make_params
    from paper_2112_13930_amd.channel import Channel
    nx = 16384
    ny = ((1 << 31) - 1) // 19 // nx
    kw = dict(bc="link", precision=precision, tau_f=0.7, tau_m=0.9, b0=0.002, c_lower=1.0,
              c_upper=1.0, u_upper=0.05)
    assert lib().lks_mhd_validate(ctypes.byref(make_params(nx, ny + 1, **kw))) == LKS_EINVAL
    ch = Channel(nx, ny, **kw)
    ch.step(20)
    m = ch.moments()
    cols = [0, 1, nx // 2, nx - 1]
    got = {k: m[k][:, cols].cpu().numpy() for k in ("ux", "bx")}
    del m
    ch.close()
    p = Params(nx=4, ny=ny, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.002, c_lo=1.0, c_hi=1.0,
               u_hi=0.05)
    s = oracle.run(p, oracle.init_state(p), 20, nthreads=8)
    o = oracle.observe(p, s)
    for k, g in got.items():
        ref = np.broadcast_to(o[k][:, :1], g.shape)
        assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < TOL[precision], k


def test_empty_batch_steps_and_refills(P):
    """A batch with no channels steps (with and without a graph) as a no-op;
    a channel admitted afterwards, and one admitted after every other was
    retired, each equal their solo runs."""
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    p = params("257x5_link")
    kw = lib_kwargs(p, "fp32")
    b = Batch("fp32", max_channels=4, max_nodes=10_000)
    b.step(3, graph=False)
    b.step(4, graph=True)
    torch.cuda.synchronize()
    s1 = b.admit(make_params(p.nx, p.ny, **kw))
    b.step(6, graph=True)
    torch.cuda.synchronize()
    solo = Channel(p.nx, p.ny, **kw)
    solo.step(6)
    assert torch.equal(b.save_state(s1).cpu(), solo.save_state().cpu())
    b.retire(s1)
    b.step(2, graph=True)
    s2 = b.admit(make_params(p.nx, p.ny, **kw))
    b.step(5, graph=False)
    torch.cuda.synchronize()
    solo = Channel(p.nx, p.ny, **kw)
    solo.step(5)
    assert torch.equal(b.save_state(s2).cpu(), solo.save_state().cpu())
    b.close()


@pytest.mark.parametrize("shape,side", [((1, 2, 3), False), ((3, 3, 2), True), ((257, 4, 2), True)],
                         ids=["1x2x3", "3x3x2_duct", "257x4x2_duct"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_degenerate_3d_sizes_match_oracle(P, shape, side, precision):
    """3D channels and ducts of the fewest rows and layers (two wall rows;
    two layers that are both side walls) and rows one node past a block,
    from a random x-, y- and z-dependent state."""
    from oracle import d3
    from paper_2112_13930_amd.channel3 import Channel3
    from paper_2112_13930_amd.workloads import random_populations3
    nx, ny, nz = shape
    p3 = d3.Params3(nx=nx, ny=ny, nz=nz, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=2e-5,
                    fz=1e-5, c_lo=0.3, c_hi=math.inf, u_hi=0.03, side_walls=side, cs_lo=0.5,
                    cs_hi=math.inf)
    s0 = random_populations3(nx, ny, nz, seed=79, b0=p3.b0)
    ch = Channel3(nx, ny, nz, fz=p3.fz, side_walls=side, c_side=(p3.cs_lo, p3.cs_hi), bc="link",
                  precision=precision, tau_f=0.7, tau_m=0.9, b0=p3.b0, fx=p3.fx,
                  c_lower=p3.c_lo, c_upper=p3.c_hi, u_upper=p3.u_hi)
    ch.load_state(torch.from_numpy(s0))
    ch.step(10)
    g = {k: v.cpu().numpy() for k, v in ch.moments().items()}
    st = ch.save_state().cpu().numpy()
    ch.close()
    s = d3.run(p3, s0.copy(), 10)
    o = d3.observe(p3, s)
    for k in ("ux", "bx", "uz", "bz"):
        scale = np.linalg.norm(o["ux" if k[0] == "u" else "bx"])
        assert np.linalg.norm(g[k] - o[k]) / scale < TOL[precision], k
    if precision == "fp64":
        assert np.abs(st - s).max() < 1e-14
