"""Parity of the HIP enclosure (Shercliff walls bounding x as well as y)
with the oracle.  Tolerances as for the channel: relative L2 against the
FP64 oracle at equal step counts, 1e-12 (FP64), 1e-5 (FP32 storage), 2e-3
(binary16 storage)."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, Params, derive
from tests.helpers import TOL, assert_close, field_errors, lib_kwargs, mrt, to_numpy, trt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2112_13930_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    return P


def gpu_channel(p: Params, precision: str, **extra):
    from paper_2112_13930_amd.channel import Channel
    return Channel(p.nx, p.ny, **lib_kwargs(p, precision), **extra)


CASES = [
    # c_lo, c_hi (Hartmann), cx_lo, cx_hi (enclosure), u_lo, u_hi, fx, fy, trt
    (0.0, 0.0, 0.0, 0.0, 0.0, 0.04, 0.0, 0.0, False),
    (0.3, 2.0, 0.5, math.inf, -0.02, 0.03, 1e-5, -1e-5, False),
    (math.inf, 0.1, math.inf, 0.0, 0.0, 0.0, 2e-5, 1e-5, False),
    (1.0, 1.0, 0.2, 3.0, 0.0, 0.05, 0.0, 0.0, True),
    (0.5, math.inf, 1.0, 0.0, 0.0, 0.04, 1e-5, 0.0, "mrt"),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_enclosure_random_state_parity(P, case, precision):
    from paper_2112_13930_amd.workloads import random_populations
    cl, cu, xl, xh, ul, uu, fx, fy, use_trt = case
    p = Params(nx=45, ny=21, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=fy, c_lo=cl,
               c_hi=cu, u_lo=ul, u_hi=uu, x_walls=True, cx_lo=xl, cx_hi=xh)
    if use_trt == "mrt":
        p = mrt(p, (1.2, 1.7, 1.3, 0.9, 1.6))
    elif use_trt:
        p = trt(p)
    s0 = random_populations(p.nx, p.ny, seed=41, b0=p.b0)
    ch = gpu_channel(p, precision)
    ch.load_state(torch.from_numpy(s0))
    ch.step(12)
    m = to_numpy(ch.moments())
    s = oracle.run(p, s0.copy(), 12)
    keys = ("ux", "bx", "uy", "by", "rho") + (("jz",) if precision == "fp64" else ())
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=keys)
    if precision == "fp64":
        assert np.abs(ch.save_state().cpu().numpy() - s).max() < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lid_driven_cavity_from_rest(P, precision):
    p = Params(nx=40, ny=32, bc=LINK, tau_f=0.8, tau_m=0.8, b0=0.01, c_lo=0.5, c_hi=0.5,
               u_hi=0.05, x_walls=True, cx_lo=0.1, cx_hi=0.1)
    ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
    ch.set_graph(50)
    ch.step(3000)
    m = to_numpy(ch.moments())
    s = oracle.run(p, oracle.init_state(p), 3000, nthreads=8)
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision],
                 keys=("ux", "uy", "bx"))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_enclosure_launch_shapes_and_graph_bitwise(P, precision):
    """Every launch shape (including the vector kernels, whose x groups
    contain the walls) gives the same bits, and so do graph replays."""
    from paper_2112_13930_amd.workloads import random_populations
    p = Params(nx=300, ny=37, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=1e-5, c_lo=0.2,
               c_hi=math.inf, u_hi=0.03, x_walls=True, cx_lo=0.4, cx_hi=math.inf)
    s0 = torch.from_numpy(random_populations(300, 37, seed=43))
    ref = None
    for shape in range(7):
        ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
        ch.set_launch_shape(shape)
        ch.load_state(s0)
        ch.step(9)
        out = ch.save_state().cpu()
        if ref is None:
            ref = out
        else:
            assert torch.equal(out, ref), shape
    ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
    ch.set_graph(4)
    ch.load_state(s0)
    ch.step(9)
    assert torch.equal(ch.save_state().cpu(), ref)


def test_enclosure_run_to_steady_matches_oracle_residual(P):
    K = 100
    p = Params(nx=16, ny=16, bc=LINK, tau_f=0.8, tau_m=0.8, b0=0.02, c_lo=1.0, c_hi=1.0,
               u_hi=0.01, x_walls=True, cx_lo=0.5, cx_hi=0.5)
    ch = gpu_channel(p, "fp64")
    rc, steps, res, q = ch.run_to_steady(tol=1e-9, check_every=K, max_steps=200000)
    assert rc == 0 and res < 1e-9 and steps % K == 0
    s = oracle.init_state(p)
    oracle.run(p, s, steps - K)
    o_a = oracle.observe(p, s)
    oracle.run(p, s, K - 1)
    o_b = oracle.observe(p, s)
    r = max(np.linalg.norm(o_b[k] - o_a[k]) / np.linalg.norm(o_b[k]) for k in ("ux", "bx")) / (K - 1)
    assert abs(res - r) < 1e-3 * r, (res, r)


def test_batches_and_3d_reject_enclosures(P):
    from paper_2112_13930_amd._lib import LksError, LksParams3, lib, make_params
    from paper_2112_13930_amd.batch import Batch
    b = Batch("fp32", max_channels=4, max_nodes=10_000)
    with pytest.raises(LksError):
        b.admit(make_params(16, 16, precision="fp32", x_walls=True))
    b.close()
    p3 = LksParams3()
    p3.base = make_params(16, 16, precision="fp32", x_walls=True)
    p3.nz = 4
    assert lib().lks_mhd3_state_bytes(ctypes.byref(p3)) == 0
