"""Parity of the HIP link-based Hartmann walls at cut distances q != 1/2
with the oracle's closure.  Tolerances as for the channel: relative L2
against the FP64 oracle at equal step counts, 1e-12 (FP64), 1e-5 (FP32
storage), 2e-3 (binary16 storage)."""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, Params
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
    # q_lo, q_hi, c_lo, c_hi, u_lo, u_hi, fx, trt
    (0.25, 0.75, 0.0, 0.5, 0.0, 0.03, 2e-5, False),
    (1.0, 0.3, math.inf, 2.0, -0.02, 0.0, 1e-5, False),
    (0.6, 0.4, 0.3, 0.0, 0.0, 0.04, 0.0, False),
    (0.2, 1.0, 1.0, math.inf, 0.01, 0.02, 1e-5, True),
    (0.7, 0.25, 0.4, 1.5, 0.0, 0.03, 2e-5, "mrt"),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_cut_walls_random_state_parity(P, case, precision):
    from paper_2112_13930_amd.workloads import random_populations
    ql, qh, cl, ch, ul, uh, fx, use_trt = case
    p = Params(nx=45, ny=19, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=-1e-5, c_lo=cl,
               c_hi=ch, u_lo=ul, u_hi=uh, q_lo=ql, q_hi=qh)
    if use_trt == "mrt":
        p = mrt(p, (1.2, 1.7, 1.3, 0.9, 1.6))
    elif use_trt:
        p = trt(p)
    s0 = random_populations(p.nx, p.ny, seed=47, b0=p.b0)
    ch_ = gpu_channel(p, precision)
    ch_.load_state(torch.from_numpy(s0))
    ch_.step(12)
    m = to_numpy(ch_.moments())
    s = oracle.run(p, s0.copy(), 12)
    keys = ("ux", "bx", "uy", "by", "rho") + (("jz",) if precision == "fp64" else ())
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=keys)
    if precision == "fp64":
        assert np.abs(ch_.save_state().cpu().numpy() - s).max() < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cut_walls_hartmann_flow_from_rest(P, precision):
    p = Params(nx=8, ny=40, bc=LINK, tau_f=0.8, tau_m=0.8, b0=0.01, fx=2e-6, c_lo=0.5,
               c_hi=0.5, q_lo=0.3, q_hi=0.8)
    ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
    ch.set_graph(50)
    ch.step(4000)
    m = to_numpy(ch.moments())
    s = oracle.run(p, oracle.init_state(p), 4000, nthreads=8)
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=("ux", "bx"))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_cut_walls_launch_shapes_and_graph_bitwise(P, precision):
    from paper_2112_13930_amd.workloads import random_populations
    p = Params(nx=300, ny=37, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=1e-5, c_lo=0.2,
               c_hi=math.inf, u_hi=0.03, q_lo=0.35, q_hi=0.9)
    s0 = torch.from_numpy(random_populations(300, 37, seed=53))
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


def test_batches_reject_cut_walls(P):
    from paper_2112_13930_amd._lib import LksError, make_params
    from paper_2112_13930_amd.batch import Batch
    b = Batch("fp32", max_channels=4, max_nodes=10_000)
    with pytest.raises(LksError):
        b.admit(make_params(16, 16, precision="fp32", q=0.3))
    b.close()
