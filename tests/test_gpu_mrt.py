"""Parity of the HIP multiple-relaxation-time (MRT) collision with the
oracle's.  Tolerances as for the channel: relative L2 against the FP64
oracle at equal step counts, 1e-12 (FP64), 1e-5 (FP32 storage), 2e-3
(binary16 storage)."""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params
from tests.helpers import TOL, assert_close, field_errors, lib_kwargs, mrt, to_numpy

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


OTHER = (1.2, 1.7, 1.3, 0.9, 1.6)
CASES = [
    # bc, c_lo, c_hi, u_lo, u_hi, fx, fy, rates
    (LINK, 0.3, math.inf, 0.0, 0.03, 2e-5, -1e-5, None),
    (MOMENT, 0.0, 2.0, -0.02, 0.0, 1e-5, 0.0, None),
    (LINK, 1.0, 0.0, 0.01, 0.02, 0.0, 1e-5, OTHER),
    (MOMENT, math.inf, 0.5, 0.0, 0.04, 2e-5, 0.0, OTHER),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_mrt_random_state_parity(P, case, precision):
    from paper_2112_13930_amd.workloads import random_populations
    bc, cl, ch, ul, uh, fx, fy, rates = case
    p = mrt(Params(nx=45, ny=19, bc=bc, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=fy, c_lo=cl,
                   c_hi=ch, u_lo=ul, u_hi=uh), rates)
    s0 = random_populations(p.nx, p.ny, seed=61, b0=p.b0)
    ch_ = gpu_channel(p, precision)
    ch_.load_state(torch.from_numpy(s0))
    ch_.step(12)
    m = to_numpy(ch_.moments())
    s = oracle.run(p, s0.copy(), 12)
    keys = ("ux", "bx", "uy", "by", "rho") + (("jz",) if precision == "fp64" else ())
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=keys)
    if precision == "fp64":
        assert np.abs(ch_.save_state().cpu().numpy() - s).max() < 1e-14


@pytest.mark.parametrize("bc", [LINK, MOMENT])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mrt_hartmann_flow_from_rest(P, bc, precision):
    p = mrt(Params(nx=8, ny=40, bc=bc, tau_f=0.8, tau_m=0.8, b0=0.01, fx=2e-6, c_lo=0.5,
                   c_hi=0.5, u_hi=0.01))
    ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
    ch.set_graph(50)
    ch.step(4000)
    m = to_numpy(ch.moments())
    s = oracle.run(p, oracle.init_state(p), 4000, nthreads=8)
    assert_close(field_errors(m, oracle.observe(p, s), p.b0), TOL[precision], keys=("ux", "bx"))


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp64"])
def test_mrt_launch_shapes_and_graph_bitwise(P, precision):
    from paper_2112_13930_amd.workloads import random_populations
    p = mrt(Params(nx=300, ny=37, bc=LINK, tau_f=0.7, tau_m=0.9, b0=0.05, fx=1e-5, c_lo=0.2,
                   c_hi=math.inf, u_hi=0.03), OTHER)
    s0 = torch.from_numpy(random_populations(300, 37, seed=67))
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


def test_mrt_run_to_steady_matches_oracle_residual(P):
    K = 100
    p = mrt(Params(nx=4, ny=24, bc=LINK, tau_f=0.8, tau_m=0.8, b0=0.02, fx=1e-6, c_lo=1.0,
                   c_hi=1.0))
    ch = gpu_channel(p, "fp64")
    rc, steps, res, _ = ch.run_to_steady(tol=1e-9, check_every=K, max_steps=200000)
    assert rc == 0 and res < 1e-9 and steps % K == 0
    s = oracle.init_state(p)
    oracle.run(p, s, steps - K)
    o_a = oracle.observe(p, s)
    oracle.run(p, s, K - 1)
    o_b = oracle.observe(p, s)
    r = max(np.linalg.norm(o_b[k] - o_a[k]) / np.linalg.norm(o_b[k]) for k in ("ux", "bx")) / (K - 1)
    assert abs(res - r) < 1e-3 * r, (res, r)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp64", "fp16_f64"])
def test_mrt_trt_and_bgk_channels_in_one_batch_equal_solo_runs(P, precision):
    """The batched kernel runs MRT channels through its TRT scheme with the
    corrections switched on per channel: every channel of a mixed batch
    equals its solo run bit for bit."""
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    from tests.helpers import trt
    base = [Params(nx=33, ny=20, bc=LINK, tau_f=0.75, tau_m=0.85, b0=0.03, fx=1e-4,
                   c_lo=0.5, c_hi=0.5),
            Params(nx=70, ny=9, bc=MOMENT, tau_f=0.75, tau_m=0.85, b0=0.02, c_lo=0.0,
                   c_hi=math.inf, u_hi=0.05)]
    chans = [mrt(base[0]), base[0], trt(base[0]), mrt(base[1], OTHER), trt(base[1]), base[1],
             mrt(base[0], OTHER)]
    b = Batch(precision, max_channels=8, max_nodes=50_000)
    slots = [b.admit(make_params(c.nx, c.ny, **lib_kwargs(c, precision))) for c in chans]
    b.step(12, graph=True)
    b.step(1, graph=False)
    torch.cuda.synchronize()
    for s, c in zip(slots, chans):
        solo = Channel(c.nx, c.ny, **lib_kwargs(c, precision))
        solo.set_rebase(0)
        solo.step(13)
        assert torch.equal(b.save_state(s).cpu(), solo.save_state().cpu()), c
    b.close()
