"""Parity of the HIP two-relaxation-time (TRT) collision with the oracle's.

The even part of f relaxes at tau_f and its odd part at the rate the magic
parameter lambda_f gives; the odd part of g relaxes at tau_m and its even part
at the rate lambda_m gives.  Tolerances as for BGK: relative L2 against the
FP64 oracle at equal step counts, 1e-12 (FP64), 1e-5 (FP32 storage), 2e-3
(binary16 storage).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import LINK, MOMENT, Params, derive
from tests.helpers import TOL, assert_close, field_errors, lib_kwargs, to_numpy, trt

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
    # (bc, c_lo, c_hi, u_lo, u_hi, fx, fy, lambda_f, lambda_m)
    (LINK, 0.0, 0.0, 0.0, 0.0, 1e-4, 0.0, 3 / 16, 1 / 4),
    (LINK, 0.3, 2.0, 0.0, 0.04, 0.0, 0.0, 1 / 4, 1 / 12),
    (LINK, math.inf, 0.1, -0.03, 0.02, 2e-5, -1e-5, 3 / 16, 1.0),
    (MOMENT, 0.0, 0.0, 0.0, 0.0, 1e-4, 0.0, 3 / 16, 1 / 4),
    (MOMENT, 0.3, 2.0, 0.0, 0.04, 0.0, 0.0, 1 / 12, 1 / 4),
    (MOMENT, math.inf, 0.1, -0.03, 0.02, 2e-5, -1e-5, 3 / 16, 1 / 6),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_trt_random_state_parity(P, case, precision):
    """x- and y-dependent random state, 12 steps, odd nx (ragged tiles)."""
    from paper_2112_13930_amd.workloads import random_populations
    bc, cl, cu, ul, uu, fx, fy, lf, lm = case
    nx, ny = 77, 21
    p = trt(Params(nx=nx, ny=ny, bc=bc, tau_f=0.7, tau_m=0.9, b0=0.05, fx=fx, fy=fy,
                   c_lo=cl, c_hi=cu, u_lo=ul, u_hi=uu), lf, lm)
    s0 = random_populations(nx, ny, seed=17, b0=0.05)
    ch = gpu_channel(p, precision)
    ch.load_state(torch.from_numpy(s0))
    ch.step(12)
    m = to_numpy(ch.moments())
    s = oracle.run(p, s0.copy(), 12)
    o = oracle.observe(p, s)
    keys = ("ux", "bx", "uy", "by", "rho") + (("jz",) if precision == "fp64" else ())
    assert_close(field_errors(m, o, p.b0), TOL[precision], keys=keys)
    if precision == "fp64":
        assert np.abs(ch.save_state().cpu().numpy() - s).max() < 1e-14
        # and the odd rate matters: BGK from the same state differs
        q = Params(**{**p.__dict__, "collision": oracle.BGK})
        sb = oracle.run(q, s0.copy(), 12)
        assert np.abs(sb - s).max() > 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tau_f", [0.6, 1.2])
def test_trt_poiseuille_exact_on_gpu(P, precision, tau_f):
    """Half-way bounce-back Poiseuille flow at lambda_f = 3/16 is the exact
    parabola with the walls half-way between nodes, at any tau_f."""
    ny, fx = 16, 1e-5
    p = trt(Params(nx=5, ny=ny, bc=LINK, tau_f=tau_f, tau_m=0.9, fx=fx))
    ch = gpu_channel(p, precision, stream=torch.cuda.Stream())
    ch.set_graph(50)
    ch.step(60000)
    ux = to_numpy(ch.moments())["ux"]
    a = ny / 2.0
    y = np.arange(ny) + 0.5 - a
    exact = fx / (2 * derive.nu_of(tau_f)) * (a * a - y * y)
    err = np.abs(ux - exact[:, None]).max() / exact.max()
    assert err < (1e-10 if precision == "fp64" else 1e-5), err


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_trt_launch_shapes_and_graph_bitwise(P, precision):
    from paper_2112_13930_amd.workloads import random_populations
    p = trt(Params(nx=300, ny=37, bc=MOMENT, tau_f=0.7, tau_m=0.9, b0=0.05, fx=1e-5,
                   c_lo=0.2, c_hi=math.inf, u_hi=0.03))
    s0 = torch.from_numpy(random_populations(300, 37, seed=12))
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


def test_trt_run_to_steady_matches_oracle_residual(P):
    """The record and residual steps of run_to_steady collide with TRT too."""
    K = 100
    p = trt(derive.couette_params(4, 24, LINK, 0.8, 0.8, 5.0, 0.0, 0.5, 0.05))
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
    s = oracle.step(p, s)
    assert_close(field_errors(to_numpy(ch.moments()), oracle.observe(p, s), p.b0), 1e-12,
                 keys=("ux", "bx"))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_trt_and_bgk_channels_in_one_batch_equal_solo_runs(P, precision):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    base = [Params(nx=33, ny=20, bc=LINK, tau_f=0.75, tau_m=0.85, b0=0.03, fx=1e-4,
                   c_lo=0.5, c_hi=0.5),
            Params(nx=70, ny=9, bc=MOMENT, tau_f=0.75, tau_m=0.85, b0=0.02, c_lo=0.0,
                   c_hi=math.inf, u_hi=0.05)]
    chans = [base[0], trt(base[0]), base[1], trt(base[1], 1 / 12, 1 / 6)]
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


def test_trt_x_invariant_channel_matches_oracle_column(P):
    """A 1024 x 512 FP32 Hartmann-Couette channel with TRT, 1000 steps from
    rest: every column equals the oracle's (run at nx = 4; the flow is
    x-invariant)."""
    p4 = trt(derive.couette_params(4, 512, MOMENT, 0.7, 0.9, 50.0, 1.0, 1.0, 0.05))
    big = Params(**{**p4.__dict__, "nx": 1024})
    ch = gpu_channel(big, "fp32")
    ch.step(1000)
    m = to_numpy(ch.moments())
    s = oracle.init_state(p4)
    oracle.run(p4, s, 1000, nthreads=8)
    o = oracle.observe(p4, s)
    for k in ("ux", "bx"):
        ref = np.broadcast_to(o[k][:, :1], m[k].shape)
        assert np.linalg.norm(m[k] - ref) / np.linalg.norm(ref) < TOL["fp32"], k
