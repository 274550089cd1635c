"""Batched persistent launch: every channel of a mixed batch evolves exactly
as it does alone (bitwise, same precision and step count), whatever the
batch composition, admission time, tile shapes or graph replay; FP64 batched
channels match the oracle; per-channel residuals match the single-channel
definition."""
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
    assert torch.cuda.is_available()
    P.lib()
    return P


MIX = [
    # nx, ny, bc, c_lo, c_hi, u_lo, u_hi, fx, b0
    (5, 33, LINK, 0.0, 0.0, 0.0, 0.0, 1e-4, 0.03),
    (12, 17, MOMENT, 0.5, 0.5, 0.0, 0.05, 0.0, 0.02),
    (31, 40, LINK, math.inf, 0.1, 0.0, 0.05, 0.0, 0.04),
    (64, 9, MOMENT, 0.0, math.inf, 0.0, 0.0, 2e-5, 0.01),
    (100, 26, LINK, 1e-3, 1e3, 0.02, 0.0, 1e-5, 0.05),
    (257, 7, MOMENT, 2.0, 0.3, 0.0, 0.03, 1e-5, 0.02),
    (8, 64, MOMENT, math.inf, math.inf, 0.0, 0.0, 1e-4, 0.03),
    (130, 3, MOMENT, 0.1, 0.1, 0.0, 0.0, 1e-5, 0.01),
]


def mix_params(i):
    nx, ny, bc, cl, cu, ul, uu, fx, b0 = MIX[i]
    return Params(nx=nx, ny=ny, bc=bc, tau_f=0.75, tau_m=0.85, b0=b0, fx=fx,
                  c_lo=cl, c_hi=cu, u_lo=ul, u_hi=uu)


def solo_state(p, precision, nsteps):
    from paper_2112_13930_amd.channel import Channel
    ch = Channel(p.nx, p.ny, **lib_kwargs(p, precision))
    ch.set_rebase(0)  # batch steps outside check windows do not rebase
    ch.step(nsteps)
    return ch.save_state().cpu()


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp64", "fp16_f64"])
def test_mixed_batch_equals_solo_runs(P, precision):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    b = Batch(precision, max_channels=16, max_nodes=200_000)
    slots = {}
    # admit half, take an odd number of steps, admit the rest (other parity)
    for i in range(4):
        slots[i] = b.admit(make_params(**{"nx": mix_params(i).nx, "ny": mix_params(i).ny},
                                       **lib_kwargs(mix_params(i), precision)))
    b.step(3, graph=True)
    for i in range(4, len(MIX)):
        slots[i] = b.admit(make_params(mix_params(i).nx, mix_params(i).ny,
                                       **lib_kwargs(mix_params(i), precision)))
    b.step(10, graph=True)
    b.step(1, graph=False)
    torch.cuda.synchronize()
    for i, s in slots.items():
        n = b.steps_done(s)
        assert n == (14 if i < 4 else 11)
        got = b.save_state(s).cpu()
        ref = solo_state(mix_params(i), precision, n)
        assert torch.equal(got, ref), (i, MIX[i])
    # retire two, reuse the space, and check the newcomer and a survivor
    b.retire(slots[1])
    b.retire(slots[5])
    s_new = b.admit(make_params(mix_params(1).nx, mix_params(1).ny, **lib_kwargs(mix_params(1), precision)))
    b.step(6, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(b.save_state(s_new).cpu(), solo_state(mix_params(1), precision, 6))
    assert torch.equal(b.save_state(slots[2]).cpu(), solo_state(mix_params(2), precision, 20))
    b.close()


def test_fp64_batch_matches_oracle(P):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    b = Batch("fp64", max_channels=8, max_nodes=100_000)
    slots = [b.admit(make_params(mix_params(i).nx, mix_params(i).ny, **lib_kwargs(mix_params(i), "fp64")))
             for i in range(len(MIX))]
    b.step(40, graph=True)
    torch.cuda.synchronize()
    for i, s in enumerate(slots):
        p = mix_params(i)
        st = oracle.init_state(p)
        oracle.run(p, st, 40)
        o = oracle.observe(p, st)
        m = to_numpy(b.moments(s))
        errs = field_errors(m, o, p.b0)
        assert_close(errs, TOL["fp64"], keys=("ux", "bx", "uy", "by", "rho", "jz"))
        got = b.save_state(s).cpu().numpy()
        assert np.abs(got - st).max() < 1e-14
    b.close()


def test_batch_residuals_match_single_channel(P):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.channel import Channel
    b = Batch("fp64", max_channels=8, max_nodes=100_000)
    slots = [b.admit(make_params(mix_params(i).nx, mix_params(i).ny, **lib_kwargs(mix_params(i), "fp64")))
             for i in (0, 2, 4)]
    res, bad = b.step_check(300, graph=True)
    for i, s in zip((0, 2, 4), slots):
        ch = Channel(mix_params(i).nx, mix_params(i).ny, **lib_kwargs(mix_params(i), "fp64"))
        rc, steps, r, q = ch.run_to_steady(tol=0.0, check_every=300, max_steps=300)
        assert steps == 300 and bad[s] == 0
        assert abs(res[s] - r) <= 1e-9 * r, (i, res[s], r)
    assert all(math.isnan(res[k]) for k in range(8) if k not in slots)
    b.close()


def test_autotune_and_tile_shapes_keep_results(P):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    outs = []
    for mode in ("default", "tuned", "narrow", "wide-linear"):
        b = Batch("fp32", max_channels=16, max_nodes=300_000)
        slots = [b.admit(make_params(mix_params(i).nx, mix_params(i).ny, **lib_kwargs(mix_params(i), "fp32")))
                 for i in range(len(MIX))]
        if mode == "tuned":
            tiles = b.autotune(trial_steps=4)
            assert all(w * h == 256 or (w == 0 and h in (1, 2, 4)) for w, h in tiles)
        if mode == "narrow":
            for k in range(7):
                b.set_tile(k, 8, 32)
        if mode == "wide-linear":
            for k in range(7):
                b.set_tile(k, 0, 4)
        b.step(12, graph=True)
        n = b.steps_done(slots[0])
        torch.cuda.synchronize()
        outs.append((n, [b.save_state(s).cpu() for s in slots]))
        b.close()
    for i in range(len(MIX)):
        for n, st in outs:
            ref = solo_state(mix_params(i), "fp32", n)
            assert torch.equal(st[i], ref), (i, n)


def test_pool_exhaustion_is_reported(P):
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    b = Batch("fp32", max_channels=4, max_nodes=10_000)
    assert b.try_admit(make_params(50, 50, precision="fp32")) is not None
    assert b.try_admit(make_params(100, 100, precision="fp32")) is None  # node budget
    b.close()


def test_config4_mix_1000_batched_steps_match_oracle(P):
    """The benchmark's 256 uneven channels (seed 2024, stability screen) in
    one FP32 batch for 1000 graph-replayed steps from rest; 16 channels spread
    over the mix against the oracle at the same step count (every column
    against the oracle's column: the draws are x-invariant)."""
    from paper_2112_13930_amd._lib import make_params
    from paper_2112_13930_amd.batch import Batch
    from paper_2112_13930_amd.serve import screened_mix
    from tests.helpers import oracle_params_of_draw
    draws, _ = screened_mix(256, 2024)
    nodes = sum(d.nx * d.ny for d in draws)
    b = Batch("fp32", max_channels=256, max_nodes=nodes + 1024)
    slots = [b.admit(make_params(d.nx, d.ny, precision="fp32", **d.kwargs())) for d in draws]
    b.step(1000, graph=True)
    torch.cuda.synchronize()
    checked = 0
    for i in range(0, 256, 16):
        d = draws[i]
        m = to_numpy(b.moments(slots[i]))
        q = oracle_params_of_draw(d)
        st = oracle.init_state(q)
        oracle.run(q, st, 1000)
        o = {k: np.repeat(v, d.nx, axis=1) for k, v in oracle.observe(q, st).items()}
        errs = field_errors(m, o, q.b0)
        assert_close(errs, TOL["fp32"], keys=("ux", "bx", "uy", "by", "rho"))
        checked += 1
    b.close()
    assert checked == 16
