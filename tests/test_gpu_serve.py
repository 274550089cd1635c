"""Continuous batching on the GPU: each request's result is the same alone
and in a mix (bitwise: same stop step and same populations), and equals the
plain single-channel path at that step count (binary16 states rebased at the
same steps)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2112_13930_amd as P
    assert torch.cuda.is_available()
    P.lib()
    return P


def serve(reqs, precision):
    from paper_2112_13930_amd.serve import GpuExecutor, Server
    ex = GpuExecutor(precision, max_channels=32, max_nodes=1 << 20)
    srv = Server(ex, tol=1e-7, check_every=100, max_steps=60_000, keep_result=True)
    for r in reqs:
        srv.submit(r)
    done = srv.run()
    ex.close()
    return {r.rid: r for r in done}


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_alone_equals_in_mix(P, precision):
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.serve import serve_requests_from_mix
    mix = serve_requests_from_mix(12, seed=3, nx_range=(4, 24), ny_range=(12, 32),
                                  ha_range=(2.0, 20.0), precision=precision, rate=2000.0)
    mixed = serve(mix, precision)
    for rid in (0, 5, 11):
        alone_req = serve_requests_from_mix(12, seed=3, nx_range=(4, 24), ny_range=(12, 32),
                                            ha_range=(2.0, 20.0), precision=precision,
                                            rate=2000.0)[rid]
        alone_req.arrival = 0.0
        alone = serve([alone_req], precision)[rid]
        a, m = alone, mixed[rid]
        assert a.status == m.status and a.steps == m.steps, (rid, a.status, m.status, a.steps, m.steps)
        assert a.residual == m.residual
        assert torch.equal(a.result["state"], m.result["state"])
        # the plain single-channel path reaches the same populations (binary16
        # states are rebased at the start of every check window)
        ch = Channel(params=alone_req.params)
        ch.set_rebase(100)
        ch.step(a.steps)
        assert torch.equal(ch.save_state().cpu(), a.result["state"])
    assert all(r.status != "unstable" for r in mixed.values()), \
        {r.rid: r.status for r in mixed.values()}


@pytest.mark.parametrize("precision", ["fp32", "fp16_f64"])
def test_trt_and_mrt_requests_alone_equal_in_mix(P, precision):
    """Requests with the TRT and MRT collisions share the service with BGK
    ones: each result is the same alone and in the mix, and (FP32 storage,
    whose state involves no row rebase) equals the plain single-channel
    path."""
    from paper_2112_13930_amd._lib import LKS_BGK, LKS_MRT, LKS_TRT
    from paper_2112_13930_amd.channel import Channel
    from paper_2112_13930_amd.serve import serve_requests_from_mix

    def requests():
        mix = serve_requests_from_mix(9, seed=4, nx_range=(4, 16), ny_range=(12, 24),
                                      ha_range=(2.0, 10.0), precision=precision, rate=2000.0)
        for r in mix:
            r.params.collision = (LKS_BGK, LKS_TRT, LKS_MRT)[r.rid % 3]
        return mix

    mixed = serve(requests(), precision)
    assert all(r.status != "unstable" for r in mixed.values())
    for rid in (1, 2, 4, 8):
        req = requests()[rid]
        req.arrival = 0.0
        alone = serve([req], precision)[rid]
        m = mixed[rid]
        assert alone.status == m.status and alone.steps == m.steps, rid
        assert torch.equal(alone.result["state"], m.result["state"])
        if precision != "fp32":
            continue
        ch = Channel(params=req.params)
        ch.step(m.steps)
        assert torch.equal(ch.save_state().cpu(), m.result["state"])


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_served_results_match_oracle(P, precision):
    """Requests of the serving workload (the uneven-channel generator at
    Ny <= 256: Ha up to 200, c from 0 to infinity) served with continuous
    batching and retired by the service's own rule (converged, stagnated or
    a step budget of 6000): every retired request's u_x and B_x, against the
    FP64 oracle run from rest to that request's step count, within the
    precision's bar (every column against the oracle's: the channels are
    x-invariant).  A request retired as unstable (the distribution holds
    strongly driven channels whose induced field grows without bound) must
    be diverging in the oracle too at that step: non-finite, or a velocity
    above five times the driving one."""
    import numpy as np

    import oracle
    from paper_2112_13930_amd.serve import (SERVE_RANGES, GpuExecutor, Server,
                                            requests_from_draws, screened_mix)
    from tests.helpers import TOL, oracle_params_of_draw, rel_l2
    draws, _ = screened_mix(24, 11, **SERVE_RANGES)
    reqs = requests_from_draws(draws, rate=2000.0, seed=12, precision=precision)
    ex = GpuExecutor(precision, max_channels=32, max_nodes=1 << 21)
    srv = Server(ex, tol=1e-8, check_every=200, max_steps=6000, keep_result=True)
    for r in reqs:
        srv.submit(r)
    done = srv.run()
    ex.close()
    assert len(done) == 24
    for r in done:
        q = oracle_params_of_draw(r.draw)
        st = oracle.init_state(q)
        oracle.run(q, st, r.steps)
        o = oracle.observe(q, st)
        if r.status == "unstable":
            u = np.abs(o["ux"]).max()
            assert not np.isfinite(u) or u > 5 * r.draw.u, (r.rid, r.steps, u, r.draw)
            continue
        for k in ("ux", "bx"):
            ref = np.repeat(o[k], r.draw.nx, axis=1)
            if np.linalg.norm(ref) == 0.0:
                continue
            err = rel_l2(r.result[k], ref)
            assert err <= TOL[precision], (r.rid, r.status, r.steps, k, err, r.draw)
