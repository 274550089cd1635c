"""Scheduler logic of the solve service, driven by a fake executor on the CPU.

The fake is a test double for scheduling only: it counts steps, reports a
residual that falls geometrically per request, and models the HBM footprint
of each request as a number of bytes; it computes nothing of the method.
"""
import math

import numpy as np
import pytest

from paper_2112_13930_amd.serve import (CONVERGED, MAX_STEPS, STAGNATED, UNSTABLE,
                                        Request, Server)


class FakeExecutor:
    def __init__(self, capacity_bytes, max_channels=8):
        self.capacity = capacity_bytes
        self.max_channels = max_channels
        self.used = 0
        self.slots = {}
        self.admit_log = []
        self.step_calls = 0

    def try_admit(self, params):
        if self.used + params["bytes"] > self.capacity or len(self.slots) >= self.max_channels:
            return None
        s = next(i for i in range(self.max_channels) if i not in self.slots)
        self.slots[s] = {"p": params, "steps": 0}
        self.used += params["bytes"]
        self.admit_log.append(params["name"])
        return s

    def retire(self, slot):
        self.used -= self.slots[slot]["p"]["bytes"]
        del self.slots[slot]

    def step_check(self, n):
        self.step_calls += 1
        res = np.full(self.max_channels, np.nan)
        bad = np.zeros(self.max_channels, dtype=np.int32)
        for s, st in self.slots.items():
            st["steps"] += n
            p = st["p"]
            if p.get("blowup_at") is not None and st["steps"] >= p["blowup_at"]:
                res[s], bad[s] = math.nan, 1
            elif p.get("floor") is not None:
                res[s] = max(p["r0"] * p["rate"] ** (st["steps"] / n), p["floor"])
            else:
                res[s] = p["r0"] * p["rate"] ** (st["steps"] / n)
        return res, bad

    def steps_done(self, slot):
        return self.slots[slot]["steps"]

    def fetch(self, slot):
        return dict(self.slots[slot])


class FakeClock:
    def __init__(self, dt_per_call=0.0):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += d


def req(rid, bytes_, arrival=0.0, r0=1.0, rate=0.5, **kw):
    return Request(rid=rid, arrival=arrival,
                   params={"name": rid, "bytes": bytes_, "r0": r0, "rate": rate, **kw})


def test_all_converge_and_free_memory():
    ex = FakeExecutor(100)
    srv = Server(ex, tol=1e-3, check_every=10)
    for i in range(5):
        srv.submit(req(i, 30, rate=0.5 + 0.05 * i))
    done = srv.run()
    assert [r.status for r in done] == [CONVERGED] * 5
    assert ex.used == 0 and not ex.slots
    # convergence step = first multiple of K where r0 * rate^k < tol
    for r in done:
        rate = 0.5 + 0.05 * r.rid
        k = math.floor(math.log(1e-3) / math.log(rate)) + 1
        assert r.steps == 10 * k


def test_admission_by_footprint_is_fifo():
    ex = FakeExecutor(100)
    srv = Server(ex, tol=1e-3, check_every=10)
    srv.submit(req(0, 60, rate=0.1))   # long-ish
    srv.submit(req(1, 60, rate=0.9))   # cannot fit beside 0
    srv.submit(req(2, 10, rate=0.9))   # fits, but must not overtake 1
    srv.run()
    assert ex.admit_log == [0, 1, 2]


def test_requests_wait_for_arrival():
    clock = FakeClock()
    ex = FakeExecutor(1000)
    srv = Server(ex, tol=1e-3, check_every=10, clock=clock, sleep=clock.sleep)
    srv.submit(req(0, 10, arrival=0.0))
    srv.submit(req(1, 10, arrival=5.0))
    done = srv.run()
    assert done[1].t_admit >= 5.0
    assert all(r.status == CONVERGED for r in done)


def test_failure_of_one_request_does_not_touch_others():
    ex = FakeExecutor(1000)
    srv = Server(ex, tol=1e-4, check_every=10, max_steps=200, stagnation_checks=5)
    srv.submit(req(0, 10, rate=0.5))                      # converges
    srv.submit(req(1, 10, rate=0.5, blowup_at=30))        # non-finite
    srv.submit(req(2, 10, rate=0.5, floor=1e-2))          # stagnates
    srv.submit(req(3, 10, rate=0.97))                     # hits max_steps
    srv.submit(req(4, 10, rate=0.995, floor=None))        # slow but steady: not stagnated
    done = srv.run()
    assert [r.status for r in done] == [CONVERGED, UNSTABLE, STAGNATED, MAX_STEPS, MAX_STEPS]
    assert done[1].steps == 30
    assert done[3].steps == 200
    assert done[0].steps == 10 * (math.floor(math.log(1e-4) / math.log(0.5)) + 1)


def test_oversized_request_is_reported():
    ex = FakeExecutor(10)
    srv = Server(ex, tol=1e-3, check_every=10)
    srv.submit(req(0, 50))
    with pytest.raises(RuntimeError):
        srv.run()


def test_check_every_validated():
    with pytest.raises(ValueError):
        Server(FakeExecutor(1), check_every=1)
