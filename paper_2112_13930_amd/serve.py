"""Continuous-batching solve service for channel steady states on one GPU.

Requests (one channel parameter set each) arrive over time.  The scheduler
admits them into a shared batch in arrival order as soon as their state fits
(HBM footprint, slot table and node budget), advances every resident channel
together with the batched persistent kernel, checks the per-channel FP64
residual every `check_every` steps, and retires a request when it converges
(residual < tol), stagnates (no new minimum 1% below the previous one within
`stagnation_checks` checks: a precision floor, or a mode too slow for the
budget), becomes non-finite, or reaches `max_steps` (see :func:`stop_status`).  Admissions and retirements
happen only at check boundaries, so every channel is checked at multiples of
`check_every` steps after its own admission and its result does not depend on
what else is resident.

The scheduler drives an executor with the interface of batch.Batch
(try_admit, retire, step_check, steps_done, fetch); the GPU executor is
:class:`GpuExecutor`.
"""
from __future__ import annotations

import math
import statistics
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

CONVERGED, STAGNATED, UNSTABLE, MAX_STEPS = "converged", "stagnated", "unstable", "max_steps"


@dataclass
class Request:
    rid: int
    params: object           # LksParams (or anything the executor accepts)
    arrival: float = 0.0     # seconds after the service starts
    status: str = "pending"
    steps: int = 0
    residual: float = math.nan
    t_admit: float = math.nan
    t_done: float = math.nan
    slot: int = -1
    result: object = None
    history: list = field(default_factory=list)
    draw: object = None      # the generator's draw the parameters come from

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def stop_status(history, steps, tol, max_steps, stagnation_checks):
    """Stopping decision after a check (None: keep going)."""
    r = history[-1]
    if not math.isfinite(r):
        return UNSTABLE
    if r < tol:
        return CONVERGED
    if steps >= max_steps:
        return MAX_STEPS
    n = stagnation_checks
    if len(history) > n and min(history[-n:]) > 0.99 * min(history[:-n]):
        return STAGNATED
    return None


class Server:
    def __init__(self, executor, tol: float = 1e-8, check_every: int = 200,
                 max_steps: int = 2_000_000, stagnation_checks: int = 20,
                 keep_result: bool = False, clock=time.perf_counter, sleep=time.sleep):
        if check_every < 2:
            raise ValueError("check_every must be >= 2")
        self.ex = executor
        self.tol = tol
        self.K = check_every
        self.max_steps = max_steps
        self.stag = stagnation_checks
        self.keep_result = keep_result
        self.clock = clock
        self.sleep = sleep
        self.queue: deque[Request] = deque()
        self.active: dict[int, Request] = {}
        self.done: list[Request] = []

    def submit(self, req: Request):
        self.queue.append(req)

    def _admit(self, now: float):
        # FIFO: the head of the queue blocks later arrivals (no overtaking)
        while self.queue and self.queue[0].arrival <= now:
            req = self.queue[0]
            slot = self.ex.try_admit(req.params)
            if slot is None:
                break
            self.queue.popleft()
            req.slot = slot
            req.t_admit = now
            req.status = "running"
            self.active[slot] = req

    def _retire(self, req: Request, status: str, now: float):
        if self.keep_result:
            req.result = self.ex.fetch(req.slot)
        self.ex.retire(req.slot)
        req.status = status
        req.t_done = now
        del self.active[req.slot]
        self.done.append(req)

    def run(self):
        """Serve until every submitted request is done; returns them."""
        t0 = self.clock()
        while self.queue or self.active:
            now = self.clock() - t0
            self._admit(now)
            if not self.active:
                wait = self.queue[0].arrival - now
                if wait > 0:
                    self.sleep(wait)
                    continue
                raise RuntimeError("a queued request can never be admitted (too large for the pool)")
            res, bad = self.ex.step_check(self.K)
            now = self.clock() - t0
            for slot, req in list(self.active.items()):
                req.steps = self.ex.steps_done(slot)
                r = math.nan if bad[slot] else float(res[slot])
                req.residual = r
                req.history.append(r)
                st = stop_status(req.history, req.steps, self.tol, self.max_steps, self.stag)
                if st is not None:
                    self._retire(req, st, now)
        return sorted(self.done, key=lambda q: q.rid)


class GpuExecutor:
    """The batched HIP path behind the scheduler's executor interface."""

    def __init__(self, precision: str = "fp32", max_channels: int = 256,
                 max_nodes: int = 1 << 24, pool_bytes: int | None = None,
                 tiles=None, use_graph: bool = True):
        from .batch import Batch
        self.batch = Batch(precision, max_channels=max_channels, max_nodes=max_nodes,
                           pool_bytes=pool_bytes)
        self.max_channels = max_channels
        self.use_graph = use_graph
        if tiles is not None:
            for k, (w, h) in enumerate(tiles):
                self.batch.set_tile(k, w, h)

    def try_admit(self, params):
        return self.batch.try_admit(params)

    def retire(self, slot):
        self.batch.retire(slot)

    def step_check(self, n):
        return self.batch.step_check(n, graph=self.use_graph)

    def steps_done(self, slot):
        return self.batch.steps_done(slot)

    def fetch(self, slot):
        st = self.batch.save_state(slot)
        m = self.batch.moments(slot)
        return {"state": st.cpu(), "ux": m["ux"].cpu().numpy(), "bx": m["bx"].cpu().numpy()}

    def close(self):
        self.batch.close()


def percentile(vals, q):
    if not vals:
        return math.nan
    return float(np.percentile(np.asarray(vals), q))


def sequential_baseline(requests, precision="fp32", tol=1e-8, check_every=200,
                        max_steps=2_000_000, stagnation_checks=20, graph_steps=32, log=None):
    """The same requests solved one after another by the plain single-channel
    path (arrival order; a solve starts when the GPU is free and the request
    has arrived), with the service's own stopping rule: each check window is
    one run_to_steady call of check_every steps.  Returns per-request
    (status, steps, residual, latency) and the makespan."""
    import torch

    from ._lib import LKS_EUNSTABLE, PRECISIONS
    from .channel import Channel
    out = []
    t0 = time.perf_counter()
    for req in requests:
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        p = req.params
        p.precision = PRECISIONS[precision]
        ch = Channel(params=p, stream=torch.cuda.Stream())
        ch.set_graph(graph_steps)
        hist, status, steps, res = [], None, 0, math.nan
        while status is None:
            rc, steps, res, _ = ch.run_to_steady(tol=0.0, check_every=check_every,
                                                 max_steps=check_every)
            hist.append(math.nan if rc == LKS_EUNSTABLE else res)
            status = stop_status(hist, steps, tol, max_steps, stagnation_checks)
        ch.close()
        t_done = time.perf_counter() - t0
        out.append({"rid": req.rid, "status": status, "steps": steps, "residual": res,
                    "latency": t_done - req.arrival})
        if log and (req.rid % 8 == 7):
            log(f"sequential: {req.rid + 1} requests solved, {t_done:.2f} s")
    return out, time.perf_counter() - t0


def screened_mix(n, seed, b0_max=0.1, **ranges):
    """n channels from the uneven-channel generator (workloads.channel_mix;
    keyword ranges as there), rejecting draws whose imposed field exceeds
    b0_max (the Alfven speed near the lattice limit; equivalently a Hartmann
    layer thinner than one node at tau = 0.8).  Draws are taken in order
    from the seeds seed, seed + 7919, ...  Returns (draws, rejected)."""
    from ._lib import derive, make_params
    from .workloads import channel_mix
    draws, rejected, k = [], 0, 0
    while len(draws) < n:
        for d in channel_mix(n, seed + 7919 * k, **ranges):
            if len(draws) == n:
                break
            p = make_params(d.nx, d.ny, precision="fp32", **d.kwargs())
            if derive(p).b0 > b0_max:
                rejected += 1
                continue
            draws.append(d)
        k += 1
    return draws, rejected


def serve_requests_from_mix(n, seed, nx_range=(4, 32), ny_range=(16, 48), ha_range=(2.0, 30.0),
                            precision="fp32", rate=200.0, c_range=(1e-3, 1.0)):
    """Requests drawn with the uneven-channel generator on a sub-range whose
    steady solves take thousands (not millions) of steps: small channels and
    c <= 1 (no perfectly conducting walls, whose shear-driven case has no
    steady state and whose large-c slow modes take ~c a^2 / eta steps)."""
    from ._lib import derive, make_params
    from .workloads import channel_mix, poisson_arrivals
    draws = channel_mix(4 * n, seed, nx_range=nx_range, ny_range=ny_range, ha_range=ha_range,
                        c_range=c_range, p_zero=0.1, p_inf=0.0)
    arr = poisson_arrivals(rate, n, seed + 1)
    reqs = []
    for d in draws:
        if len(reqs) == n:
            break
        p = make_params(d.nx, d.ny, precision=precision, **d.kwargs())
        if derive(p).b0 > 0.1:
            continue
        reqs.append(Request(rid=len(reqs), params=p, arrival=float(arr[len(reqs)])))
    return reqs


def requests_from_draws(draws, rate, seed, precision="fp32"):
    """Requests for the given channel draws (workloads.ChannelDraw), arriving
    as a Poisson process of the given rate (seeded)."""
    from ._lib import make_params
    from .workloads import poisson_arrivals
    arr = poisson_arrivals(rate, len(draws), seed)
    return [Request(rid=i, params=make_params(d.nx, d.ny, precision=precision, **d.kwargs()),
                    arrival=float(arr[i]), draw=d) for i, d in enumerate(draws)]


# The serving workload: the uneven-channel generator restricted to Ny <= 256
# (its other ranges unchanged: Nx 4-256, Ha 1-200 under the stability
# screen, c = 0 or inf 10% each, else log-uniform in [1e-3, 1e3]).
SERVE_RANGES = dict(ny_range=(32, 256))


def _summary(lat, statuses, span, n):
    return {"makespan_s": round(span, 3), "solves_per_s": round(n / span, 2),
            "p50_latency_s": round(percentile(lat, 50), 4),
            "p99_latency_s": round(percentile(lat, 99), 4), "statuses": statuses}


def serve_benchmark(n_requests=48, rate=200.0, seed=5, precisions=("fp32", "fp16"),
                    baseline_precision="fp32", tol=1e-8, check_every=200, max_steps=200_000,
                    log=None):
    """Serve a fixed set of Poisson-arriving requests with continuous batching
    in each storage precision, then solve the same requests one after another
    with the plain single-channel path in baseline_precision; report solves/s
    and p50/p99 latency for each."""
    import torch
    out = {"requests": n_requests, "arrival_rate_per_s": rate, "tol": tol,
           "check_every": check_every, "max_steps": max_steps,
           "workload": "uneven channels nx 4-32, ny 16-48, Ha 2-30, c = 0 (10%) or "
                       "log-uniform in [1e-3, 1], body or shear driven, link or moment walls; "
                       "Poisson arrivals",
           "batched": {}}
    steps_by = {}
    for prec in precisions:
        reqs = serve_requests_from_mix(n_requests, seed, precision=prec, rate=rate)
        ex = GpuExecutor(prec, max_channels=max(64, n_requests), max_nodes=1 << 22)
        srv = Server(ex, tol=tol, check_every=check_every, max_steps=max_steps)
        for r in reqs:
            srv.submit(r)
        t0 = time.perf_counter()
        done = srv.run()
        torch.cuda.synchronize()
        span = time.perf_counter() - t0
        ex.close()
        statuses = {}
        for r in done:
            statuses[r.status] = statuses.get(r.status, 0) + 1
        out["batched"][prec] = _summary([r.latency for r in done], statuses, span, len(done))
        out["batched"][prec]["mean_steps"] = round(statistics.mean(r.steps for r in done), 1)
        steps_by[prec] = [r.steps for r in done]
        if log:
            log(f"serving: rate {rate}/s, batched {prec}: {span:.2f} s for {len(done)} requests")
    seq_reqs = serve_requests_from_mix(n_requests, seed, precision=baseline_precision, rate=rate)
    seq, seq_span = sequential_baseline(seq_reqs, precision=baseline_precision, tol=tol,
                                        check_every=check_every, max_steps=max_steps, log=log)
    statuses = {}
    for r in seq:
        statuses[r["status"]] = statuses.get(r["status"], 0) + 1
    out["sequential_" + baseline_precision] = _summary([r["latency"] for r in seq], statuses,
                                                       seq_span, len(seq))
    out["speedup_solves_per_s"] = {
        prec: round(seq_span / out["batched"][prec]["makespan_s"], 2) for prec in precisions}
    if baseline_precision in steps_by:
        same = sum(1 for a, b in zip(steps_by[baseline_precision], seq) if a == b["steps"])
        out["same_stop_step_" + baseline_precision] = f"{same}/{len(seq)}"
    return out


def fifo_from_service_times(arrivals, service):
    """Latencies and makespan of one server taking requests in arrival order,
    each for its own service time (a solve alone on the GPU)."""
    t, lat = 0.0, []
    for a, d in zip(arrivals, service):
        t = max(t, a) + d
        lat.append(t - a)
    return lat, t


def serve_workload_benchmark(rates=(50.0, 100.0, 200.0, 500.0, 1000.0, 2000.0),
                             n_requests=256, seed=5, precisions=("fp32", "fp16"),
                             tol=1e-8, check_every=200, max_steps=20_000,
                             stagnation_checks=20, pool_fraction=0.25, log=None):
    """The serving workload (SERVE_RANGES: the uneven-channel generator at
    Ny <= 256, stability screen) at each arrival rate, served with continuous
    batching in each storage precision from a pool capped at pool_fraction of
    the requests' total footprint (so that admission by footprint queues
    them), against the same requests solved one after another by the plain
    FP32 single-channel path with the same stopping rule.  The sequential
    solves are timed once, alone; their latencies at each rate follow from a
    first-come-first-served queue of those service times."""
    import torch

    from ._lib import LKS_EUNSTABLE, PRECISIONS, lib, make_params
    from .batch import Batch
    from .channel import Channel
    draws, rejected = screened_mix(n_requests, seed, **SERVE_RANGES)
    probe = {}
    for prec in precisions:
        b = Batch(prec, max_channels=1, max_nodes=1 << 10, pool_bytes=1 << 20)
        probe[prec] = [b.channel_bytes(make_params(d.nx, d.ny, precision=prec, **d.kwargs()))
                       for d in draws]
        b.close()
    nodes = sum(d.nx * d.ny for d in draws)
    out = {"workload": "uneven-channel generator at Ny <= 256: Nx 4-256, Ny log-uniform "
                       "32-256, Ha log-uniform 1-200 (draws with B0 > 0.1 rejected), c = 0 or "
                       "inf (10% each) else log-uniform 1e-3..1e3, body or shear driven at "
                       "0.05, link or moment walls; Poisson arrivals",
           "requests": n_requests, "rejected_draws": rejected, "nodes_total": nodes,
           "tol": tol, "check_every": check_every, "max_steps": max_steps,
           "stagnation_checks": stagnation_checks, "rates": list(rates), "batched": {}}
    for prec in precisions:
        total = sum(probe[prec])
        cap_channels = max(int(pool_fraction * total), 2 * max(probe[prec]))
        overhead = int(lib().lks_mhd_batch_overhead_bytes(n_requests, nodes))
        pool = overhead + cap_channels
        rows = []
        for rate in rates:
            reqs = requests_from_draws(draws, rate, seed + 1, precision=prec)
            ex = GpuExecutor(prec, max_channels=n_requests, max_nodes=nodes, pool_bytes=pool)
            srv = Server(ex, tol=tol, check_every=check_every, max_steps=max_steps,
                         stagnation_checks=stagnation_checks)
            for r in reqs:
                srv.submit(r)
            t0 = time.perf_counter()
            done = srv.run()
            torch.cuda.synchronize()
            span = time.perf_counter() - t0
            ex.close()
            statuses = {}
            for r in done:
                statuses[r.status] = statuses.get(r.status, 0) + 1
            row = {"rate": rate, **_summary([r.latency for r in done], statuses, span, len(done)),
                   "mean_steps": round(statistics.mean(r.steps for r in done), 1),
                   "max_queue_wait_s": round(max(r.t_admit - r.arrival for r in done), 4)}
            rows.append(row)
            if log:
                log(f"serving workload: {prec} at {rate}/s: {span:.2f} s, {statuses}")
        out["batched"][prec] = {"pool_bytes_for_channels": cap_channels,
                                "requests_footprint_bytes": total, "runs": rows}
    # sequential plain FP32 solves, each timed alone
    service, seq_status, seq_steps = [], {}, []
    for i, d in enumerate(draws):
        p = make_params(d.nx, d.ny, precision="fp32", **d.kwargs())
        p.precision = PRECISIONS["fp32"]
        ch = Channel(params=p, stream=torch.cuda.Stream())
        ch.set_graph(32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, status, steps = [], None, 0
        while status is None:
            rc, steps, res, _ = ch.run_to_steady(tol=0.0, check_every=check_every,
                                                 max_steps=check_every)
            hist.append(math.nan if rc == LKS_EUNSTABLE else res)
            status = stop_status(hist, steps, tol, max_steps, stagnation_checks)
        service.append(time.perf_counter() - t0)
        ch.close()
        seq_status[status] = seq_status.get(status, 0) + 1
        seq_steps.append(steps)
        if log and i % 64 == 63:
            log(f"serving workload: sequential {i + 1} solves, {sum(service):.1f} s")
    seq_rows = []
    for rate in rates:
        arr = [r.arrival for r in requests_from_draws(draws, rate, seed + 1)]
        lat, span = fifo_from_service_times(arr, service)
        seq_rows.append({"rate": rate, **_summary(lat, seq_status, span, len(draws))})
    out["sequential_fp32"] = {"solve_seconds_total": round(sum(service), 3),
                              "mean_steps": round(statistics.mean(seq_steps), 1),
                              "runs": seq_rows}
    out["speedup_solves_per_s"] = {
        prec: [round(b["solves_per_s"] / s["solves_per_s"], 2)
               for b, s in zip(out["batched"][prec]["runs"], seq_rows)] for prec in precisions}
    return out
