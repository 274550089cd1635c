"""Run-to-steady driver for the oracle (TEST INFRASTRUCTURE).

The paper runs every case "until steady state" without a stopping rule.  The
rule used here: every K steps compare the observables u_x and B_x of step n
with those of step n-1,
    R(n) = max over phi in {u_x, B_x} of ||phi(n) - phi(n-1)||_2 / ||phi(n)||_2,
and stop when R < tol.
"""
from __future__ import annotations

import numpy as np

from . import Params, init_state, observe, run, step


def residual(prev: dict, cur: dict) -> float:
    """max over u_x, B_x of the relative step change; NaN if anything is
    non-finite (NaN is propagated, not dropped by the max)."""
    r = 0.0
    for k in ("ux", "bx"):
        num = float(np.linalg.norm(cur[k] - prev[k]))
        den = max(float(np.linalg.norm(cur[k])), 1e-300)
        q = num / den
        if not np.isfinite(q):
            return float("nan")
        r = max(r, q)
    return r


def run_to_steady(p: Params, tol: float = 1e-11, check_every: int = 500,
                  max_steps: int = 2_000_000, nthreads: int = 1, state=None):
    """Return (state, observables, steps, residual)."""
    s = init_state(p) if state is None else state
    scratch = np.empty_like(s)
    n = 0
    res = float("inf")
    while n < max_steps:
        run(p, s, check_every - 1, nthreads, scratch)
        prev = observe(p, s)
        s = step(p, s, nthreads)
        n += check_every
        cur = observe(p, s)
        res = residual(prev, cur)
        if not np.isfinite(res):
            raise FloatingPointError("oracle run became non-finite")
        if res < tol:
            return s, cur, n, res
    return s, observe(p, s), n, res
