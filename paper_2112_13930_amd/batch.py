"""Many channels advanced together (thin owner of the device pool).

All computation runs in liblks_mhd.so: one persistent launch per step walks a
packed tile list that covers every active channel.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import PRECISIONS, STORE_BYTES, LksParams, check, lib, make_params


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Batch:
    def __init__(self, precision: str = "fp32", max_channels: int = 256,
                 max_nodes: int = 1 << 26, pool_bytes: int | None = None,
                 device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None):
        self.precision = precision
        self.prec_code = PRECISIONS[precision]
        self.max_channels = int(max_channels)
        self.device = torch.device(device)
        overhead = lib().lks_mhd_batch_overhead_bytes(self.max_channels, int(max_nodes))
        if pool_bytes is None:
            per_node = 2 * 19 * STORE_BYTES[precision] + 16
            pool_bytes = overhead + int(max_nodes) * per_node + self.max_channels * 4 * 256 * 19
            # row references: [ny][20] doubles, or the four tables of binary16
            # computed in FP32 (480 bytes a row); rows of 4 nodes and more
            ref_row = 480 if precision == "fp16" else 160
            pool_bytes += int(max_nodes) * ref_row // 4 + self.max_channels * 4 * ref_row
        self.pool_bytes = int(pool_bytes)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._pool = torch.empty(self.pool_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lks_mhd_batch_create(self.prec_code, self.max_channels, int(max_nodes),
                                             _ptr(self._pool), self.pool_bytes,
                                             ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(self._h)), "lks_mhd_batch_create")
        self.params: dict[int, LksParams] = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.stream.synchronize()
            lib().lks_mhd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def channel_bytes(self, p: LksParams) -> int:
        return int(lib().lks_mhd_batch_channel_bytes(ctypes.byref(p), self.prec_code))

    def admit(self, p: LksParams | None = None, **kw) -> int:
        if p is None:
            p = make_params(kw.pop("nx"), kw.pop("ny"), precision=self.precision, **kw)
        slot = ctypes.c_int32()
        check(lib().lks_mhd_batch_admit(self._h, ctypes.byref(p), ctypes.byref(slot)),
              "lks_mhd_batch_admit")
        self.params[slot.value] = p
        return slot.value

    def try_admit(self, p: LksParams) -> int | None:
        """Admit or return None when the pool, slots or node budget is full."""
        slot = ctypes.c_int32()
        rc = lib().lks_mhd_batch_admit(self._h, ctypes.byref(p), ctypes.byref(slot))
        if rc == -2:
            return None
        check(rc, "lks_mhd_batch_admit")
        self.params[slot.value] = p
        return slot.value

    def retire(self, slot: int):
        check(lib().lks_mhd_batch_retire(self._h, int(slot)), "lks_mhd_batch_retire")
        self.params.pop(slot, None)

    @property
    def active(self) -> int:
        return int(lib().lks_mhd_batch_active(self._h))

    @property
    def nodes(self) -> int:
        return int(lib().lks_mhd_batch_nodes(self._h))

    def steps_done(self, slot: int) -> int:
        return int(lib().lks_mhd_batch_steps_done(self._h, int(slot)))

    def set_tile(self, width_class: int, w: int, h: int):
        """w x h rectangle (w * h = 256) or, with w = 0, 256 * h consecutive nodes."""
        check(lib().lks_mhd_batch_set_tile(self._h, int(width_class), int(w), int(h)),
              "lks_mhd_batch_set_tile")

    def autotune(self, trial_steps: int = 20) -> list:
        out = (ctypes.c_int32 * 14)()
        check(lib().lks_mhd_batch_autotune(self._h, int(trial_steps), out), "lks_mhd_batch_autotune")
        return [(out[2 * k], out[2 * k + 1]) for k in range(7)]

    def step(self, n: int, graph: bool = True):
        check(lib().lks_mhd_batch_step(self._h, int(n), int(bool(graph))), "lks_mhd_batch_step")

    def rebase(self):
        """Row rebase of every active binary16 channel (no-op otherwise)."""
        check(lib().lks_mhd_batch_rebase(self._h), "lks_mhd_batch_rebase")

    def step_check(self, n: int, graph: bool = True):
        """Advance n >= 2 steps; returns (residuals, unstable) per slot."""
        res = np.empty(self.max_channels, dtype=np.float64)
        bad = np.empty(self.max_channels, dtype=np.int32)
        check(lib().lks_mhd_batch_step_check(
            self._h, int(n), int(bool(graph)),
            res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "lks_mhd_batch_step_check")
        return res, bad

    def moments(self, slot: int) -> dict:
        p = self.params[slot]
        cur = torch.cuda.current_stream(self.device)
        out = {k: torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "bx", "by", "jz")}
        self.stream.wait_stream(cur)
        check(lib().lks_mhd_batch_moments(self._h, int(slot), *(_ptr(out[k]) for k in
              ("rho", "ux", "uy", "bx", "by", "jz"))), "lks_mhd_batch_moments")
        cur.wait_stream(self.stream)
        return out

    def save_state(self, slot: int) -> torch.Tensor:
        p = self.params[slot]
        cur = torch.cuda.current_stream(self.device)
        out = torch.empty((19, p.ny, p.nx), dtype=torch.float64, device=self.device)
        self.stream.wait_stream(cur)
        check(lib().lks_mhd_batch_save_state(self._h, int(slot), _ptr(out)),
              "lks_mhd_batch_save_state")
        cur.wait_stream(self.stream)
        return out

    def synchronize(self):
        self.stream.synchronize()
