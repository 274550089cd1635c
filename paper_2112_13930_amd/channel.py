"""One channel on the GPU: a thin owner of device memory around the C ABI.

PyTorch provides the device buffer and the stream; all computation is in
liblks_mhd.so.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (LKS_OK, LksError, LksParams, check, derive, last_error, lib,
                   make_params)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Channel:
    """A periodic-in-x channel between two Shercliff walls.

    Keyword arguments are those of :func:`paper_2112_13930_amd._lib.make_params`
    (bc, precision, tau_f, tau_m, ha or b0, c_lower, c_upper, u_lower, u_upper,
    fx or u_max, fy, rho0), or pass ``params=`` directly.
    """

    def __init__(self, nx: int = 0, ny: int = 0, *, params: LksParams | None = None,
                 device: str | torch.device = "cuda", stream: torch.cuda.Stream | None = None,
                 **kw):
        self.params = params if params is not None else make_params(nx, ny, **kw)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.derived = derive(self.params)
        self.device = torch.device(device)
        nbytes = lib().lks_mhd_state_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LksError(-1, last_error())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # torch allocations are at least 512-byte aligned
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        # the buffer was allocated on torch's current stream; the library
        # initialises it on self.stream
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        with torch.cuda.device(self.device):
            check(lib().lks_mhd_create(ctypes.byref(self.params), _ptr(self._buf), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(self._h)), "lks_mhd_create")

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            # work in flight on self.stream (steps, replayed graphs) still uses
            # the buffer, which returns to torch's allocator after this
            self.stream.synchronize()
            lib().lks_mhd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def steps_done(self) -> int:
        return int(lib().lks_mhd_steps_done(self._h))

    def step(self, n: int = 1):
        check(lib().lks_mhd_step(self._h, int(n)), "lks_mhd_step")

    def set_graph(self, steps_per_graph: int):
        check(lib().lks_mhd_set_graph(self._h, int(steps_per_graph)), "lks_mhd_set_graph")

    def rebase(self):
        """Move each row's x-mean of a binary16 state into its FP32 row
        reference (no-op for FP64/FP32 storage)."""
        check(lib().lks_mhd_rebase(self._h), "lks_mhd_rebase")

    def set_rebase(self, every: int):
        """Rebase binary16 states before steps at multiples of `every` (0: off)."""
        check(lib().lks_mhd_set_rebase(self._h, int(every)), "lks_mhd_set_rebase")

    def set_launch_shape(self, shape: int):
        check(lib().lks_mhd_set_launch_shape(self._h, int(shape)), "lks_mhd_set_launch_shape")

    def run_to_steady(self, tol: float = 1e-8, check_every: int = 100,
                      max_steps: int = 10_000_000, raise_on_error: bool = False):
        """Returns (status, steps_done, residual, flow_rate)."""
        steps = ctypes.c_int64()
        res = ctypes.c_double()
        q = ctypes.c_double()
        rc = lib().lks_mhd_run_to_steady(self._h, float(tol), int(check_every), int(max_steps),
                                         ctypes.byref(steps), ctypes.byref(res), ctypes.byref(q))
        if raise_on_error and rc != LKS_OK:
            raise LksError(rc, last_error())
        return rc, steps.value, res.value, q.value

    def moments(self) -> dict:
        """FP64 device tensors rho, ux, uy, bx, by, jz of shape (ny, nx)."""
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "bx", "by", "jz")}
        self._enter()
        check(lib().lks_mhd_moments_device(self._h, *(_ptr(out[k]) for k in
                                           ("rho", "ux", "uy", "bx", "by", "jz"))),
              "lks_mhd_moments_device")
        self._leave()
        return out

    def moments_host(self) -> dict:
        """The same fields as NumPy arrays through the synchronous host-pointer
        entry point lks_mhd_moments."""
        import numpy as np
        out = {k: np.empty((self.ny, self.nx), dtype=np.float64)
               for k in ("rho", "ux", "uy", "bx", "by", "jz")}
        self._enter()
        check(lib().lks_mhd_moments(self._h, *(out[k].ctypes.data_as(ctypes.c_void_p) for k in
                                    ("rho", "ux", "uy", "bx", "by", "jz"))), "lks_mhd_moments")
        return out

    def save_state(self) -> torch.Tensor:
        out = torch.empty((19, self.ny, self.nx), dtype=torch.float64, device=self.device)
        self._enter()
        check(lib().lks_mhd_save_state(self._h, _ptr(out)), "lks_mhd_save_state")
        self._leave()
        return out

    def load_state(self, pops: torch.Tensor, steps: int = 0):
        t = pops.to(device=self.device, dtype=torch.float64).contiguous()
        assert t.shape == (19, self.ny, self.nx)
        self._enter()
        check(lib().lks_mhd_load_state(self._h, _ptr(t), int(steps)), "lks_mhd_load_state")
        self.stream.synchronize()  # keep t alive until the copy kernel ran

    def synchronize(self):
        self.stream.synchronize()

    # The library works on self.stream; tensors are produced and consumed on
    # torch's current stream.  Order the two around every exchange.
    def _enter(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
