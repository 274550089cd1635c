"""One three-dimensional channel or duct on the GPU (thin owner of device
memory).

x periodic, Shercliff walls at y = 0 and y = ny - 1, z periodic or (a duct)
bounded by Shercliff side walls; every step runs in liblks_mhd.so
(lks_mhd3_*).
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import LKS_OK, LksError, LksParams3, check, last_error, lib, make_params

OBS3 = ("rho", "ux", "uy", "uz", "bx", "by", "bz", "jx", "jy", "jz")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Channel3:
    """Keyword arguments as for Channel (make_params), plus nz and fz; with
    side_walls=True a duct whose side walls have the conductance ratios
    c_side (both) or (c_side_lower, c_side_upper)."""

    def __init__(self, nx: int, ny: int, nz: int, *, fz: float = 0.0, side_walls: bool = False,
                 c_side=0.0, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, **kw):
        self.params = LksParams3()
        self.params.base = make_params(nx, ny, **kw)
        self.params.nz = int(nz)
        self.params.fz = float(fz)
        self.params.side_walls = int(bool(side_walls))
        lo, hi = c_side if isinstance(c_side, (tuple, list)) else (c_side, c_side)
        self.params.c_side_lower, self.params.c_side_upper = float(lo), float(hi)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.device = torch.device(device)
        nbytes = lib().lks_mhd3_state_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LksError(-1, last_error())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        # the buffer was allocated on torch's current stream; the library
        # initialises it on self.stream
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        with torch.cuda.device(self.device):
            check(lib().lks_mhd3_create(ctypes.byref(self.params), _ptr(self._buf), nbytes,
                                        ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(self._h)), "lks_mhd3_create")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            # work in flight on self.stream (steps, replayed graphs) still uses
            # the buffer, which returns to torch's allocator after this
            self.stream.synchronize()
            lib().lks_mhd3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def steps_done(self) -> int:
        return int(lib().lks_mhd3_steps_done(self._h))

    def step(self, n: int = 1):
        check(lib().lks_mhd3_step(self._h, int(n)), "lks_mhd3_step")

    def set_graph(self, steps_per_graph: int):
        check(lib().lks_mhd3_set_graph(self._h, int(steps_per_graph)), "lks_mhd3_set_graph")

    def run_to_steady(self, tol: float = 1e-8, check_every: int = 100,
                      max_steps: int = 10_000_000):
        steps = ctypes.c_int64()
        res = ctypes.c_double()
        q = ctypes.c_double()
        rc = lib().lks_mhd3_run_to_steady(self._h, float(tol), int(check_every), int(max_steps),
                                          ctypes.byref(steps), ctypes.byref(res), ctypes.byref(q))
        return rc, steps.value, res.value, q.value

    def moments(self) -> dict:
        out = {k: torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64,
                              device=self.device) for k in OBS3}
        self._enter()
        check(lib().lks_mhd3_moments(self._h, *(_ptr(out[k]) for k in OBS3)), "lks_mhd3_moments")
        self._leave()
        return out

    def save_state(self) -> torch.Tensor:
        out = torch.empty((40, self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        self._enter()
        check(lib().lks_mhd3_save_state(self._h, _ptr(out)), "lks_mhd3_save_state")
        self._leave()
        return out

    def load_state(self, pops: torch.Tensor, steps: int = 0):
        t = pops.to(device=self.device, dtype=torch.float64).contiguous()
        assert t.shape == (40, self.nz, self.ny, self.nx)
        self._enter()
        check(lib().lks_mhd3_load_state(self._h, _ptr(t), int(steps)), "lks_mhd3_load_state")
        self.stream.synchronize()

    def synchronize(self):
        self.stream.synchronize()

    def _enter(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)


__all__ = ["Channel3", "OBS3", "LKS_OK"]
