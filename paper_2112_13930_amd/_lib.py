"""ctypes binding of liblks_mhd.so (argument marshalling only).

The library is the product: every step of the lattice-kinetic MHD path runs in
its HIP kernels.  If it is not built this module raises on first use; there is
no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblks_mhd.so")

LKS_BC_LINK, LKS_BC_MOMENT = 0, 1
LKS_FP64, LKS_FP32, LKS_FP16_STORE, LKS_FP16_STORE_F64 = 0, 1, 2, 3
LKS_OK, LKS_EINVAL, LKS_ENOMEM, LKS_EDEVICE, LKS_EUNSTABLE, LKS_ENOTCONV = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "LKS_OK", -1: "LKS_EINVAL", -2: "LKS_ENOMEM", -3: "LKS_EDEVICE",
                -4: "LKS_EUNSTABLE", -5: "LKS_ENOTCONV"}
# binary16 storage computed in FP32 with FP64 accumulation ("fp16") or in
# FP64 ("fp16_f64")
PRECISIONS = {"fp64": LKS_FP64, "fp32": LKS_FP32, "fp16": LKS_FP16_STORE,
              "fp16_f64": LKS_FP16_STORE_F64}
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "fp16_f64": 2}
BCS = {"link": LKS_BC_LINK, "moment": LKS_BC_MOMENT}
LKS_BGK, LKS_TRT, LKS_MRT = 0, 1, 2
COLLISIONS = {"bgk": LKS_BGK, "trt": LKS_TRT, "mrt": LKS_MRT}


class LksSolid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("r", ctypes.c_double), ("omega", ctypes.c_double),
                ("u", ctypes.c_double)]


SOLID_KINDS = {"disc": 1, "bore": 2, "below": 3, "above": 4}
MAX_SOLIDS = 4


class LksParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("tau_f", ctypes.c_double), ("tau_m", ctypes.c_double),
        ("ha", ctypes.c_double), ("b0", ctypes.c_double),
        ("c_lower", ctypes.c_double), ("c_upper", ctypes.c_double),
        ("u_lower", ctypes.c_double), ("u_upper", ctypes.c_double),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double),
        ("u_max", ctypes.c_double), ("rho0", ctypes.c_double),
        ("collision", ctypes.c_int32), ("x_walls", ctypes.c_int32),
        ("lambda_f", ctypes.c_double), ("lambda_m", ctypes.c_double),
        ("c_x_lower", ctypes.c_double), ("c_x_upper", ctypes.c_double),
        ("q_lower", ctypes.c_double), ("q_upper", ctypes.c_double),
        ("s_fe", ctypes.c_double), ("s_feps", ctypes.c_double), ("s_fq", ctypes.c_double),
        ("s_me", ctypes.c_double), ("s_md", ctypes.c_double),
        ("nsolids", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("solids", LksSolid * MAX_SOLIDS),
    ]


class LksParams3(ctypes.Structure):
    _fields_ = [("base", LksParams), ("nz", ctypes.c_int32), ("side_walls", ctypes.c_int32),
                ("fz", ctypes.c_double), ("c_side_lower", ctypes.c_double),
                ("c_side_upper", ctypes.c_double)]


class LksDerived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("nu", "eta", "a", "b0", "fx", "fy", "theta_lower", "theta_upper",
                 "phi_lower", "phi_upper", "tau_f_odd", "tau_m_even",
                 "s_fe", "s_feps", "s_fq", "s_me", "s_md")]


class LksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_c = ctypes
_P = ctypes.POINTER(LksParams)
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)

SIGNATURES = {
    "lks_mhd_abi_version": (_c.c_int, []),
    "lks_mhd_last_error": (_c.c_char_p, []),
    "lks_mhd_default_params": (None, [_P, _c.c_int32, _c.c_int32]),
    "lks_mhd_validate": (_c.c_int, [_P]),
    "lks_mhd_derive": (_c.c_int, [_P, ctypes.POINTER(LksDerived)]),
    "lks_mhd_state_bytes": (_c.c_size_t, [_P]),
    "lks_mhd_create": (_c.c_int, [_P, _vp, _c.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lks_mhd_destroy": (_c.c_int, [_vp]),
    "lks_mhd_step": (_c.c_int, [_vp, _c.c_int64]),
    "lks_mhd_set_graph": (_c.c_int, [_vp, _c.c_int32]),
    "lks_mhd_set_launch_shape": (_c.c_int, [_vp, _c.c_int32]),
    "lks_mhd_steps_done": (_c.c_int64, [_vp]),
    "lks_mhd_run_to_steady": (_c.c_int, [_vp, _c.c_double, _c.c_int64, _c.c_int64, _i64p, _dp, _dp]),
    "lks_mhd_moments": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lks_mhd_moments_device": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lks_mhd_save_state": (_c.c_int, [_vp, _vp]),
    "lks_mhd_load_state": (_c.c_int, [_vp, _vp, _c.c_int64]),
    "lks_mhd_rebase": (_c.c_int, [_vp]),
    "lks_mhd_set_rebase": (_c.c_int, [_vp, _c.c_int64]),
    "lks_mhd_bytes_per_node": (_c.c_int, [_c.c_int32]),
    "lks_mhd_advance_noalloc": (_c.c_int, [_P, _vp, _c.c_int64, _c.c_int64, _vp]),
    "lks_round_binary16": (_c.c_int, [_vp, _vp, _vp, _c.c_int64, _vp]),
    "lks_mhd_batch_overhead_bytes": (_c.c_size_t, [_c.c_int32, _c.c_int64]),
    "lks_mhd_batch_create": (_c.c_int, [_c.c_int32, _c.c_int32, _c.c_int64, _vp, _c.c_size_t, _vp,
                                        ctypes.POINTER(_vp)]),
    "lks_mhd_batch_destroy": (_c.c_int, [_vp]),
    "lks_mhd_batch_channel_bytes": (_c.c_size_t, [_P, _c.c_int32]),
    "lks_mhd_batch_admit": (_c.c_int, [_vp, _P, _i32p]),
    "lks_mhd_batch_retire": (_c.c_int, [_vp, _c.c_int32]),
    "lks_mhd_batch_active": (_c.c_int32, [_vp]),
    "lks_mhd_batch_nodes": (_c.c_int64, [_vp]),
    "lks_mhd_batch_set_tile": (_c.c_int, [_vp, _c.c_int32, _c.c_int32, _c.c_int32]),
    "lks_mhd_batch_autotune": (_c.c_int, [_vp, _c.c_int32, _i32p]),
    "lks_mhd_batch_step": (_c.c_int, [_vp, _c.c_int64, _c.c_int32]),
    "lks_mhd_batch_step_check": (_c.c_int, [_vp, _c.c_int64, _c.c_int32, _dp, _i32p]),
    "lks_mhd_batch_rebase": (_c.c_int, [_vp]),
    "lks_mhd_batch_steps_done": (_c.c_int64, [_vp, _c.c_int32]),
    "lks_mhd_batch_moments": (_c.c_int, [_vp, _c.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lks_mhd_batch_save_state": (_c.c_int, [_vp, _c.c_int32, _vp]),
    "lks_mhd3_state_bytes": (_c.c_size_t, [ctypes.POINTER(LksParams3)]),
    "lks_mhd3_bytes_per_node": (_c.c_int, [_c.c_int32]),
    "lks_mhd3_create": (_c.c_int, [ctypes.POINTER(LksParams3), _vp, _c.c_size_t, _vp,
                                   ctypes.POINTER(_vp)]),
    "lks_mhd3_destroy": (_c.c_int, [_vp]),
    "lks_mhd3_step": (_c.c_int, [_vp, _c.c_int64]),
    "lks_mhd3_set_graph": (_c.c_int, [_vp, _c.c_int32]),
    "lks_mhd3_steps_done": (_c.c_int64, [_vp]),
    "lks_mhd3_run_to_steady": (_c.c_int, [_vp, _c.c_double, _c.c_int64, _c.c_int64, _i64p, _dp,
                                          _dp]),
    "lks_mhd3_moments": (_c.c_int, [_vp] + [_vp] * 10),
    "lks_mhd3_save_state": (_c.c_int, [_vp, _vp]),
    "lks_mhd3_load_state": (_c.c_int, [_vp, _vp, _c.c_int64]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2112_13930_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().lks_mhd_last_error().decode()


def check(code: int, what: str = "") -> int:
    if code != LKS_OK:
        raise LksError(code, f"{what}: {last_error()}" if what else last_error())
    return code


def make_params(nx: int, ny: int, *, bc="link", precision="fp32", tau_f=0.8, tau_m=0.8,
                ha=None, b0=None, c_lower=0.0, c_upper=None, u_lower=0.0, u_upper=0.0,
                fx=None, fy=0.0, u_max=None, rho0=1.0, collision="bgk", lambda_f=None,
                lambda_m=None, x_walls=False, c_x=0.0, q=0.5, mrt=None, solids=()) -> LksParams:
    """Build a parameter struct.  ``ha`` derives B0; ``u_max`` derives F_x;
    ``collision`` is "bgk", "trt" or "mrt" (magic parameters ``lambda_f``,
    ``lambda_m``; the library's defaults when None); ``mrt`` is a dict of
    MRT rates (``s_fe``, ``s_feps``, ``s_fq``, ``s_me``, ``s_md``) replacing
    the library's defaults; ``x_walls`` makes an
    enclosure whose x-walls have the conductance ratios ``c_x`` (both) or
    (x = 0 side, x = nx-1 side); ``q`` puts the link-based Hartmann walls at
    that distance from their wall rows (both, or (lower, upper)); ``solids``
    lists solid bodies (curved walls) as (kind, cx, cy, r, omega, u) with kind
    "disc", "bore", "below" or "above" (lks_solid)."""
    p = LksParams()
    lib().lks_mhd_default_params(ctypes.byref(p), int(nx), int(ny))
    p.bc = BCS[bc] if isinstance(bc, str) else int(bc)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.tau_f, p.tau_m = float(tau_f), float(tau_m)
    p.ha = math.nan if ha is None else float(ha)
    p.b0 = math.nan if b0 is None else float(b0)
    if ha is None and b0 is None:
        p.b0 = 0.0
    p.c_lower = float(c_lower)
    p.c_upper = float(c_lower if c_upper is None else c_upper)
    p.u_lower, p.u_upper = float(u_lower), float(u_upper)
    if fx is None and u_max is not None:
        p.fx = math.nan
        p.u_max = float(u_max)
    else:
        p.fx = 0.0 if fx is None else float(fx)
    p.fy = float(fy)
    p.rho0 = float(rho0)
    p.collision = COLLISIONS[collision] if isinstance(collision, str) else int(collision)
    if lambda_f is not None:
        p.lambda_f = float(lambda_f)
    if lambda_m is not None:
        p.lambda_m = float(lambda_m)
    ql, qh = q if isinstance(q, (tuple, list)) else (q, q)
    p.q_lower, p.q_upper = float(ql), float(qh)
    p.x_walls = int(bool(x_walls))
    lo, hi = c_x if isinstance(c_x, (tuple, list)) else (c_x, c_x)
    p.c_x_lower, p.c_x_upper = float(lo), float(hi)
    for name, v in (mrt or {}).items():
        if name not in ("s_fe", "s_feps", "s_fq", "s_me", "s_md"):
            raise ValueError(f"unknown MRT rate {name!r}")
        setattr(p, name, float(v))
    if len(solids) > MAX_SOLIDS:
        raise ValueError(f"at most {MAX_SOLIDS} solid bodies")
    p.nsolids = len(solids)
    for k, (kind, cx, cy, r, omega, u) in enumerate(solids):
        kind = SOLID_KINDS[kind] if isinstance(kind, str) else int(kind)
        p.solids[k] = LksSolid(kind, 0, float(cx), float(cy), float(r), float(omega), float(u))
    return p


def derive(p: LksParams) -> LksDerived:
    d = LksDerived()
    check(lib().lks_mhd_derive(ctypes.byref(p), ctypes.byref(d)), "lks_mhd_derive")
    return d
