"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/lks_mhd.h declares, and its host-only paths (validation,
derivation, sizing, argument checks) behave as documented.  No compute call
is made here."""
import ctypes
import math
import os
import re

import pytest

import oracle
from oracle import derive as od

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lks_mhd.h")


@pytest.fixture(scope="module")
def L():
    from paper_2112_13930_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lks_mhd_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 30
    lib = L.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)


def test_abi_version(L):
    assert L.lib().lks_mhd_abi_version() == 9


def _v(L, **kw):
    nx = kw.pop("nx", 16)
    ny = kw.pop("ny", 16)
    p = L.make_params(nx, ny, **kw)
    return L.lib().lks_mhd_validate(ctypes.byref(p)), p


@pytest.mark.parametrize("kw", [
    dict(tau_f=0.5), dict(tau_m=0.49), dict(tau_f=float("nan")),
    dict(c_lower=-0.1), dict(c_upper=float("nan")),
    dict(ny=1), dict(ny=2, bc="moment"), dict(nx=0),
    dict(nx=20000, ny=20000),
    dict(ha=10.0, b0=0.5),                       # inconsistent
    dict(u_max=0.05, c_lower=0.1, c_upper=0.2),  # fx from u_max needs equal walls
    dict(u_upper=float("inf")), dict(rho0=0.0), dict(precision=7), dict(precision=4),
    dict(bc=5), dict(collision=3), dict(collision="trt", lambda_f=0.0),
    dict(collision="mrt", mrt=dict(s_fe=2.0)), dict(collision="mrt", mrt=dict(s_feps=0.0)),
    dict(collision="mrt", mrt=dict(s_fe=float("nan"))), dict(collision="mrt", mrt=dict(s_fq=-0.5)),
    dict(collision="mrt", mrt=dict(s_md=2.5)), dict(collision="mrt", lambda_m=0.0),

    dict(collision="trt", lambda_m=float("inf")), dict(collision="trt", lambda_m=-1.0),
    dict(x_walls=True, bc="moment"), dict(x_walls=True, nx=1), dict(x_walls=True, c_x=-1.0),
    dict(x_walls=True, c_x=(0.0, float("nan"))),
    dict(q=0.0), dict(q=1.5), dict(q=(0.5, float("nan"))), dict(q=0.3, bc="moment"),
    dict(q=0.3, x_walls=True), dict(q=0.3, ny=2),
    dict(q=0.1, c_lower=1e-3, tau_m=0.55),         # c a + q + tau_m - 1 < 1/4
])
def test_validate_rejects(L, kw):
    rc, p = _v(L, **kw)
    assert rc == L.LKS_EINVAL
    assert L.last_error()
    assert L.lib().lks_mhd_state_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("kw", [
    dict(), dict(ny=2), dict(ny=3, bc="moment"), dict(c_lower=math.inf, c_upper=0.0),
    dict(ha=10.0, u_max=0.05, c_lower=0.1), dict(ha=0.0, u_max=0.05),
    dict(ha=5.0, c_lower=math.inf, u_max=0.01, bc="moment"),
    dict(precision="fp64"), dict(precision="fp16"), dict(precision="fp16_f64"),
    dict(collision="trt"), dict(collision="trt", lambda_f=0.25, lambda_m=1.0 / 12.0),
    dict(collision="bgk", lambda_f=float("nan")),  # magic parameters unused under BGK
    dict(x_walls=True), dict(x_walls=True, nx=2, c_x=(0.0, math.inf), collision="trt"),
    dict(q=0.25), dict(q=(1.0, 0.3), c_lower=math.inf), dict(q=0.1, c_lower=0.0, tau_m=0.55),
    dict(collision="mrt"), dict(collision="mrt", bc="moment", ny=3),
    dict(collision="mrt", x_walls=True), dict(collision="mrt", q=0.3),
    dict(collision="mrt", mrt=dict(s_fe=1.9, s_feps=0.3, s_fq=1.99, s_me=0.01, s_md=1.5)),
])
def test_validate_accepts(L, kw):
    rc, p = _v(L, **kw)
    assert rc == L.LKS_OK, L.last_error()
    assert L.lib().lks_mhd_state_bytes(ctypes.byref(p)) > 0


@pytest.mark.parametrize("bc", [oracle.LINK, oracle.MOMENT])
@pytest.mark.parametrize("ha,c", [(10.0, 0.1), (20.0, 0.0), (5.0, math.inf), (0.0, 1.0)])
def test_derivation_agrees_with_oracle(L, bc, ha, c):
    """The library's host derivation is written separately from the oracle's;
    both follow Secs. IV, V, VI and VIII."""
    ny = 64
    q = od.hartmann_params(8, ny, bc, 0.8, 0.9, ha, c, 0.05)
    p = L.make_params(8, ny, bc="link" if bc == oracle.LINK else "moment", tau_f=0.8,
                      tau_m=0.9, ha=ha, u_max=0.05, c_lower=c, c_upper=c)
    d = L.derive(p)
    assert d.a == q.a
    assert math.isclose(d.b0, q.b0, rel_tol=1e-14, abs_tol=1e-300)
    assert math.isclose(d.fx, q.fx, rel_tol=1e-13)
    assert math.isclose(d.nu, od.nu_of(0.8), rel_tol=1e-15)
    assert math.isclose(d.eta, od.eta_of(0.9), rel_tol=1e-15)
    theta = math.inf if math.isinf(c) else c * q.a / (0.9 - 0.5)
    assert d.theta_lower == pytest.approx(theta, rel=1e-15)
    if bc == oracle.LINK:   # walls at cut distances change the half-width
        pq = L.make_params(8, ny, bc="link", tau_f=0.8, tau_m=0.9, ha=ha, u_max=0.05,
                           c_lower=c, c_upper=c, q=(0.25, 1.0))
        oq = oracle.Params(nx=8, ny=ny, bc=oracle.LINK, q_lo=0.25, q_hi=1.0)
        assert L.derive(pq).a == oq.half_width() == (ny - 1 + 1.25) / 2


@pytest.mark.parametrize("tau_f,tau_m,lf,lm", [(0.8, 0.9, 3 / 16, 0.25), (0.55, 1.7, 0.01, 2.0)])
def test_trt_times_agree_with_oracle(L, tau_f, tau_m, lf, lm):
    p = L.make_params(8, 8, tau_f=tau_f, tau_m=tau_m, collision="trt", lambda_f=lf, lambda_m=lm)
    d = L.derive(p)
    assert (d.tau_f_odd, d.tau_m_even) == od.trt_times(tau_f, tau_m, lf, lm)
    assert math.isclose((tau_f - 0.5) * (d.tau_f_odd - 0.5), lf, rel_tol=1e-14)
    assert math.isclose((d.tau_m_even - 0.5) * (tau_m - 0.5), lm, rel_tol=1e-14)
    q = L.make_params(8, 8, tau_f=tau_f, tau_m=tau_m)
    assert q.collision == L.LKS_BGK and (q.lambda_f, q.lambda_m) == (3 / 16, 0.25)
    e = L.derive(q)
    assert (e.tau_f_odd, e.tau_m_even) == (tau_f, tau_m)


def test_bytes_per_node(L):
    f = L.lib().lks_mhd_bytes_per_node
    assert (f(0), f(1), f(2), f(3), f(4), f(9)) == (304, 152, 76, 76, 0, 0)


def test_state_bytes_cover_two_buffers(L):
    for prec, b in (("fp64", 8), ("fp32", 4), ("fp16", 2), ("fp16_f64", 2)):
        p = L.make_params(4096, 4096, precision=prec)
        assert L.lib().lks_mhd_state_bytes(ctypes.byref(p)) >= 2 * 19 * 4096 * 4096 * b


def test_create_argument_checks_need_no_device(L):
    p = L.make_params(16, 16)
    h = ctypes.c_void_p()
    lib = L.lib()
    assert lib.lks_mhd_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(h)) == L.LKS_EINVAL
    assert lib.lks_mhd_create(ctypes.byref(p), ctypes.c_void_p(256 + 8), 1 << 20, None,
                              ctypes.byref(h)) == L.LKS_EINVAL
    assert lib.lks_mhd_create(ctypes.byref(p), ctypes.c_void_p(4096), 16, None,
                              ctypes.byref(h)) == L.LKS_ENOMEM
    assert not h.value
    assert lib.lks_mhd_destroy(None) == L.LKS_OK


def test_batch_sizing(L):
    lib = L.lib()
    assert lib.lks_mhd_batch_overhead_bytes(256, 1 << 24) > 0
    assert lib.lks_mhd_batch_overhead_bytes(0, 1 << 24) == 0
    p = L.make_params(100, 50)
    assert lib.lks_mhd_batch_channel_bytes(ctypes.byref(p), 1) >= 2 * 19 * 100 * 50 * 4
    h = ctypes.c_void_p()
    assert lib.lks_mhd_batch_create(1, 0, 100, ctypes.c_void_p(4096), 1 << 20, None,
                                    ctypes.byref(h)) == L.LKS_EINVAL
    assert lib.lks_mhd_batch_create(1, 4, 1000, ctypes.c_void_p(4096), 64, None,
                                    ctypes.byref(h)) == L.LKS_ENOMEM


@pytest.mark.parametrize("tau_f,tau_m,lf,lm", [(0.8, 0.9, 3 / 16, 0.25), (0.55, 1.7, 0.01, 2.0)])
def test_mrt_rates_agree_with_oracle(L, tau_f, tau_m, lf, lm):
    """Unset (NaN) MRT rates resolve to TRT's from the magic parameters, as
    the oracle's mrt_rates gives them; set ones are used as given; BGK and
    TRT report the rates they amount to."""
    p = L.make_params(8, 8, tau_f=tau_f, tau_m=tau_m, collision="mrt", lambda_f=lf, lambda_m=lm)
    d = L.derive(p)
    assert (d.s_fe, d.s_feps, d.s_fq, d.s_me, d.s_md) == od.mrt_rates(tau_f, tau_m, lf, lm)
    r = dict(s_fe=1.1, s_feps=1.2, s_fq=1.3, s_me=1.4, s_md=1.5)
    e = L.derive(L.make_params(8, 8, tau_f=tau_f, tau_m=tau_m, collision="mrt", mrt=r))
    assert (e.s_fe, e.s_feps, e.s_fq, e.s_me, e.s_md) == tuple(r.values())
    t = L.derive(L.make_params(8, 8, tau_f=tau_f, tau_m=tau_m, collision="trt", lambda_f=lf,
                               lambda_m=lm))
    assert (t.s_fe, t.s_feps, t.s_fq) == (1 / tau_f, 1 / tau_f, 1 / t.tau_f_odd)
    assert (t.s_me, t.s_md) == (1 / t.tau_m_even, 1 / t.tau_m_even)
    with pytest.raises(ValueError):
        L.make_params(8, 8, collision="mrt", mrt=dict(s_nu=1.0))


def test_3d_sizing_and_validation(L):
    lib = L.lib()
    p = L.LksParams3()
    p.base = L.make_params(64, 32, precision="fp32")
    p.nz = 16
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) >= 2 * 37 * 64 * 32 * 16 * 4
    assert (lib.lks_mhd3_bytes_per_node(0), lib.lks_mhd3_bytes_per_node(1),
            lib.lks_mhd3_bytes_per_node(2)) == (592, 296, 0)
    p.nz = 0
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0 and "nz" in L.last_error()
    p.nz = 4
    p.base = L.make_params(64, 32, precision="fp16")
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0
    p.base = L.make_params(2048, 2048, precision="fp32")
    p.nz = 1024
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0
    p.base = L.make_params(64, 32, precision="fp32", collision="trt")
    p.nz = 4
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) > 0
    p.base = L.make_params(64, 32, precision="fp32", collision="trt", lambda_f=-1.0)
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0 and "lambda" in L.last_error()
    p.base = L.make_params(64, 32, precision="fp32", collision="mrt")
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) > 0
    p.base = L.make_params(64, 32, precision="fp32", collision="mrt", mrt=dict(s_md=2.0))
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0
    # ducts: link walls only, nz >= 2, conductances in [0, inf]
    p.base = L.make_params(64, 32, precision="fp32")
    p.nz, p.side_walls, p.c_side_lower, p.c_side_upper = 8, 1, 0.5, math.inf
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) > 0
    for bad in (dict(nz=1), dict(side_walls=2), dict(c_side_lower=-1.0),
                dict(c_side_upper=float("nan"))):
        q = L.LksParams3()
        ctypes.pointer(q)[0] = p
        for k, v in bad.items():
            setattr(q, k, v)
        assert lib.lks_mhd3_state_bytes(ctypes.byref(q)) == 0, bad
    p.base = L.make_params(64, 32, precision="fp32", bc="moment")
    assert lib.lks_mhd3_state_bytes(ctypes.byref(p)) == 0 and "link" in L.last_error()
    p.side_walls = 0
    h = ctypes.c_void_p()
    p.base = L.make_params(8, 8, precision="fp64")
    p.nz = 2
    assert lib.lks_mhd3_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(h)) == L.LKS_EINVAL
