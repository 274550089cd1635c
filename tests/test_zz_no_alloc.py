"""lks_mhd_advance_noalloc: the entry point that allocates nothing (its
working memory is a static device array of the library).  Called through the
C ABI, it must reproduce bit for bit the create + load_state + step +
save_state sequence of the existing entry points, on two calls in a row (the
second with a smaller channel, in the array the first one left behind), in
every storage precision; a channel too large for the array is refused."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_2112_13930_amd import _lib
    assert torch.cuda.is_available()
    _lib.lib()
    return _lib


def reference(L, params, pops, step0, nsteps):
    from paper_2112_13930_amd.channel import Channel
    ch = Channel(params=params, stream=torch.cuda.current_stream())
    ch.load_state(pops, steps=step0)
    ch.step(nsteps)
    out = ch.save_state()
    torch.cuda.synchronize()
    ch.close()
    return out


def noalloc(L, params, pops, step0, nsteps):
    t = pops.to(device="cuda", dtype=torch.float64).contiguous().clone()
    stream = torch.cuda.current_stream()
    rc = L.lib().lks_mhd_advance_noalloc(ctypes.byref(params), ctypes.c_void_p(t.data_ptr()),
                                         int(step0), int(nsteps),
                                         ctypes.c_void_p(stream.cuda_stream))
    assert rc == L.LKS_OK, L.last_error()
    torch.cuda.synchronize()
    return t


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "fp16_f64"])
def test_noalloc_equals_existing_entry_points(L, precision):
    from paper_2112_13930_amd.workloads import random_populations
    cases = [
        # (nx, ny, bc, extra keywords, step0, nsteps): the second is smaller
        (96, 40, "moment", dict(c_lower=0.3, c_upper=float("inf"), u_upper=0.04), 0, 37),
        (34, 21, "link", dict(c_lower=0.0, c_upper=2.0, u_lower=-0.02), 995, 12),
    ]
    for nx, ny, bc, kw, step0, nsteps in cases:
        params = L.make_params(nx, ny, bc=bc, precision=precision, tau_f=0.75, tau_m=0.85,
                               b0=0.02, fx=1e-5, **kw)
        pops = torch.from_numpy(random_populations(nx, ny, seed=nx, b0=0.02)).cuda()
        want = reference(L, params, pops, step0, nsteps)
        got = noalloc(L, params, pops, step0, nsteps)
        assert torch.equal(got, want), (precision, nx, ny, (got - want).abs().max().item())


def test_noalloc_refuses_a_channel_beyond_its_array(L):
    params = L.make_params(1024, 1024, bc="link", precision="fp64", tau_f=0.8, tau_m=0.8, b0=0.01)
    t = torch.zeros((19, 1024, 1024), dtype=torch.float64, device="cuda")
    rc = L.lib().lks_mhd_advance_noalloc(ctypes.byref(params), ctypes.c_void_p(t.data_ptr()), 0, 1,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.LKS_ENOMEM and "scratch" in L.last_error()
