"""The binary16 storage rounding on the GPU, bit for bit against its
definition (lks_round_binary16; the kernels round every binary16 value this
way).

Definition (written out here with NumPy, independently of the library): with
r13 the top 13 bits of the random word, a value of magnitude >= 2^-14 (and
zeros, infinities, NaN) has r13 added to its binary32 bits, 13 bits below
binary16's last place, and is truncated there (a carry past 65504 gives
infinity); below 2^-14 the result is sign(v) trunc(|v| 2^24 + r13 2^-13)
2^-24.  Inputs span the binary16 range, its subnormals, binary32 subnormals,
the overflow boundary and non-finite values, with random words, and a sweep
of the 2^13 words at fixed values."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    from paper_2112_13930_amd import _lib
    assert torch.cuda.is_available()
    return _lib.lib()


def _definition(v, r):
    v = np.asarray(v, np.float32)
    b = v.view(np.uint32).astype(np.uint64)
    r13 = (np.asarray(r, np.uint32) >> 19).astype(np.uint64)
    m = b & 0x7FFFFFFF
    out = np.empty(v.size, np.float16)
    upper = (m >= 0x38800000) | (m == 0)
    t = ((b + r13) & 0xFFFFFFFF) & ~np.uint64(0x1FFF)
    with np.errstate(over="ignore", invalid="ignore"):
        out[upper] = t[upper].astype(np.uint32).view(np.float32).astype(np.float16)
    low = ~upper
    # |v| 2^37 is exact in float64 (|v| < 2^-14 has at most 24 significant
    # bits); trunc(|v| 2^24 + r13 2^-13) = (trunc(|v| 2^37) + r13) >> 13
    u = np.floor(np.abs(v[low].astype(np.float64)) * 2.0 ** 37).astype(np.uint64)
    q = (u + r13[low]) >> np.uint64(13)
    mag = q.astype(np.float64) * 2.0 ** -24
    out[low] = np.where(np.signbit(v[low]), -mag, mag).astype(np.float16)
    return out


def _inputs(seed=11):
    rng = np.random.default_rng(seed)
    vals, words = [], []
    k = rng.integers(0, 8192, 50000)
    vals.append((1.0 + k * 2.0 ** -23).astype(np.float32))
    e = rng.uniform(-40, 17, 200000)
    vals.append((2.0 ** e * np.where(rng.uniform(size=e.size) < 0.5, -1, 1)).astype(np.float32))
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 65504, 65519, 65520, 65535, 65536, 1e6,
                        -65520, 1e-40, -1e-40, 2 ** -24, 2 ** -25, 3 * 2 ** -26, 2 ** -14,
                        2 ** -14 - 2 ** -24, 6.0e-5, 2 ** -149], dtype=np.float32)
    vals.append(np.repeat(special, 64))
    n = sum(x.size for x in vals)
    words.append(rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32))
    # every 13-bit word at a few fixed values (both ranges)
    fixed = np.array([1.0 + 1234 * 2.0 ** -23, -3.3e-6, 7.1e-8, 2.0 ** -14 - 2.0 ** -30, 1000.37],
                     np.float32)
    sweep = (np.arange(8192, dtype=np.uint32) << 19) | 0x5A5A5
    vals.append(np.repeat(fixed, 8192))
    words.append(np.tile(sweep, fixed.size))
    return np.concatenate(vals), np.concatenate(words)


def test_binary16_rounding_matches_definition(lib):
    v, r = _inputs()
    dv = torch.from_numpy(v).cuda()
    dr = torch.from_numpy(r.view(np.int32)).cuda()
    out = torch.empty(v.size, dtype=torch.int16, device="cuda")
    stream = torch.cuda.current_stream()
    print(f"lks_round_binary16: {v.size} values", flush=True)
    rc = lib.lks_round_binary16(ctypes.c_void_p(dv.data_ptr()), ctypes.c_void_p(dr.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), v.size,
                                ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0
    got = out.cpu().numpy().view(np.float16)
    want = _definition(v, r)
    both_nan = np.isnan(got.astype(np.float32)) & np.isnan(want.astype(np.float32))
    bad = (got.view(np.uint16) != want.view(np.uint16)) & ~both_nan
    idx = np.nonzero(bad)[0][:5]
    assert not bad.any(), [(float(v[i]), hex(int(r[i])), float(got[i]), float(want[i])) for i in idx]
    # the sweep rounds up in exactly the share the fraction below the last
    # place gives (13 bits): 1234 of 8192 at 1 + 1234 2^-23
    ups = int((got[-5 * 8192:-4 * 8192].astype(np.float64) > 1.0).sum())
    assert ups == 1234


def test_binary16_rounding_arguments(lib):
    assert lib.lks_round_binary16(None, None, None, 0, None) == 0
    assert lib.lks_round_binary16(None, None, None, 5, None) != 0
    assert lib.lks_round_binary16(None, None, None, -1, None) != 0
