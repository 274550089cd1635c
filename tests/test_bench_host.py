"""Host checks of bench.py's configuration table of profiled variants (no
GPU): every variant of the headline channel is a parameter set the library
accepts in each storage precision it supports (solid bodies: FP64 and FP32
only, refused otherwise), and the variants differ from the headline only in
the scheme they name."""
import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as b
    return b


@pytest.fixture(scope="module")
def L():
    import paper_2112_13930_amd._lib as lib
    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("liblks_mhd.so not built")
    return lib


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp16_f64", "fp64"])
def test_profile_variants_are_valid_channels(bench, L, precision):
    for name, over in bench.PROFILE_VARIANTS.items():
        kw = dict(bench.HEADLINE, precision=precision, **over)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        p = L.make_params(nx, ny, **kw)
        if "solids" in over and precision.startswith("fp16"):
            # solid bodies are built for FP64 and FP32 storage only
            assert L.lib().lks_mhd_validate(ctypes.byref(p)) != 0
            assert "solid" in L.last_error()
            continue
        assert L.lib().lks_mhd_validate(ctypes.byref(p)) == 0, (name, L.last_error())
        assert L.lib().lks_mhd_state_bytes(ctypes.byref(p)) > 0, name


def test_profile_variants_change_only_their_scheme(bench):
    assert bench.PROFILE_VARIANTS["headline"] == {}
    for name, over in bench.PROFILE_VARIANTS.items():
        assert set(over) <= {"bc", "collision", "x_walls", "c_x", "q", "solids"}, name
