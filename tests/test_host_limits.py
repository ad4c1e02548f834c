"""Host-side limits of the search, compiled from the HIP sources for the host
(no GPU): the global search counts its work in 64 bits (chunks of 256
queries times tiles of 1024 targets pass 2^31 at about 24M points per pair),
its launcher refuses batches it cannot take instead of returning silently,
and grids are limited to coordinates within +-1e18, where every float32
squared distance between two points of the grid is finite."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def hl(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("limits") / "liblimits.so")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2512_04996_amd", "csrc"),
           os.path.join(HERE, "host_limits_harness.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = C.CDLL(out)
    L.vicp_test_fallback_items.argtypes = [C.c_int64, C.c_int64]
    L.vicp_test_fallback_items.restype = C.c_int64
    L.vicp_test_launch_fallback_refuses.argtypes = [C.c_int, C.c_int]
    L.vicp_test_grid_box_fits.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float)]
    return L


def test_global_search_work_count_is_64_bit(hl):
    for F, n in ((0, 10), (1, 1), (256, 1024), (257, 1025), (200000, 226000), (24_000_000, 24_000_000),
                 (2**31 - 1, 2**31 - 1)):
        want = 0 if F == 0 else -(-F // 256) * -(-n // 1024)
        assert hl.vicp_test_fallback_items(F, n) == want
    assert hl.vicp_test_fallback_items(24_000_000, 24_000_000) > 2**31


def test_global_search_launcher_refuses_what_it_cannot_take(hl):
    for npairs, grid in ((0, 64), (4097, 64), (100000, 128), (-3, 64), (1, 0), (8, -1)):
        assert hl.vicp_test_launch_fallback_refuses(npairs, grid) == 1, (npairs, grid)


def test_coordinate_limit(hl):
    def fits(lo, hi):
        lo = np.asarray(lo, np.float32)
        hi = np.asarray(hi, np.float32)
        return hl.vicp_test_grid_box_fits(lo.ctypes.data_as(C.POINTER(C.c_float)),
                                          hi.ctypes.data_as(C.POINTER(C.c_float)))
    assert fits([-1e18, -5, 0], [1e18, 5, 1])
    assert not fits([-2e18, 0, 0], [0, 1, 1])
    assert not fits([0, 0, 0], [1, 1e19, 1])
    assert not fits([0, 0, -np.inf], [1, 1, 1])
    assert not fits([0, np.nan, 0], [1, 1, 1])
    # at the limit every float32 squared distance inside the box is finite
    a = np.float32(1e18)
    d = np.float32(a - (-a))
    assert np.isfinite(np.float32(d * d) * np.float32(3))
