"""The C-ABI library loads and exports every entry point include/faco.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2203_02228_amd import faco as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "faco.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(faco_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("faco_build_instance", "faco_run_iterations", "faco_get_best_tour"):
        assert must in names
    assert sorted(F.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("HIP library not built")
    L = ctypes.CDLL(F.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_footprint_is_pure_arithmetic():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("HIP library not built")
    p = F.make_params(n_ants=32, cl_size=16, bl_size=64)
    b = F.faco_footprint_bytes(200000, p)
    # coords + cl/eta/tau + backup + source/gbest + ant arrays
    assert b >= 8 * 200000 + 12 * 200000 * 16 + 4 * 200000 * 64 + 12 * 200000 + 12 * 200000 * 32
    assert F.faco_footprint_bytes(3, p) == 0


def test_tour_segment_setting_checked_on_the_host():
    """faco_set_tour_segments validates its arguments and, with segment lists
    asked for, the footprint of a build grows by the second array buffer and
    the per-city record labels (24 n bytes per ant); flat arrays are the
    default (host arithmetic only)."""
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("HIP library not built")
    for args in [(3, 0, 0), (-1, 0, 0), (2, 25, 0), (2, -1, 0), (2, 0, 7), (2, 0, 2049)]:
        with pytest.raises(F.FacoError) as e:
            F.faco_set_tour_segments(*args)
        assert e.value.code == F.FACO_EINVAL
    p = F.make_params(n_ants=16, cl_size=16, bl_size=64)
    n = 100000
    flat = F.faco_footprint_bytes(n, p)
    F.faco_set_tour_segments(2, 0, 0)
    try:
        seg = F.faco_footprint_bytes(n, p)
    finally:
        F.faco_set_tour_segments(0, 0, 0)
    assert seg - flat >= 24 * n * 16
    assert seg - flat < 24 * n * 16 + 16 * 4096
    assert F.faco_footprint_bytes(n, p) == flat


def test_set_stream_rejects_null_handle():
    """faco_set_stream checks its handle on the host (no GPU needed)."""
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("HIP library not built")
    assert F.lib().faco_set_stream(None, None) == F.FACO_EINVAL
