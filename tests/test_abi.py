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
