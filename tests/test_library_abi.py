"""The C-ABI library loads on the CPU and exports every symbol that
include/ikr.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ikr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ikr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2505_02319_amd import LIB_PATH, SIGNATURES, lib
    if not os.path.exists(LIB_PATH):
        pytest.fail("libikr.so is not built (run __graft_entry__.build())")
    L = lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
        assert name in SIGNATURES, name
    assert set(SIGNATURES) == set(names)


def test_host_only_entry_points():
    from paper_2505_02319_amd import default_opts, lib
    L = lib()
    for n in (20, 48, 60, 96, 108):
        assert L.ikr_supported_fft_size(n) == 1
    for n in (7, 50, 1000):
        assert L.ikr_supported_fft_size(n) == 0
    o = default_opts()
    assert o.strategy == 1 and o.restart_m == 20 and o.tol == 1e-8 and o.s0 == 1.0
    assert o.cg_min_iter == 1 and o.tol_is_relative == 1
    assert L.ikr_last_error() is not None
